"""The C ABI library loads on the CPU and exports every entry point that
include/gfc.h declares (no compute call is made: there is no GPU here)."""

import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gfc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(gfc_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gfc_render_stamps", "gfc_render_stamps_backward", "gfc_psf_create", "gfc_mix_create",
                 "gfc_server_submit", "gfc_sched_step"):
        assert must in names
    assert len(names) >= 35


def test_library_exports_every_declared_symbol():
    import paper_2012_15797_amd as gfc

    lib = gfc.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_prototypes_cover_the_header():
    from paper_2012_15797_amd._lib import PROTOTYPES

    assert sorted(PROTOTYPES) == declared_functions()


def test_host_only_calls_work_without_a_gpu():
    import paper_2012_15797_amd as gfc

    lib = gfc.lib()
    assert lib.gfc_stamp_size_supported(64) == 1 and lib.gfc_stamp_size_supported(48) == 0
    assert lib.gfc_status_str(-6) == b"rejected"
    assert lib.gfc_backward_workspace_bytes(10) >= 10 * 16 * 4


def test_rate_probe_library_exports_its_header():
    """libgfc_microbench.so (the roofline denominators' probes) exports every
    function include/gfc_microbench.h declares."""
    import ctypes

    text = open(os.path.join(ROOT, "include", "gfc_microbench.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"^int\s+(gfc_mb_\w+)\s*\(", text, flags=re.M)))
    assert names == ["gfc_mb_exp", "gfc_mb_exp_fma", "gfc_mb_fma", "gfc_mb_hbm_copy", "gfc_mb_hbm_write"]
    import paper_2012_15797_amd  # noqa: F401  (torch's HIP runtime first)

    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2012_15797_amd", "libgfc_microbench.so"))
    assert all(hasattr(lib, n) for n in names)


def test_gfc_log_writes_json_lines():
    """GFC_LOG=1: a failing call writes one JSON line (event "error", its
    status and message) to stderr; without it nothing is written."""
    import json
    import subprocess
    import sys

    lib = os.path.join(ROOT, "paper_2012_15797_amd", "libgfc.so")
    code = ("import ctypes, sys\n"
            "lib = ctypes.CDLL(sys.argv[1])\n"
            "lib.gfc_server_submit.restype = ctypes.c_int\n"
            "print(lib.gfc_server_submit(None, None, None))\n")
    env = dict(os.environ, GFC_LOG="1")
    r = subprocess.run([sys.executable, "-c", code, lib], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    lines = [json.loads(ln) for ln in r.stderr.splitlines() if ln.startswith("{")]
    errs = [ln for ln in lines if ln["event"] == "error"]
    assert len(errs) == 1 and errs[0]["status"] == int(r.stdout.strip()) and "null" in errs[0]["message"]
    assert isinstance(errs[0]["t"], float)
    env.pop("GFC_LOG")
    r = subprocess.run([sys.executable, "-c", code, lib], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and not [ln for ln in r.stderr.splitlines() if ln.startswith("{")], r.stderr
