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
