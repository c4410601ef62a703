"""The continuous-batching server on the GPU: every request's stamps equal
those of a direct render of that request alone (bit for bit: stamps are
independent and rendered by the same kernels), under mixed traffic of
stamp sizes, PSFs and mixtures, memory back-pressure and the plain mode."""

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2012_15797_amd as gfc
    return gfc.Context.default(0)


def _objects(ctx, trace, n_psf):
    import paper_2012_15797_amd as gfc

    psfs = [gfc.Psf(ctx, p) for p in trace["psfs"][:n_psf]]
    mix = gfc.Mixture.from_workload(ctx, trace["mix"].as_f32())
    return psfs, mix


def _direct(ctx, psf, mix, r):
    import torch
    import paper_2012_15797_amd as gfc

    g = r["gal"]
    out = gfc.gfc_render_stamps(ctx, psf, mix, g.x, g.y, g.flux, g.r_e, g.e1, g.e2, r["W"], mix_id=g.mix_id)
    torch.cuda.synchronize()
    return out


def test_mixed_traffic_matches_direct_render(ctx):
    import torch
    from paper_2012_15797_amd.serving import Server

    tr = wl.config4_trace(duration_s=0.03, rate_hz=2000.0, n_psf=3)
    reqs = [dict(r, psf=r["psf"] % 3) for r in tr["requests"]]
    reqs = [r for r in reqs if r["W"] < 256 or len(r["gal"]) <= 256][:40]
    psfs, mix = _objects(ctx, tr, 3)
    srv = Server(ctx, mem_budget_bytes=8 << 30, n_streams=2, max_batch_stamps=1 << 16)
    tickets = [srv.submit(psfs[r["psf"]], mix, r["W"], r["gal"].x, r["gal"].y, r["gal"].flux, r["gal"].r_e,
                          r["gal"].e1, r["gal"].e2, mix_id=r["gal"].mix_id) for r in reqs]
    for t, r in zip(tickets, reqs):
        srv.wait(t)
        got = srv.result(t)
        torch.cuda.synchronize()
        ref = _direct(ctx, psfs[r["psf"]], mix, r)
        assert torch.equal(got, ref)
        srv.release(t)
    st = srv.stats()
    assert st["done"] == len(reqs) and st["launches"] <= len(reqs)
    srv.close()


def test_requests_with_different_psfs_share_a_launch(ctx):
    """Stamps of six PSFs fuse into one launch per stamp size (the batch key
    is the mixture, the size and the flags; each galaxy reads its request's
    PSF from the server's resident tables).  At 16 x 16 four stamps share a
    wavefront, so neighbouring lanes read different PSFs.  Each request's
    stamps equal, bit for bit, those of the same request launched alone
    (the plain mode) and of a direct render."""
    import torch
    from paper_2012_15797_amd.serving import Server

    tr = wl.config4_trace(duration_s=0.01, rate_hz=2000.0, n_psf=6)
    psfs, mix = _objects(ctx, tr, 6)
    rng = np.random.Generator(np.random.PCG64(4711))
    reqs = []
    for W in (16, 64, 256):
        for i in range(12 if W < 256 else 6):
            n = int(rng.integers(1, 40))
            reqs.append((i % 6, W, wl.draw_galaxies(rng, n, W, (np.arange(n) % 2).astype(np.int32))))

    def submit_all(srv):
        return [srv.submit(psfs[p], mix, W, g.x, g.y, g.flux, g.r_e, g.e1, g.e2, mix_id=g.mix_id)
                for p, W, g in reqs]

    srv = Server(ctx, mem_budget_bytes=8 << 30, n_streams=1, max_batch_stamps=1 << 16)
    # first pass: the server enters each PSF at each size (its transform is made
    # then, on this thread)
    for t in submit_all(srv):
        srv.wait(t)
        srv.release(t)
    l1 = srv.stats()["launches"]
    # a long request holds the only stream while the others queue behind it
    blk = wl.draw_galaxies(rng, 20000, 256, 0)
    tb = srv.submit(psfs[0], mix, 256, blk.x, blk.y, blk.flux, blk.r_e, blk.e1, blk.e2)
    tickets = submit_all(srv)
    srv.wait(tb)
    srv.release(tb)
    fused = []
    for t in tickets:
        srv.wait(t)
        fused.append(srv.result(t).clone())
        srv.release(t)
    st = srv.stats()
    srv.close()
    assert st["done"] == 2 * len(reqs) + 1
    assert st["launches"] - l1 <= 1 + 3 + 1, (st, l1)   # a launch per PSF would take 1 + 6 + 6 + 6
    plain = Server(ctx, mem_budget_bytes=8 << 30, n_streams=1, max_batch_stamps=0)
    for t, (p, W, g), got in zip(submit_all(plain), reqs, fused):
        plain.wait(t)
        alone = plain.result(t)
        torch.cuda.synchronize()
        assert torch.equal(got, alone)
        assert torch.equal(got, _direct(ctx, psfs[p], mix, dict(gal=g, W=W)))
        plain.release(t)
    assert plain.stats()["launches"] == len(reqs)
    plain.close()


def test_backpressure_small_budget(ctx):
    import torch
    from paper_2012_15797_amd.serving import Server

    tr = wl.config4_trace(duration_s=0.02, rate_hz=2000.0, restricted=True)
    reqs = tr["requests"][:12]
    psfs, mix = _objects(ctx, tr, 1)
    biggest = (max(len(r["gal"]) for r in reqs) * (64 * 64 * 4 + 32) + 255) // 256 * 256
    srv = Server(ctx, mem_budget_bytes=biggest + 1, n_streams=2, max_batch_stamps=1 << 16)
    tickets = [srv.submit(psfs[0], mix, 64, r["gal"].x, r["gal"].y, r["gal"].flux, r["gal"].r_e,
                          r["gal"].e1, r["gal"].e2) for r in reqs]
    for t, r in zip(tickets, reqs):
        srv.wait(t, timeout_ms=60_000)
        assert torch.equal(srv.result(t), _direct(ctx, psfs[0], mix, r))
        srv.release(t)
    srv.close()


def test_rejects_request_larger_than_budget(ctx):
    import paper_2012_15797_amd as gfc
    from paper_2012_15797_amd.serving import Server

    tr = wl.config4_trace(duration_s=0.01, rate_hz=2000.0, restricted=True)
    psfs, mix = _objects(ctx, tr, 1)
    srv = Server(ctx, mem_budget_bytes=1 << 20, n_streams=1)
    g = wl.draw_galaxies(np.random.Generator(np.random.PCG64(1)), 100, 64, 0)
    with pytest.raises(gfc.GfcError) as e:
        srv.submit(psfs[0], mix, 64, g.x, g.y, g.flux, g.r_e, g.e1, g.e2)
    assert e.value.status == -6
    srv.close()


def test_plain_mode_and_trace_replay(ctx):
    from paper_2012_15797_amd.serving import Server, replay_trace

    import torch

    tr = wl.config4_trace(duration_s=0.25, rate_hz=2000.0, restricted=True)
    psfs, mix = _objects(ctx, tr, 1)
    picked = [0, len(tr["requests"]) // 2, len(tr["requests"]) - 1]
    for max_batch, n_streams in ((0, 1), (1 << 16, 2)):
        srv = Server(ctx, mem_budget_bytes=8 << 30, n_streams=n_streams, max_batch_stamps=max_batch)
        keep = {i: torch.full((len(tr["requests"][i]["gal"]), 64, 64), float("nan"), device="cuda") for i in picked}
        res = replay_trace(srv, tr["requests"], psfs, mix, keep=keep)
        assert res["requests"] == len(tr["requests"]) and res["p99_ms"] > 0
        if max_batch == 0:
            assert res["launches"] == res["requests"]
        for i in picked:  # the kept stamps are the requests' own
            assert torch.equal(keep[i], _direct(ctx, psfs[0], mix, tr["requests"][i]))
        srv.close()


def test_native_replay_errors(ctx):
    """gfc_server_replay validates the arrival times before submitting
    anything, and stops at a rejected request after draining the ones it
    submitted (the server stays usable)."""
    import ctypes

    import paper_2012_15797_amd as gfc
    from paper_2012_15797_amd._lib import call, gfc_request
    from paper_2012_15797_amd.serving import Server

    tr = wl.config4_trace(duration_s=0.05, rate_hz=2000.0, restricted=True)
    psfs, mix = _objects(ctx, tr, 1)
    g = wl.draw_galaxies(np.random.Generator(np.random.PCG64(3)), 64, 64, 0)
    srv = Server(ctx, mem_budget_bytes=8 << 20, n_streams=1)
    small = srv.prepare(psfs[0], mix, 64, g.x[:8], g.y[:8], g.flux[:8], g.r_e[:8], g.e1[:8], g.e2[:8])
    big = srv.prepare(psfs[0], mix, 64, g.x, g.y, g.flux, g.r_e, g.e1, g.e2)  # 64 stamps: 1 MB, fits
    huge_g = wl.draw_galaxies(np.random.Generator(np.random.PCG64(4)), 1024, 64, 0)  # 16 MB > budget
    huge = srv.prepare(psfs[0], mix, 64, huge_g.x, huge_g.y, huge_g.flux, huge_g.r_e, huge_g.e1, huge_g.e2)
    D_p = ctypes.POINTER(ctypes.c_double)

    def replay(items, times):
        reqs = (gfc_request * len(items))(*[p[0] for p in items])
        t = np.ascontiguousarray(times, np.float64)
        lag = np.zeros(len(items))
        call("gfc_server_replay", srv.handle, reqs, t.ctypes.data_as(D_p), len(items), None, lag.ctypes.data_as(D_p), None)
        return lag

    with pytest.raises(gfc.GfcError) as e:
        replay([small, small], [0.002, 0.001])
    assert e.value.status == -1
    with pytest.raises(gfc.GfcError) as e:
        replay([small, big, huge, small], [0.0, 0.0, 0.001, 0.001])
    assert e.value.status == -6
    lag = replay([small, big, small], [0.0, 0.0005, 0.001])  # still usable; every request released
    assert (lag >= 0).all() and lag.max() < 0.5
    assert srv.stats()["done"] == 5  # two before the rejection, three after
    srv.close()
    for p in psfs:
        p.close()
    mix.close()


def test_release_right_after_copy_keeps_the_copy(ctx):
    """A request released right after gfc_server_copy was enqueued on a busy
    stream: the server must not hand its memory to the next batch before
    the copy has read it.  The copy's stream is held up by a spin kernel
    while a second request of the same size renders."""
    import torch
    from paper_2012_15797_amd.serving import Server

    tr = wl.config4_trace(duration_s=0.01, rate_hz=2000.0, restricted=True)
    psfs, mix = _objects(ctx, tr, 1)
    rng = np.random.Generator(np.random.PCG64(11))
    g1 = wl.draw_galaxies(rng, 512, 64, 0)
    g2 = wl.draw_galaxies(rng, 512, 64, 0)
    # budget for one request at a time: the second batch would take the first's block
    one = 512 * (64 * 64 * 4 + 28)
    srv = Server(ctx, mem_budget_bytes=one + 4096, n_streams=1)
    t1 = srv.submit(psfs[0], mix, 64, g1.x, g1.y, g1.flux, g1.r_e, g1.e1, g1.e2)
    srv.wait(t1)
    side = torch.cuda.Stream()
    out1 = torch.empty((512, 64, 64), device="cuda")
    with torch.cuda.stream(side):
        torch.cuda._sleep(50_000_000)  # hold the copy back
        srv.result(t1, out=out1)
    srv.release(t1)
    t2 = srv.submit(psfs[0], mix, 64, g2.x, g2.y, g2.flux, g2.r_e, g2.e1, g2.e2)
    srv.wait(t2)
    side.synchronize()
    ref1 = _direct(ctx, psfs[0], mix, dict(gal=g1, W=64))
    assert torch.equal(out1, ref1)
    out2 = srv.result(t2)
    torch.cuda.synchronize()
    assert torch.equal(out2, _direct(ctx, psfs[0], mix, dict(gal=g2, W=64)))
    srv.release(t2)
    srv.close()
    for p in psfs:
        p.close()
    mix.close()


def test_gfc_log_traces_a_served_request():
    """With GFC_LOG=1 a served run writes JSON lines: the PSF's cache fill,
    each submission, each batch launch (its requests and stamps) and its
    completion.  Run in a child process, since the setting is read once."""
    import json
    import os
    import subprocess
    import sys

    code = r'''
import numpy as np, workloads as wl, paper_2012_15797_amd as gfc
from paper_2012_15797_amd.serving import Server
ctx = gfc.Context.default(0)
cfg = wl.config_metric(10)
psf = gfc.Psf(ctx, cfg["psf"]); mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
srv = Server(ctx, mem_budget_bytes=1 << 30, n_streams=1)
g = cfg["gal"]
ts = [srv.submit(psf, mix, 64, g.x[i::2], g.y[i::2], g.flux[i::2], g.r_e[i::2], g.e1[i::2], g.e2[i::2]) for i in range(2)]
for t in ts:
    srv.wait(t); srv.release(t)
srv.close(); psf.close(); mix.close()
print("done")
'''
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, GFC_LOG="1", PYTHONPATH=root)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240, cwd=root)
    assert r.returncode == 0 and "done" in r.stdout, r.stderr[-2000:]
    ev = [json.loads(ln) for ln in r.stderr.splitlines() if ln.startswith("{")]
    kinds = [e["event"] for e in ev]
    assert "psf_cache_fill" in kinds and kinds.count("server_submit") == 2, kinds
    launches = [e for e in ev if e["event"] == "batch_launch"]
    done = {e["batch"] for e in ev if e["event"] == "batch_complete"}
    assert launches and sum(e["stamps"] for e in launches) == 10 and all(e["W"] == 64 for e in launches)
    assert {e["batch"] for e in launches} == done
    assert all(b["t"] >= a["t"] for a, b in zip(ev, ev[1:]))
