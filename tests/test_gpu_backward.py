"""GPU parity of the adjoint (gfc_render_stamps_backward, through the C ABI)
against the FP64 derivative oracle, which itself is pinned to central finite
differences on the CPU (tests/test_oracle_grad.py).

Bar: for each parameter, |gpu - oracle| <= 1e-4 |oracle| wherever |oracle| is
at least 1e-2 of its rms over the case's galaxies; below that 1e-5 rms is
added (gradients that cancel to nearly zero, or galaxies far fainter than the
case's brightest, whose float32 rounding is set by the size of the summed
terms, not by the result)."""

import math

import numpy as np
import pytest

import oracle as o
import workloads as wl
from gpu_helpers import assert_grads_close as assert_close, gpu_grads, lib_objects, oracle_grads
from oracle.grad import PARAMS

pytestmark = pytest.mark.gpu

@pytest.fixture(scope="module")
def ctx():
    import paper_2012_15797_amd as gfc
    return gfc.Context.default(0)


@pytest.mark.parametrize("W", [16, 32, 64, 128, 256])
def test_backward_each_size(ctx, W):
    rng = np.random.Generator(np.random.PCG64(300 + W))
    cfg = wl.config2(10)
    n = 40 if W < 128 else (12 if W == 128 else 10)
    gal = wl.draw_galaxies(rng, n, W, (np.arange(n) % 2).astype(np.int32), r_e_range=(0.4, W / 5.0))
    g = rng.standard_normal((n, W, W)).astype(np.float32)
    psf, mix = lib_objects(ctx, cfg)
    gp, ga = gpu_grads(ctx, psf, mix, gal, W, g)
    rp, ra, ra_abs = oracle_grads(cfg, gal, g)
    assert_close(gp, rp, f"params W={W}")
    assert_close(ga, ra, f"amplitudes W={W}", scale=ra_abs)
    psf.close(); mix.close()


def test_backward_w256_across_chunks(ctx):
    """W = 256 runs in chunks of 1024 stamps over one reused device slab;
    galaxies on both sides of the chunk boundary, and the last, are checked
    against the oracle (the others must be finite)."""
    rng = np.random.Generator(np.random.PCG64(310))
    cfg = wl.config2(10)
    W, n = 256, 1030
    gal = wl.draw_galaxies(rng, n, W, (np.arange(n) % 2).astype(np.int32), r_e_range=(0.4, W / 5.0))
    g = rng.standard_normal((n, W, W)).astype(np.float32)
    psf, mix = lib_objects(ctx, cfg)
    gp, _ = gpu_grads(ctx, psf, mix, gal, W, g)
    assert np.isfinite(gp).all()
    idx = [0, 1, 1022, 1023, 1024, 1025, 1029]
    rp, _, _ = oracle_grads(cfg, gal.subset(idx), g[idx])
    assert_close(gp[idx], rp, "params W=256 chunk boundary")
    psf.close(); mix.close()


@pytest.mark.parametrize("flags", [1, 2, 4])
def test_backward_routing_flags(ctx, flags):
    rng = np.random.Generator(np.random.PCG64(400 + flags))
    cfg = wl.config_metric(10)
    W, n = 32, 30
    gal = wl.draw_galaxies(rng, n, W, 0, r_e_range=(0.4, 6.0))
    g = rng.standard_normal((n, W, W)).astype(np.float32)
    psf, mix = lib_objects(ctx, cfg)
    gp, ga = gpu_grads(ctx, psf, mix, gal, W, g, flags=flags)
    rp, ra, ra_abs = oracle_grads(cfg, gal, g, flags=flags)
    assert_close(gp, rp, f"params flags={flags}")
    assert_close(ga, ra, f"amplitudes flags={flags}", scale=ra_abs)
    psf.close(); mix.close()


@pytest.mark.parametrize("W", [16, 64, 128, 256])
def test_backward_forced_real_each_size(ctx, W):
    """Every component in real space (GFC_FORCE_REAL = 2): the adjoint's
    pixel-space sums alone carry the shape, position and amplitude terms, at
    each kernel's stamp size (the 256 kernel sums over 512 threads)."""
    rng = np.random.Generator(np.random.PCG64(450 + W))
    cfg = wl.config2(10)
    n = 16 if W < 128 else 6
    gal = wl.draw_galaxies(rng, n, W, (np.arange(n) % 2).astype(np.int32), r_e_range=(0.4, W / 5.0))
    g = rng.standard_normal((n, W, W)).astype(np.float32)
    psf, mix = lib_objects(ctx, cfg)
    gp, ga = gpu_grads(ctx, psf, mix, gal, W, g, flags=2)
    rp, ra, ra_abs = oracle_grads(cfg, gal, g, flags=2)
    assert_close(gp, rp, f"params W={W} forced real")
    assert_close(ga, ra, f"amplitudes W={W} forced real", scale=ra_abs)
    psf.close(); mix.close()


def test_backward_fit_workload(ctx):
    """The differentiation workload: DEV8, 64x64, upstream gradient
    (I - T) / sigma^2 with T = render at perturbed parameters plus noise of
    0.01 x peak; 40 galaxies."""
    cfg = wl.config5(40)
    gal, tgt = cfg["gal"], cfg["target_gal"]
    idx = list(range(len(gal)))
    I = np.stack(o.render_batch(cfg["psf"].astype(np.float64), cfg["mix"].as_f32(), gal, idx=idx))
    T = np.stack(o.render_batch(cfg["psf"].astype(np.float64), cfg["mix"].as_f32(), tgt, idx=idx))
    peak = np.abs(T).max(axis=(1, 2), keepdims=True)
    sigma = 0.01 * peak
    T = T + sigma * wl.generate.noise_field(cfg["noise_seed"], len(gal), 64)
    g = ((I - T) / sigma**2).astype(np.float32)
    psf, mix = lib_objects(ctx, cfg)
    gp, ga = gpu_grads(ctx, psf, mix, gal, 64, g)
    rp, ra, ra_abs = oracle_grads(cfg, gal, g)
    assert_close(gp, rp, "params fit workload")
    assert_close(ga, ra, "amplitudes fit workload", scale=ra_abs)
    psf.close(); mix.close()


def test_backward_cd_matrix(ctx):
    rng = np.random.Generator(np.random.PCG64(500))
    cfg = wl.config_metric(10)
    W, n = 32, 20
    gal = wl.draw_galaxies(rng, n, W, 0, r_e_range=(0.4, 6.0))
    g = rng.standard_normal((n, W, W)).astype(np.float32)
    cd = np.array([0.9, 0.15, -0.2, 1.1], np.float32)
    psf, mix = lib_objects(ctx, cfg)
    gp, ga = gpu_grads(ctx, psf, mix, gal, W, g, cd=cd)
    rp, ra, ra_abs = oracle_grads(cfg, gal, g, cd=cd.astype(np.float64))
    assert_close(gp, rp, "params cd")
    assert_close(ga, ra, "amplitudes cd", scale=ra_abs)
    psf.close(); mix.close()


def test_backward_deterministic_and_accumulating(ctx):
    import torch
    import paper_2012_15797_amd as gfc

    rng = np.random.Generator(np.random.PCG64(600))
    cfg = wl.config_metric(10)
    W, n = 64, 300
    gal = wl.draw_galaxies(rng, n, W, 0)
    g = torch.as_tensor(rng.standard_normal((n, W, W)).astype(np.float32)).cuda()
    psf, mix = lib_objects(ctx, cfg)
    args = (ctx, psf, mix, gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2, W, g)
    gp1, ga1 = gfc.gfc_render_stamps_backward(*args)
    gp2, ga2 = gfc.gfc_render_stamps_backward(*args)
    assert torch.equal(gp1, gp2) and torch.equal(ga1, ga2)
    acc = torch.zeros_like(ga1)
    gfc.gfc_render_stamps_backward(*args, grad_amp=acc)
    gfc.gfc_render_stamps_backward(*args, grad_amp=acc)
    torch.cuda.synchronize()
    assert torch.allclose(acc, 2 * ga1, rtol=1e-6, atol=0)
    # grad_amp NULL: no amplitude reduction, the parameter gradients unchanged
    gp3, ga3 = gfc.gfc_render_stamps_backward(*args, amp_grad=False)
    torch.cuda.synchronize()
    assert ga3 is None and torch.equal(gp3, gp1)
    psf.close(); mix.close()


@pytest.mark.parametrize("W", [16, 128, 256])
def test_backward_without_amplitude_gradient(ctx, W):
    """grad_amp NULL launches no amplitude reduction and leaves the parameter
    gradients bit for bit as they are with it (the bench times the adjoint
    kernel alone this way)."""
    import torch
    import paper_2012_15797_amd as gfc

    rng = np.random.Generator(np.random.PCG64(650 + W))
    cfg = wl.config2(10)
    n = 37 if W < 128 else 9
    gal = wl.draw_galaxies(rng, n, W, (np.arange(n) % 2).astype(np.int32), r_e_range=(0.4, W / 5.0))
    g = torch.as_tensor(rng.standard_normal((n, W, W)).astype(np.float32)).cuda()
    psf, mix = lib_objects(ctx, cfg)
    args = (ctx, psf, mix, gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2, W, g)
    gp1, ga1 = gfc.gfc_render_stamps_backward(*args, mix_id=gal.mix_id)
    gp2, ga2 = gfc.gfc_render_stamps_backward(*args, mix_id=gal.mix_id, amp_grad=False)
    torch.cuda.synchronize()
    assert ga2 is None and bool(torch.isfinite(ga1).all())
    assert torch.equal(gp1, gp2)
    psf.close(); mix.close()


def test_autograd_function_matches_adjoint(ctx):
    """torch.autograd through RenderStamps gives the library adjoint, with the
    log r_e chain applied (dL/dr_e = dL/dlog r_e / r_e) and amplitude
    gradients for a torch-held amplitude table."""
    import torch
    import paper_2012_15797_amd as gfc

    rng = np.random.Generator(np.random.PCG64(700))
    cfg = wl.config_metric(10)
    W, n = 32, 25
    gal = wl.draw_galaxies(rng, n, W, 0, r_e_range=(0.5, 5.0))
    psf, mix = lib_objects(ctx, cfg)
    dev = torch.device("cuda")
    t = lambda a: torch.tensor(a, device=dev, requires_grad=True)
    x, y, fl, re, e1, e2 = map(t, (gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2))
    m = cfg["mix"].as_f32()
    table = np.asarray(m.amp, np.float32)
    new_amp = (table * np.linspace(0.5, 1.5, 16, dtype=np.float32)[None, :]).astype(np.float32)
    amp = torch.tensor(new_amp, device=dev, requires_grad=True)
    g = torch.as_tensor(rng.standard_normal((n, W, W)).astype(np.float32), device=dev)
    before = gfc.gfc_render_stamps(ctx, psf, mix, gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2, W)
    out = gfc.render(psf, mix, x, y, fl, re, e1, e2, W, amp=amp)
    (out * g).sum().backward()
    gp, ga = gfc.gfc_render_stamps_backward(ctx, psf, mix, gal.x, gal.y, gal.flux, gal.r_e, gal.e1,
                                            gal.e2, W, g, mix_amp=amp.detach())
    torch.cuda.synchronize()
    # the per-call amplitudes leave the shared mixture as it was ...
    after = gfc.gfc_render_stamps(ctx, psf, mix, gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2, W)
    torch.cuda.synchronize()
    assert torch.equal(before, after) and not torch.equal(before, out.detach())
    # ... and render as a mixture made with them would
    mix2 = gfc.Mixture(ctx, np.asarray(m.K, np.int32), new_amp, np.asarray(m.var, np.float32))
    ref = gfc.gfc_render_stamps(ctx, psf, mix2, gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2, W)
    torch.cuda.synchronize()
    assert torch.equal(out.detach(), ref)
    mix2.close()
    for i, tt in enumerate((x, y, fl)):
        assert torch.allclose(tt.grad, gp[:, i])
    assert torch.allclose(re.grad, gp[:, 3] / re.detach())
    assert torch.allclose(e1.grad, gp[:, 4]) and torch.allclose(e2.grad, gp[:, 5])
    assert torch.allclose(amp.grad, ga)
    psf.close(); mix.close()


_PER_GALAXY = {}  # contributions from the first case, compared bit for bit by the others


@pytest.mark.parametrize("n_tables", [1700, 70000, (1 << 20) // 14 + 1])
def test_amplitude_sums_across_chunks_and_tables(ctx, n_tables):
    """The per-table amplitude sums over 1,700 galaxies (14 chunks of 128 in
    the two-pass reduction, the last one ragged).  Every table is a copy of
    one mixture, so a call that gives each galaxy its own table returns each
    galaxy's contribution exactly (one term per sum); a call with four shared
    tables must then equal their float64 sums per table.  70,000 tables take
    two launches of the first pass (at most 65,535 tables per grid row); with
    74,899 the chunk partials would pass 64 MiB and the one-pass reduction
    runs instead (its single-term sums must equal the others bit for bit)."""
    import torch
    import paper_2012_15797_amd as gfc

    n, W = 1700, 16
    rng = np.random.Generator(np.random.PCG64(700))  # the same galaxies in every case
    cfg = wl.config_metric(10)
    m = cfg["mix"].as_f32()
    K = np.full(n_tables, int(m.K[0]), np.int32)
    amp = np.broadcast_to(np.asarray(m.amp, np.float32)[:1], (n_tables, 16))
    var = np.broadcast_to(np.asarray(m.var, np.float32)[:1], (n_tables, 16))
    psf = gfc.Psf(ctx, cfg["psf"], cfg.get("psf_gauss"))
    mix = gfc.Mixture(ctx, K, amp, var)
    gal = wl.draw_galaxies(rng, n, W, 0)
    g = torch.as_tensor(rng.standard_normal((n, W, W)).astype(np.float32)).cuda()

    def amp_sums(mix_id):
        _, ga = gfc.gfc_render_stamps_backward(ctx, psf, mix, gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2,
                                               W, g, mix_id=np.asarray(mix_id, np.int32))
        torch.cuda.synchronize()
        return ga.cpu().numpy()

    own = np.arange(n) % n_tables
    per_gal = amp_sums(own)[own].astype(np.float64)  # [n, 16], galaxy i's contribution
    used = np.array(sorted({0, min(65535, n_tables - 1), n_tables // 3, n_tables - 1}))
    shared = used[rng.integers(0, len(used), n)]
    got = amp_sums(shared)
    ref = np.zeros((n_tables, 16))
    scale = np.zeros((n_tables, 16))
    np.add.at(ref, shared, per_gal)
    np.add.at(scale, shared, np.abs(per_gal))
    err = np.abs(got - ref)
    assert (err <= 1e-5 * scale).all(), float((err / np.maximum(scale, 1e-300)).max())
    unused = np.setdiff1d(np.arange(n_tables), used)
    assert (got[unused] == 0).all()
    first = _PER_GALAXY.setdefault("per_gal", per_gal)
    assert np.array_equal(per_gal, first)
    psf.close(); mix.close()
