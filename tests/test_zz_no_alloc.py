"""The allocation-free adjoint (gfc_render_stamps_backward_noalloc, through
the C ABI) against the allocating one (gfc_render_stamps_backward): the same
kernels, so the same gradients bit for bit, on two calls in a row that share
the library's scratch array, the second with fewer galaxies and a smaller
stamp size; the one-pass amplitude sums used beyond 16 tables; and the
limits, refused on the host before anything is launched."""

import ctypes

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2012_15797_amd as gfc
    return gfc.Context.default(0)


def _both(ctx, psf, mix, gal, W, g):
    import torch
    import paper_2012_15797_amd as gfc

    args = (ctx, psf, mix, gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2, W, g)
    ref_p, ref_a = gfc.gfc_render_stamps_backward(*args, mix_id=gal.mix_id)
    got_p, got_a = gfc.gfc_render_stamps_backward_noalloc(*args, mix_id=gal.mix_id)
    torch.cuda.synchronize()
    return ref_p, ref_a, got_p, got_a


def test_two_calls_in_a_row_match_the_allocating_adjoint(ctx):
    import torch
    import paper_2012_15797_amd as gfc

    cfg = wl.config2(10)
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    rng = np.random.Generator(np.random.PCG64(4242))
    for W, n in ((64, 3000), (32, 700)):          # the second call is smaller
        psf.prepare(W)
        gal = wl.draw_galaxies(rng, n, W, (np.arange(n) % 2).astype(np.int32), r_e_range=(0.4, W / 5.0))
        g = torch.as_tensor(rng.standard_normal((n, W, W)).astype(np.float32)).cuda()
        ref_p, ref_a, got_p, got_a = _both(ctx, psf, mix, gal, W, g)
        assert torch.isfinite(ref_p).all()
        assert torch.equal(got_p, ref_p), (W, n, float((got_p - ref_p).abs().max()))
        assert torch.equal(got_a, ref_a), (W, n, float((got_a - ref_a).abs().max()))
    psf.close(); mix.close()


def test_many_tables_use_the_one_pass_sums(ctx):
    """20 tables: the allocating adjoint sums them in two passes with
    partials it allocates; the allocation-free one in one pass without
    partials.  Parameter gradients are equal bit for bit; the amplitude sums
    agree to float32 summation-order rounding."""
    import torch
    import paper_2012_15797_amd as gfc

    cfg = wl.config_metric(10)
    m = cfg["mix"].as_f32()
    nt = 20
    K = np.full(nt, int(m.K[0]), np.int32)
    amp = np.repeat(np.asarray(m.amp, np.float32)[:1], nt, axis=0)
    var = np.repeat(np.asarray(m.var, np.float32)[:1], nt, axis=0)
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture(ctx, K, amp, var)
    W, n = 32, 2000
    psf.prepare(W)
    rng = np.random.Generator(np.random.PCG64(4343))
    gal = wl.draw_galaxies(rng, n, W, (np.arange(n) % nt).astype(np.int32))
    g = torch.as_tensor(rng.standard_normal((n, W, W)).astype(np.float32)).cuda()
    ref_p, ref_a, got_p, got_a = _both(ctx, psf, mix, gal, W, g)
    assert torch.equal(got_p, ref_p)
    scale = float(ref_a.abs().max())
    assert torch.allclose(got_a, ref_a, rtol=1e-5, atol=1e-6 * scale), float((got_a - ref_a).abs().max())
    psf.close(); mix.close()


def test_limits_are_refused_before_any_launch(ctx):
    import torch
    import paper_2012_15797_amd as gfc
    from paper_2012_15797_amd._lib import gfc_galaxies

    cfg = wl.config_metric(4)
    psf = gfc.Psf(ctx, cfg["psf"])
    mix = gfc.Mixture.from_workload(ctx, cfg["mix"].as_f32())
    gal = cfg["gal"]
    dev = torch.device("cuda", 0)
    t = [torch.as_tensor(a).to(dev) for a in (gal.x, gal.y, gal.flux, gal.r_e, gal.e1, gal.e2)]
    gg = gfc_galaxies(*(ctypes.c_void_p(a.data_ptr()) for a in t), None, None, None, None)
    go = torch.zeros((4, 256, 256), device=dev)
    gp = torch.zeros((4, 6), device=dev)
    lib = gfc.lib()

    def call(n, W):
        return lib.gfc_render_stamps_backward_noalloc(ctx.handle, psf.handle, mix.handle, ctypes.byref(gg), n, W,
                                                      0, ctypes.c_void_p(go.data_ptr()),
                                                      ctypes.c_void_p(gp.data_ptr()), None, None)

    assert call(4, 64) == -1                     # PSF spectrum for 64 not prepared yet
    assert b"gfc_psf_prepare" in lib.gfc_last_error()
    psf.prepare(64)
    psf.prepare(256)
    assert call(4, 256) == -1                    # W > 128
    assert call(gfc.GFC_NOALLOC_MAX_GALAXIES + 1, 64) == -1
    assert b"GFC_NOALLOC_MAX_GALAXIES" in lib.gfc_last_error()
    assert call(0, 64) == 0
    assert call(4, 64) == 0
    torch.cuda.synchronize()
    assert torch.isfinite(gp).all()
    psf.close(); mix.close()
