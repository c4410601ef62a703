"""Python objects over the C ABI.  torch provides device memory and the
current HIP stream; every computation runs in libgfc.so."""

from __future__ import annotations

import ctypes
import threading

import numpy as np
import torch

from . import _lib
from ._lib import GFC_KMAX, call, gfc_galaxies, lib

_ctx_lock = threading.Lock()
_default_ctx = {}


def _stream_ptr(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _f32_dev(t, device, name):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t, np.float32))
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    return t.to(device).contiguous()


class Context:
    """One library context per HIP device (owns PSF-FT caches and the
    invalid-galaxy counter)."""

    def __init__(self, device: int = 0):
        self.device = int(device)
        h = ctypes.c_void_p()
        call("gfc_ctx_create", self.device, ctypes.byref(h))
        self.handle = h
        self._objects = []

    @staticmethod
    def default(device: int = 0) -> "Context":
        with _ctx_lock:
            if device not in _default_ctx:
                _default_ctx[device] = Context(device)
            return _default_ctx[device]

    @property
    def torch_device(self):
        return torch.device("cuda", self.device)

    def invalid_count(self) -> int:
        v = ctypes.c_uint64()
        call("gfc_ctx_invalid_count", self.handle, ctypes.byref(v))
        return int(v.value)


class Psf:
    """A pixelized PSF (host array, centre pixel at (S_y/2, S_x/2)) and its
    single-Gaussian approximation {mu_x, mu_y, c_xx, c_xy, c_yy, amp}."""

    def __init__(self, ctx: Context, pixels, gauss=None):
        self.ctx = ctx
        pix = np.ascontiguousarray(pixels)
        if pix.ndim != 2:
            raise ValueError("PSF must be 2-D")
        g = None
        if gauss is not None:
            g = (ctypes.c_double * 6)(*[float(v) for v in gauss])
        h = ctypes.c_void_p()
        if pix.dtype == np.float64:
            call("gfc_psf_create_f64", ctx.handle, pix.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                 pix.shape[0], pix.shape[1], g, ctypes.byref(h))
        else:
            pix = np.ascontiguousarray(pix, np.float32)
            call("gfc_psf_create", ctx.handle, pix.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                 pix.shape[0], pix.shape[1], g, ctypes.byref(h))
        self.handle = h
        self.shape = pix.shape

    @classmethod
    def eigen(cls, ctx: Context, comps, coef, degree: int, norm) -> "Psf":
        """A spatially varying PSF (gfc_psf_create_eigen): component images
        [J, S_y, S_x], polynomial coefficients [J, T] over the terms 1, u, ...,
        v, u v, ... of (u, v) = ((X - norm[0]) / norm[1], (Y - norm[2]) / norm[3])."""
        self = cls.__new__(cls)
        self.ctx = ctx
        c = np.ascontiguousarray(comps, np.float32)
        if c.ndim != 3:
            raise ValueError("eigen-PSF components must be [J, S_y, S_x]")
        T = (degree + 1) * (degree + 2) // 2
        cf = np.ascontiguousarray(coef, np.float64)
        if cf.shape != (c.shape[0], T):
            raise ValueError(f"coef must be [J, {T}] for degree {degree}")
        nm = np.ascontiguousarray(norm, np.float64).reshape(4)
        h = ctypes.c_void_p()
        call("gfc_psf_create_eigen", ctx.handle, c.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
             c.shape[0], c.shape[1], c.shape[2], int(degree),
             cf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
             nm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(h))
        self.handle = h
        self.shape = c.shape[1:]
        self.n_components = c.shape[0]
        return self

    @property
    def gauss(self) -> np.ndarray:
        out = (ctypes.c_double * 6)()
        call("gfc_psf_gauss", self.handle, out)
        return np.array(out[:])

    def prepare(self, W: int) -> None:
        call("gfc_psf_prepare", self.handle, int(W), _stream_ptr(self.ctx.device))

    def spectrum(self, W: int) -> torch.Tensor:
        """The cached PSF spectrum for stamp size W, complex64 [W, W/2+1]
        ([J, W, W/2+1] for an eigen-PSF)."""
        J = getattr(self, "n_components", 0)
        out = torch.empty((max(J, 1), W, W // 2 + 1, 2), dtype=torch.float32, device=self.ctx.torch_device)
        call("gfc_psf_spectrum", self.handle, int(W), ctypes.c_void_p(out.data_ptr()),
             _stream_ptr(self.ctx.device))
        out = torch.view_as_complex(out)
        return out if J else out[0]

    def close(self):
        if self.handle:
            call("gfc_psf_destroy", self.handle)
            self.handle = None


class Mixture:
    """Mixture-of-Gaussians tables: K[t] components with amplitudes and
    isotropic variances (r_e^2 units)."""

    def __init__(self, ctx: Context, K, amp, var):
        self.ctx = ctx
        K = np.asarray(K, np.int32).reshape(-1)
        n = K.shape[0]
        a = np.zeros((n, GFC_KMAX), np.float32)
        v = np.ones((n, GFC_KMAX), np.float32)
        amp = np.asarray(amp, np.float32).reshape(n, -1)
        var = np.asarray(var, np.float32).reshape(n, -1)
        for t in range(n):
            a[t, :K[t]] = amp[t, :K[t]]
            v[t, :K[t]] = var[t, :K[t]]
        self.K = K
        h = ctypes.c_void_p()
        call("gfc_mix_create", ctx.handle, int(n), K.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
             a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
             v.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(h))
        self.handle = h
        self.n_tables = n

    @classmethod
    def from_workload(cls, ctx, mixtures) -> "Mixture":
        return cls(ctx, mixtures.K, mixtures.amp, mixtures.var)

    def device_tables(self):
        a, v = ctypes.c_void_p(), ctypes.c_void_p()
        call("gfc_mix_device_tables", self.handle, ctypes.byref(a), ctypes.byref(v))
        return a.value, v.value

    def close(self):
        if self.handle:
            call("gfc_mix_destroy", self.handle)
            self.handle = None


class SersicFamily:
    """Mixture tables on a grid of Sersic indices (gfc_sersic_create):
    n_grid [S] strictly increasing, amp and var [S, K]."""

    def __init__(self, ctx: Context, n_grid, amp, var):
        self.ctx = ctx
        g = np.ascontiguousarray(n_grid, np.float32).reshape(-1)
        a = np.ascontiguousarray(amp, np.float32)
        v = np.ascontiguousarray(var, np.float32)
        if a.shape != v.shape or a.ndim != 2 or a.shape[0] != g.shape[0]:
            raise ValueError("amp and var must be [S, K] with S = len(n_grid)")
        fp = ctypes.POINTER(ctypes.c_float)
        h = ctypes.c_void_p()
        call("gfc_sersic_create", ctx.handle, int(g.shape[0]), g.ctypes.data_as(fp), int(a.shape[1]),
             a.ctypes.data_as(fp), v.ctypes.data_as(fp), ctypes.byref(h))
        self.handle = h
        self.K = a.shape[1]

    @classmethod
    def from_workload(cls, ctx, fam) -> "SersicFamily":
        return cls(ctx, fam["n_grid"], fam["amp"], fam["var"])

    def close(self):
        if self.handle:
            call("gfc_sersic_destroy", self.handle)
            self.handle = None


def _galaxies(dev, x, y, flux, r_e, e1, e2, mix_id, cd, psf_x=None, psf_y=None, mix_amp=None, n_tables=0):
    ts = [_f32_dev(t, dev, nm) for t, nm in
          zip((x, y, flux, r_e, e1, e2), ("x", "y", "flux", "r_e", "e1", "e2"))]
    n = ts[0].numel()
    if any(t.numel() != n for t in ts):
        raise ValueError("galaxy parameter arrays differ in length")
    mid = None
    if mix_id is not None:
        mid = torch.as_tensor(mix_id).to(device=dev, dtype=torch.int32).contiguous()
        if mid.numel() != n:
            raise ValueError("mix_id length differs")
    g = gfc_galaxies()
    for name, t in zip(("x", "y", "flux", "r_e", "e1", "e2"), ts):
        setattr(g, name, t.data_ptr())
    g.mix_id = mid.data_ptr() if mid is not None else None
    cdbuf = None
    if cd is not None:
        cdbuf = (ctypes.c_float * 4)(*[float(v) for v in np.asarray(cd).reshape(4)])
        g.cd = ctypes.cast(cdbuf, ctypes.POINTER(ctypes.c_float))
    pos = None
    if psf_x is not None or psf_y is not None:
        if psf_x is None or psf_y is None:
            raise ValueError("psf_x and psf_y go together")
        pos = (_f32_dev(psf_x, dev, "psf_x"), _f32_dev(psf_y, dev, "psf_y"))
        if pos[0].numel() != n or pos[1].numel() != n:
            raise ValueError("psf_x/psf_y length differs")
        g.psf_x, g.psf_y = pos[0].data_ptr(), pos[1].data_ptr()
    amp = None
    if mix_amp is not None:
        amp = _f32_dev(mix_amp, dev, "mix_amp")
        if amp.numel() != n_tables * GFC_KMAX:
            raise ValueError("mix_amp must hold n_tables x 16 values")
        g.mix_amp = amp.data_ptr()
    keep = (ts, mid, cdbuf, pos, amp)
    return g, n, keep


def gfc_render_stamps(ctx, psf, mix, x, y, flux, r_e, e1, e2, W, mix_id=None, flags=0, cd=None,
                      out=None, psf_x=None, psf_y=None, mix_amp=None):
    """Forward render (gfc_render_stamps): float32 stamps [n, W, W] on the
    context's device, enqueued on torch's current stream.  psf_x/psf_y: the
    galaxies' image positions, for a spatially varying PSF.  mix_amp: an
    [n_tables, 16] amplitude table for this call (the mixture is unchanged)."""
    dev = ctx.torch_device
    g, n, keep = _galaxies(dev, x, y, flux, r_e, e1, e2, mix_id, cd, psf_x, psf_y, mix_amp, mix.n_tables)
    if out is None:
        out = torch.empty((n, W, W), dtype=torch.float32, device=dev)
    elif out.dtype != torch.float32 or not out.is_contiguous() or out.numel() != n * W * W:
        raise ValueError("out must be a contiguous float32 tensor of n*W*W elements")
    call("gfc_render_stamps", ctx.handle, psf.handle, mix.handle, ctypes.byref(g), int(n), int(W),
         int(flags), ctypes.c_void_p(out.data_ptr()), _stream_ptr(ctx.device))
    del keep
    return out


def _out_tensor(dev, n, W, out):
    if out is None:
        return torch.empty((n, W, W), dtype=torch.float32, device=dev)
    if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() != n * W * W:
        raise ValueError("out must be a contiguous float32 tensor of n*W*W elements")
    return out


def gfc_render_stamps_sersic(ctx, psf, family, x, y, flux, r_e, e1, e2, sersic_n, W, flags=0, cd=None,
                             out=None, psf_x=None, psf_y=None):
    """General-Sersic render (gfc_render_stamps_sersic): each galaxy's mixture
    is interpolated from `family` at its Sersic index."""
    dev = ctx.torch_device
    g, n, keep = _galaxies(dev, x, y, flux, r_e, e1, e2, None, cd, psf_x, psf_y)
    sn = _f32_dev(sersic_n, dev, "sersic_n")
    if sn.numel() != n:
        raise ValueError("sersic_n length differs")
    out = _out_tensor(dev, n, W, out)
    call("gfc_render_stamps_sersic", ctx.handle, psf.handle, family.handle, ctypes.byref(g),
         ctypes.c_void_p(sn.data_ptr()), int(n), int(W), int(flags), ctypes.c_void_p(out.data_ptr()),
         _stream_ptr(ctx.device))
    del keep, sn
    return out


def gfc_render_stamps_composite(ctx, psf, mix, disk_table, bulge_table, x, y, flux, r_e, e1, e2, bulge_frac,
                                bulge_rho, W, flags=0, cd=None, out=None, psf_x=None, psf_y=None):
    """Bulge + disk render with one ellipticity (gfc_render_stamps_composite);
    r_e is the disk's, bulge_rho the bulge-to-disk radius ratio."""
    dev = ctx.torch_device
    g, n, keep = _galaxies(dev, x, y, flux, r_e, e1, e2, None, cd, psf_x, psf_y)
    fr = _f32_dev(bulge_frac, dev, "bulge_frac")
    rh = _f32_dev(bulge_rho, dev, "bulge_rho")
    if fr.numel() != n or rh.numel() != n:
        raise ValueError("bulge_frac/bulge_rho length differs")
    out = _out_tensor(dev, n, W, out)
    call("gfc_render_stamps_composite", ctx.handle, psf.handle, mix.handle, int(disk_table), int(bulge_table),
         ctypes.byref(g), ctypes.c_void_p(fr.data_ptr()), ctypes.c_void_p(rh.data_ptr()), int(n), int(W),
         int(flags), ctypes.c_void_p(out.data_ptr()), _stream_ptr(ctx.device))
    del keep, fr, rh
    return out


def gfc_backward_workspace_bytes(n: int) -> int:
    return int(lib().gfc_backward_workspace_bytes(int(n)))


def gfc_render_stamps_backward(ctx, psf, mix, x, y, flux, r_e, e1, e2, W, grad_out, mix_id=None,
                               flags=0, cd=None, grad_params=None, grad_amp=None, workspace=None, mix_amp=None,
                               amp_grad=True):
    """Adjoint (gfc_render_stamps_backward): returns (grad_params [n, 6] =
    dL/d(x, y, flux, log r_e, e1, e2), grad_amp [n_tables, 16] accumulated).
    mix_amp: the per-call amplitude table of the forward render, if it had one.
    amp_grad=False passes NULL for grad_amp (no amplitude gradient, so no
    reduction launches) and returns None in its place."""
    dev = ctx.torch_device
    g, n, keep = _galaxies(dev, x, y, flux, r_e, e1, e2, mix_id, cd, mix_amp=mix_amp, n_tables=mix.n_tables)
    go = grad_out.to(dev, torch.float32).contiguous()
    if go.numel() != n * W * W:
        raise ValueError("grad_out must hold n*W*W elements")
    if grad_params is None:
        grad_params = torch.empty((n, 6), dtype=torch.float32, device=dev)
    if not amp_grad:
        grad_amp = None
    elif grad_amp is None:
        grad_amp = torch.zeros((mix.n_tables, GFC_KMAX), dtype=torch.float32, device=dev)
    ws = ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else None
    call("gfc_render_stamps_backward", ctx.handle, psf.handle, mix.handle, ctypes.byref(g), int(n),
         int(W), int(flags), ctypes.c_void_p(go.data_ptr()), ctypes.c_void_p(grad_params.data_ptr()),
         ctypes.c_void_p(grad_amp.data_ptr()) if grad_amp is not None else None, ws, _stream_ptr(ctx.device))
    del keep
    return grad_params, grad_amp


def gfc_render_stamps_backward_noalloc(ctx, psf, mix, x, y, flux, r_e, e1, e2, W, grad_out, mix_id=None,
                                       flags=0, cd=None, grad_params=None, grad_amp=None):
    """Allocation-free adjoint (gfc_render_stamps_backward_noalloc): the
    library's scratch is a fixed per-device array, so the C call allocates
    nothing (W <= 128, n <= GFC_NOALLOC_MAX_GALAXIES, the PSF spectrum for W
    prepared beforehand).  Output tensors are allocated here by torch unless
    the caller passes them.  Returns (grad_params [n, 6], grad_amp
    [n_tables, 16] accumulated)."""
    dev = ctx.torch_device
    g, n, keep = _galaxies(dev, x, y, flux, r_e, e1, e2, mix_id, cd)
    go = grad_out.to(dev, torch.float32).contiguous()
    if go.numel() != n * W * W:
        raise ValueError("grad_out must hold n*W*W elements")
    if grad_params is None:
        grad_params = torch.empty((n, 6), dtype=torch.float32, device=dev)
    if grad_amp is None:
        grad_amp = torch.zeros((mix.n_tables, GFC_KMAX), dtype=torch.float32, device=dev)
    call("gfc_render_stamps_backward_noalloc", ctx.handle, psf.handle, mix.handle, ctypes.byref(g), int(n),
         int(W), int(flags), ctypes.c_void_p(go.data_ptr()), ctypes.c_void_p(grad_params.data_ptr()),
         ctypes.c_void_p(grad_amp.data_ptr()), _stream_ptr(ctx.device))
    del keep
    return grad_params, grad_amp
