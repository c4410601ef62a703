"""Python front ends of the serving layer.

`Server` wraps gfc_server_* (continuous batching on the device).  `Scheduler`
wraps gfc_sched_*: the same scheduling core with the device replaced by
Python callbacks, stepped explicitly (a simulated clock makes its policy
testable without a GPU)."""

from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import call, gfc_request, lib

STATE = {0: "pending", 1: "admitted", 2: "launched", 3: "done", 4: "failed"}


class Server:
    def __init__(self, ctx, mem_budget_bytes: int, n_streams: int = 2, max_batch_stamps: int = 65536):
        self.ctx = ctx
        h = ctypes.c_void_p()
        call("gfc_server_create", ctx.handle, int(mem_budget_bytes), int(n_streams), int(max_batch_stamps),
             ctypes.byref(h))
        self.handle = h
        self._meta = {}

    @staticmethod
    def prepare(psf, mix, W, x, y, flux, r_e, e1, e2, mix_id=None, flags=0):
        """Marshals one request (host arrays) into a gfc_request, ready to submit."""
        arrs = [np.ascontiguousarray(a, np.float32) for a in (x, y, flux, r_e, e1, e2)]
        n = arrs[0].shape[0]
        q = gfc_request()
        q.psf, q.mix, q.W, q.n, q.flags = psf.handle.value, mix.handle.value, int(W), int(n), int(flags)
        for name, a in zip(("x", "y", "flux", "r_e", "e1", "e2"), arrs):
            setattr(q, name, a.ctypes.data)
        mid = None
        if mix_id is not None:
            mid = np.ascontiguousarray(mix_id, np.int32)
            q.mix_id = mid.ctypes.data
        return (q, arrs, mid, n, int(W))

    def submit_prepared(self, prepared) -> int:
        q, _arrs, _mid, n, W = prepared
        t = ctypes.c_uint64()
        call("gfc_server_submit", self.handle, ctypes.byref(q), ctypes.byref(t))
        self._meta[t.value] = (n, W)
        return t.value

    def submit(self, psf, mix, W, x, y, flux, r_e, e1, e2, mix_id=None, flags=0) -> int:
        """Queues a request with host parameter arrays (copied); returns its ticket."""
        return self.submit_prepared(self.prepare(psf, mix, W, x, y, flux, r_e, e1, e2, mix_id, flags))

    def poll(self, ticket: int):
        done, st = ctypes.c_int(), ctypes.c_int()
        call("gfc_server_poll", self.handle, ticket, ctypes.byref(done), None, ctypes.byref(st))
        return bool(done.value), st.value

    def wait(self, ticket: int, timeout_ms: int = -1) -> None:
        call("gfc_server_wait", self.handle, ticket, int(timeout_ms), None)

    def result(self, ticket: int, out=None):
        """Copies a finished request's stamps into a torch tensor [n, W, W]."""
        import torch

        from .api import _stream_ptr

        n, W = self._meta[ticket]
        if out is None:
            out = torch.empty((n, W, W), dtype=torch.float32, device=self.ctx.torch_device)
        call("gfc_server_copy", self.handle, ticket, ctypes.c_void_p(out.data_ptr()),
             _stream_ptr(self.ctx.device))
        return out

    def release(self, ticket: int) -> None:
        call("gfc_server_release", self.handle, ticket)
        self._meta.pop(ticket, None)

    def stats(self) -> dict:
        d = [ctypes.c_double() for _ in range(4)]
        u = [ctypes.c_uint64() for _ in range(2)]
        call("gfc_server_stats", self.handle, *[ctypes.byref(v) for v in d], *[ctypes.byref(v) for v in u])
        return dict(p50_ms=d[0].value, p99_ms=d[1].value, max_ms=d[2].value, stamps_per_s=d[3].value,
                    launches=u[0].value, done=u[1].value)

    def close(self) -> None:
        if self.handle:
            call("gfc_server_destroy", self.handle)
            self.handle = None


class Scheduler:
    """Scheduling core with callback-simulated device.  `launch(batch, stream,
    tickets, n_stamps) -> int`, `poll(batch) -> int`, `release(batch)` and
    `now() -> float` are Python callables."""

    def __init__(self, now, launch, poll, release, mem_budget_bytes, n_streams=1, max_batch_stamps=1 << 20):
        self._cb = [
            _lib.SCHED_NOW(lambda u: float(now())),
            _lib.SCHED_LAUNCH(lambda u, b, s, nr, t, ns: int(launch(b, s, [t[i] for i in range(nr)], ns))),
            _lib.SCHED_POLL(lambda u, b: int(poll(b))),
            _lib.SCHED_RELEASE(lambda u, b: release(b)),
        ]
        ex = _lib.gfc_sched_executor(None, *self._cb)
        self._ex = ex
        h = ctypes.c_void_p()
        call("gfc_sched_create", ctypes.byref(ex), int(mem_budget_bytes), int(n_streams),
             int(max_batch_stamps), ctypes.byref(h))
        self.handle = h

    def submit(self, key: int, n_stamps: int, nbytes: int) -> int:
        t = ctypes.c_uint64()
        call("gfc_sched_submit", self.handle, int(key), int(n_stamps), int(nbytes), ctypes.byref(t))
        return t.value

    def step(self) -> None:
        call("gfc_sched_step", self.handle)

    def query(self, ticket: int):
        st, b = ctypes.c_int(), ctypes.c_uint64()
        call("gfc_sched_query", self.handle, int(ticket), ctypes.byref(st), ctypes.byref(b))
        return STATE[st.value], b.value

    def release(self, ticket: int) -> None:
        call("gfc_sched_release", self.handle, int(ticket))

    def usage(self):
        b, p = ctypes.c_size_t(), ctypes.c_uint64()
        call("gfc_sched_usage", self.handle, ctypes.byref(b), ctypes.byref(p))
        return b.value, p.value

    def stats(self) -> dict:
        d = [ctypes.c_double() for _ in range(4)]
        u = [ctypes.c_uint64() for _ in range(2)]
        call("gfc_sched_stats", self.handle, *[ctypes.byref(v) for v in d], *[ctypes.byref(v) for v in u])
        return dict(p50_ms=d[0].value, p99_ms=d[1].value, max_ms=d[2].value, stamps_per_s=d[3].value,
                    launches=u[0].value, done=u[1].value)

    def close(self) -> None:
        if self.handle:
            call("gfc_sched_destroy", self.handle)
            self.handle = None


def replay_trace(server, requests, psfs, mix, flags=0, keep=None):
    """Open-loop replay of a request trace (dicts with t [s], psf index, W,
    gal) against a server with the library's native load generator
    (gfc_server_replay): submissions at the arrival times and in-order
    waits and releases run on host threads of their own, so the Python
    interpreter does not pace the trace.  Returns server-side latency
    percentiles (submit to completion observed by the server), throughput
    over the trace, and the submission lag behind the schedule.  keep:
    {request index: device tensor [n, W, W]} receiving those requests'
    stamps before their release."""
    n_req = len(requests)
    prepared = []
    stamps = 0
    for r in requests:
        g = r["gal"]
        prepared.append(server.prepare(psfs[r["psf"]], mix, r["W"], g.x, g.y, g.flux, g.r_e, g.e1, g.e2,
                                       mix_id=g.mix_id, flags=flags))
        stamps += len(g)
    reqs = (gfc_request * n_req)(*[p[0] for p in prepared])
    t_arr = np.ascontiguousarray([r["t"] for r in requests], np.float64)
    lag = np.zeros(n_req, np.float64)
    span = ctypes.c_double()
    D_p = ctypes.POINTER(ctypes.c_double)
    keep_arr = None
    if keep:
        keep_arr = (ctypes.c_void_p * n_req)()
        for i, t in keep.items():
            keep_arr[i] = t.data_ptr()
    call("gfc_server_replay", server.handle, reqs, t_arr.ctypes.data_as(D_p), n_req, keep_arr,
         lag.ctypes.data_as(D_p), ctypes.byref(span))
    st = server.stats()
    return dict(requests=n_req, stamps=stamps, offered_rate_hz=n_req / max(requests[-1]["t"], 1e-9),
                p50_ms=round(st["p50_ms"], 4), p99_ms=round(st["p99_ms"], 4), max_ms=round(st["max_ms"], 4),
                stamps_per_s=round(stamps / max(span.value, 1e-9), 1), launches=st["launches"],
                submit_lag_p99_ms=round(float(np.percentile(lag, 99)) * 1e3, 4))
