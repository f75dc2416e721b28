"""Serving driver: replays a request trace against libqsv's serving engine.

The engine (qsv_server_*: admission by HBM footprint, three native worker
lanes whose device work overlaps: persistent launches over slices of the
admitted shots requests, wide requests on the tile passes, energy+gradient
requests batched per program) is native; this module only submits requests at
their arrival times, calls the non-blocking admission step and records
latencies.
"""
import ctypes as C
import time

import numpy as np

from . import _abi as A
from .api import QsvError, ShotResultArrays, _ptr


class Server:
    def __init__(self, ctx, hbm_budget, shots_per_tick=256):
        self.ctx = ctx
        h = C.c_void_p()
        rc = A.lib().qsv_server_create(ctx.handle, int(hbm_budget), int(shots_per_tick), C.byref(h))
        if rc:
            raise QsvError(rc, "qsv_server_create failed")
        self.handle = h
        self._keep = {}

    def close(self):
        if self.handle:
            A.lib().qsv_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, prog, shots, theta=None, seed=0):
        th = None
        if prog.info.n_params:
            th = np.ascontiguousarray(theta, dtype=np.float64)
        t = C.c_uint64()
        self.ctx.check(A.lib().qsv_submit(self.handle, prog.handle, _ptr(th), int(shots),
                                          int(seed) & 0xFFFFFFFFFFFFFFFF, C.byref(t)))
        self._keep[t.value] = ("shots", prog, int(shots))
        return t.value

    def submit_expval_grad(self, prog, theta, coeffs, codes):
        th = np.ascontiguousarray(theta, dtype=np.float64)
        h, keep = prog._pauli(coeffs, codes)
        t = C.c_uint64()
        self.ctx.check(A.lib().qsv_submit_expval_grad(self.handle, prog.handle, _ptr(th), C.byref(h), C.byref(t)))
        self._keep[t.value] = ("vqe", prog, 0)
        return t.value

    def profile(self):
        """qsv_server_profile: the lanes' summed profile as a dict."""
        p = A.Profile()
        self.ctx.check(A.lib().qsv_server_profile(self.handle, C.byref(p)))
        return {k: getattr(p, k) for k, _ in A.Profile._fields_}

    def step(self):
        r, w = C.c_uint32(), C.c_uint32()
        self.ctx.check(A.lib().qsv_server_step(self.handle, C.byref(r), C.byref(w)))
        return r.value, w.value

    def done(self, ticket):
        d = C.c_int32()
        self.ctx.check(A.lib().qsv_poll(self.handle, ticket, C.byref(d)))
        return bool(d.value)

    def fetch(self, ticket):
        kind, prog, shots = self._keep.pop(ticket)
        if kind == "vqe":
            e = np.zeros(1)
            g = np.zeros(max(1, prog.info.n_params))
            self.ctx.check(A.lib().qsv_fetch_expval_grad(self.handle, ticket, _ptr(e), _ptr(g)))
            return float(e[0]), g[:prog.info.n_params]
        bufs = prog._result_buffers(shots)
        res = A.ShotResults(*[_ptr(b) for b in bufs])
        self.ctx.check(A.lib().qsv_fetch_shots(self.handle, ticket, C.byref(res)))
        creg, record, nev, prob, status = bufs
        return ShotResultArrays(creg, record[:, :prog.info.max_events], nev, prob, status, None,
                                prog.lowered.n_clbits)


def replay(ctx, requests, hbm_budget, shots_per_tick=256, drain_limit_s=60.0, log=None, profile=False):
    """Replays requests (dicts with arrival, kind, prog, shots/theta/coeffs/codes, seed)
    in real time. Returns per-request latencies and aggregate counters (and the
    lanes' profile with profile=True)."""
    srv = Server(ctx, hbm_budget, shots_per_tick)
    reqs = sorted(requests, key=lambda r: r["arrival"])
    t0 = time.perf_counter()
    nxt, tickets, lat, results = 0, {}, {}, {}
    window = reqs[-1]["arrival"] if reqs else 0.0
    shots_done = 0
    ticks = 0
    backlog_at_window = None
    while True:
        now = time.perf_counter() - t0
        while nxt < len(reqs) and reqs[nxt]["arrival"] <= now:
            r = reqs[nxt]
            if r["kind"] == "vqe":
                t = srv.submit_expval_grad(r["prog"], r["theta"], r["coeffs"], r["codes"])
            else:
                t = srv.submit(r["prog"], r["shots"], seed=r["seed"])
            tickets[t] = r
            nxt += 1
        running, waiting = srv.step()
        ticks += 1
        now = time.perf_counter() - t0
        progressed = False
        for t in list(tickets):
            if srv.done(t):
                r = tickets.pop(t)
                results[r["id"]] = srv.fetch(t)
                lat[r["id"]] = now - r["arrival"]
                shots_done += r.get("shots", 0)
                progressed = True
        if backlog_at_window is None and now >= window:
            backlog_at_window = len(tickets) + (len(reqs) - nxt)
        if nxt == len(reqs) and not tickets:
            break
        if now > window + drain_limit_s:
            break
        if not progressed:
            # nothing finished: wait a little for the lanes or the next arrival
            nxt_t = reqs[nxt]["arrival"] - now if nxt < len(reqs) else 0.002
            time.sleep(max(0.0, min(0.0005, nxt_t)))
        if log and ticks % 2000 == 0:
            log(f"t={now:.1f}s submitted {nxt}/{len(reqs)} done {len(lat)} running {running} waiting {waiting}")
    elapsed = time.perf_counter() - t0
    prof = srv.profile() if profile else None
    srv.close()
    return {"latency": lat, "results": results, "elapsed": elapsed, "window": window, "ticks": ticks,
            "shots_done": shots_done, "completed": len(lat), "submitted": nxt,
            "backlog_at_window_end": backlog_at_window if backlog_at_window is not None else 0,
            "unfinished": len(tickets) + (len(reqs) - nxt), "profile": prof}
