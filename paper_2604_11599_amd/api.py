"""Python binding of libqsv with the C ABI's names (argument marshalling only)."""
import ctypes as C
import weakref

import numpy as np

from . import _abi as A
from .lower import LoweredProgram, lower


class QsvError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{A.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _desc(lp):
    instr = np.ascontiguousarray(lp.instr)
    pred = np.ascontiguousarray(lp.pred)
    code = np.ascontiguousarray(lp.code)
    lin = np.ascontiguousarray(lp.lin)
    noise = np.ascontiguousarray(lp.noise)
    d = A.ProgramDesc(lp.n_qubits, lp.n_clbits, lp.n_params, len(instr), len(pred), 0,
                      instr.ctypes.data if len(instr) else None, pred.ctypes.data if len(pred) else None,
                      len(code), 0, code.ctypes.data if len(code) else None,
                      len(lin), lp.n_derived, lin.ctypes.data if len(lin) else None,
                      len(noise), 0, noise.ctypes.data if len(noise) else None)
    return d, (instr, pred, code, lin, noise)


def plan_inspect(source, tile_bits=0):
    """Host-only planner statistics (no GPU needed)."""
    lp = source if isinstance(source, LoweredProgram) else lower(source)
    d, keep = _desc(lp)
    st = A.PlanStats()
    rc = A.lib().qsv_plan_inspect(C.byref(d), tile_bits, C.byref(st))
    if rc:
        raise QsvError(rc, "planning failed")
    return st


class Context:
    """qsv_create / qsv_destroy. `stream` may be a torch.cuda.Stream or a raw hipStream_t;
    a stream whose handle is 0 (torch's default stream) is the device's null stream."""

    def __init__(self, device=0, stream=None, arena=None, arena_bytes=0, device_ptrs=False, profile=False,
                 tuned_plans=False):
        raw = None
        flags = (A.QSV_FLAG_DEVICE_PTRS if device_ptrs else 0) | (A.QSV_FLAG_PROFILE if profile else 0)
        flags |= A.QSV_FLAG_TUNED_PLANS if tuned_plans else 0
        if stream is not None:
            raw = int(getattr(stream, "cuda_stream", stream) or 0)
            if raw == 0:
                flags |= A.QSV_FLAG_NULL_STREAM
        # the stream the library orders its work on (None: its own)
        self.stream_handle = raw
        self._forks = []
        cfg = A.Config(device, raw or None, arena, arena_bytes, flags)
        h = C.c_void_p()
        rc = A.lib().qsv_create(C.byref(cfg), C.byref(h))
        if rc:
            raise QsvError(rc, "qsv_create failed")
        self.handle = h
        self.device_ptrs = device_ptrs
        self._programs = weakref.WeakSet()

    def close(self):
        """Frees the context's forks and programs that are still alive, then the
        context (a program must not outlive its context)."""
        if self.handle:
            for f in getattr(self, "_forks", []):
                f.close()
            self._forks = []
            for p in list(self._programs):
                p.free()
            A.lib().qsv_destroy(self.handle)
            self.handle = None

    def fork(self):
        """qsv_context_fork: a context of the same family with its own stream and
        scratch (for another host thread); closed with this context."""
        h = C.c_void_p()
        self.check(A.lib().qsv_context_fork(self.handle, C.byref(h)))
        f = Context.__new__(Context)
        f.handle, f.device_ptrs, f.stream_handle = h, self.device_ptrs, None
        f._programs, f._forks = weakref.WeakSet(), []
        self._forks.append(f)
        return f

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        msg = A.lib().qsv_last_error(self.handle)
        return msg.decode() if msg else ""

    def check(self, rc):
        if rc:
            raise QsvError(rc, self.last_error())

    def profile(self):
        """qsv_profile_read as a dict (context created with profile=True)."""
        p = A.Profile()
        self.check(A.lib().qsv_profile_read(self.handle, C.byref(p)))
        return {k: getattr(p, k) for k, _ in A.Profile._fields_}

    def profile_reset(self):
        self.check(A.lib().qsv_profile_reset(self.handle))

    def load(self, source, noise=False):
        """qsv_load_program on OpenQASM 3 text or a LoweredProgram. noise: lower
        the text with depolarizing slots (run_shots(depolarizing=p) sets their rate)."""
        return Program(self, lower(source, noise=True) if noise and isinstance(source, str) else source)

    def tune_lookup(self, n_qubits, complex64=False):
        """qsv_tune_lookup: the cached plan options for n_qubits, or None."""
        o, f = A.PlanOptions(), C.c_int32()
        self.check(A.lib().qsv_tune_lookup(self.handle, n_qubits, A.QSV_RUN_COMPLEX64 if complex64 else 0,
                                           C.byref(o), C.byref(f)))
        return _opts_dict(o) if f.value else None

    def run_batch(self, requests):
        """qsv_run_batch: every shot of every request in one persistent launch.

        requests: iterable of dicts with keys prog, shots and optionally theta,
        seed, shot_offset, forced, readout_error, reset_error. Returns one ShotResultArrays per request."""
        reqs = list(requests)
        arr = (A.Request * max(1, len(reqs)))()
        keep, results = [], []
        for i, rq in enumerate(reqs):
            prog, n = rq["prog"], int(rq["shots"])
            bufs = prog._result_buffers(n)
            th = prog._theta(rq.get("theta")) if prog.info.n_params else None
            f, flen = prog._forced(rq.get("forced"), n)
            keep += [th, f, bufs]
            arr[i].prog = prog.handle
            arr[i].theta = None if th is None else th.ctypes.data
            arr[i].n_shots = n
            arr[i].opts = A.RunOpts(int(rq.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF, int(rq.get("shot_offset", 0)),
                                    _ptr(f), flen, 0, None, float(rq.get("readout_error", 0.0)),
                                    float(rq.get("reset_error", 0.0)))
            arr[i].out = A.ShotResults(*[_ptr(b) for b in bufs])
            results.append(bufs)
        self.check(A.lib().qsv_run_batch(self.handle, arr, len(reqs)))
        out = []
        for rq, (creg, record, nev, prob, status) in zip(reqs, results):
            mr = rq["prog"].info.max_events
            out.append(ShotResultArrays(creg, record[:, :mr], nev, prob, status, None, rq["prog"].lowered.n_clbits))
        return out


def _opts_dict(o):
    return {"tile_bits": o.tile_bits, "low_bits": o.low_bits, "dense_min_cost": o.dense_min_cost}


class ShotResultArrays:
    def __init__(self, creg, record, n_events, record_prob, shot_status, state, n_clbits):
        self.creg, self.record, self.n_events = creg, record, n_events
        self.record_prob, self.shot_status, self.state = record_prob, shot_status, state
        self.n_clbits = n_clbits

    def bits(self):
        """Classical bits as an [n_shots, n_clbits] uint8 array."""
        out = np.zeros((self.creg.shape[0], self.n_clbits), dtype=np.uint8)
        for i in range(self.n_clbits):
            out[:, i] = (self.creg[:, i // 64] >> np.uint64(i % 64)) & np.uint64(1)
        return out


class Program:
    def __init__(self, ctx, source):
        self.ctx = ctx
        self.lowered = source if isinstance(source, LoweredProgram) else lower(source)
        d, keep = _desc(self.lowered)
        h = C.c_void_p()
        ctx.check(A.lib().qsv_load_program(ctx.handle, C.byref(d), C.byref(h)))
        self.handle = h
        ctx._programs.add(self)
        info = A.ProgramInfo()
        A.lib().qsv_program_info_get(h, C.byref(info))
        self.info = info

    def free(self):
        if self.handle:
            if self.ctx.handle:
                A.lib().qsv_program_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def n_qubits(self):
        return self.info.n_qubits

    def plan_options(self):
        """qsv_program_plan_get as a dict."""
        o = A.PlanOptions()
        self.ctx.check(A.lib().qsv_program_plan_get(self.handle, C.byref(o)))
        return _opts_dict(o)

    def replan(self, tile_bits, low_bits, dense_min_cost):
        """qsv_program_replan with explicit planner options."""
        o = A.PlanOptions(tile_bits, low_bits, dense_min_cost)
        self.ctx.check(A.lib().qsv_program_replan(self.ctx.handle, self.handle, C.byref(o)))
        self._refresh_info()

    def autotune(self, n_shots, theta=None, share=False, complex64=False):
        """qsv_autotune: measures candidate plans on this call shape, installs the
        fastest; returns the report as a dict."""
        th = self._theta(theta if theta is not None else np.zeros(self.info.n_params))
        r = A.TuneReport()
        flags = (A.QSV_RUN_SHARE_TRAJ if share else 0) | (A.QSV_RUN_COMPLEX64 if complex64 else 0)
        self.ctx.check(A.lib().qsv_autotune(self.ctx.handle, self.handle, _ptr(th), int(n_shots), flags,
                                            C.byref(r)))
        self._refresh_info()
        return {"best": _opts_dict(r.best), "default": _opts_dict(r.deflt), "best_ms": r.best_ms,
                "default_ms": r.default_ms, "n_candidates": r.n_candidates, "arch": r.arch.decode()}

    def _refresh_info(self):
        info = A.ProgramInfo()
        A.lib().qsv_program_info_get(self.handle, C.byref(info))
        self.info = info

    def _theta(self, theta, batch=None):
        p = self.info.n_params
        if p == 0:
            return np.zeros(max(1, batch or 1) * 1, dtype=np.float64)
        t = np.ascontiguousarray(theta, dtype=np.float64)
        if batch is None:
            if t.size != p:
                raise ValueError(f"theta must hold {p} values")
        elif t.size != p * batch:
            raise ValueError(f"theta must be [{batch}, {p}]")
        return t

    def _result_buffers(self, n_shots):
        cw = max(1, (self.lowered.n_clbits + 63) // 64)
        return (np.zeros((n_shots, cw), dtype=np.uint64),
                np.zeros((n_shots, max(1, self.info.max_events)), dtype=np.uint8),
                np.zeros(n_shots, dtype=np.uint32), np.zeros(n_shots, dtype=np.float64),
                np.zeros(n_shots, dtype=np.int32))

    def _forced(self, forced, n_shots):
        if forced is None:
            return None, 0
        f = np.ascontiguousarray(forced, dtype=np.uint8)
        if f.ndim == 1:
            f = np.broadcast_to(f, (n_shots, f.size)).copy()
        if f.shape[0] != n_shots:
            raise ValueError("forced must have one row per shot")
        return f, f.shape[1]

    def run_shots(self, n_shots, theta=None, seed=0, shot_offset=0, forced=None, state_out=False,
                  share=False, readout_error=0.0, reset_error=0.0, complex64=False, noalloc=False, graph=False,
                  depolarizing=0.0):
        """qsv_run_shots: returns host arrays of classical bits, records, probabilities, statuses.
        complex64: hold and evolve the state in single precision (QSV_RUN_COMPLEX64).
        depolarizing: rate of the program's noise slots (a program loaded with noise=True).
        noalloc: call qsv_run_shots_noalloc (device scratch from the library's fixed array).
        graph: capture the call's launch sequence in a HIP graph and replay it (QSV_RUN_GRAPH)."""
        lp = self.lowered
        cw = max(1, (lp.n_clbits + 63) // 64)
        mr = self.info.max_events
        creg = np.zeros((n_shots, cw), dtype=np.uint64)
        record = np.zeros((n_shots, max(1, mr)), dtype=np.uint8)
        nev = np.zeros(n_shots, dtype=np.uint32)
        prob = np.zeros(n_shots, dtype=np.float64)
        status = np.zeros(n_shots, dtype=np.int32)
        if theta is None and self.info.n_params:
            raise ValueError(f"this program takes {self.info.n_params} input parameters")
        th = self._theta(theta if theta is not None else np.zeros(self.info.n_params))
        f = None
        flen = 0
        if forced is not None:
            f = np.ascontiguousarray(forced, dtype=np.uint8)
            if f.ndim == 1:
                f = np.broadcast_to(f, (n_shots, f.size)).copy()
            if f.shape[0] != n_shots:
                raise ValueError("forced must have one row per shot")
            flen = f.shape[1]
        st = np.zeros((1 << lp.n_qubits, 2), dtype=np.float64) if state_out else None
        opts = A.RunOpts(seed & 0xFFFFFFFFFFFFFFFF, shot_offset, _ptr(f), flen,
                         (A.QSV_RUN_SHARE_TRAJ if share else 0) | (A.QSV_RUN_COMPLEX64 if complex64 else 0)
                         | (A.QSV_RUN_GRAPH if graph else 0), _ptr(st),
                         float(readout_error), float(reset_error), float(depolarizing))
        res = A.ShotResults(_ptr(creg), _ptr(record) if mr else None, _ptr(nev), _ptr(prob), _ptr(status))
        fn = A.lib().qsv_run_shots_noalloc if noalloc else A.lib().qsv_run_shots
        self.ctx.check(fn(self.ctx.handle, self.handle, _ptr(th), n_shots, C.byref(opts), C.byref(res)))
        state = None if st is None else st.view(np.complex128).reshape(-1)
        return ShotResultArrays(creg, record[:, :mr], nev, prob, status, state, lp.n_clbits)

    def _pauli(self, coeffs, codes):
        c = np.ascontiguousarray(coeffs, dtype=np.float64)
        k = np.ascontiguousarray(codes, dtype=np.uint8).reshape(len(c), self.info.n_qubits)
        return A.PauliSum(len(c), 0, _ptr(c), _ptr(k)), (c, k)

    def expval(self, thetas, coeffs, codes):
        """qsv_expval over a batch of parameter vectors thetas[B, P] (host arrays)."""
        th = np.atleast_2d(np.asarray(thetas, dtype=np.float64))
        b = th.shape[0] if self.info.n_params else max(1, th.shape[0])
        th = self._theta(th, b)
        h, keep = self._pauli(coeffs, codes)
        e = np.zeros(b, dtype=np.float64)
        self.ctx.check(A.lib().qsv_expval(self.ctx.handle, self.handle, _ptr(th), b, C.byref(h), _ptr(e)))
        return e

    def expval_grad(self, thetas, coeffs, codes):
        """qsv_expval_grad: energies [B] and gradients [B, P]."""
        th = np.atleast_2d(np.asarray(thetas, dtype=np.float64))
        b = th.shape[0]
        th = self._theta(th, b)
        h, keep = self._pauli(coeffs, codes)
        e = np.zeros(b, dtype=np.float64)
        g = np.zeros((b, max(1, self.info.n_params)), dtype=np.float64)
        self.ctx.check(A.lib().qsv_expval_grad(self.ctx.handle, self.handle, _ptr(th), b, C.byref(h),
                                               _ptr(e), _ptr(g)))
        return e, g[:, :self.info.n_params]

    def expval_grad_each(self, thetas, hamiltonians):
        """qsv_expval_grad_each: thetas [B, P] with one Hamiltonian (coeffs, codes) per row."""
        th = np.atleast_2d(np.asarray(thetas, dtype=np.float64))
        b = th.shape[0]
        th = self._theta(th, b)
        if len(hamiltonians) != b:
            raise ValueError("one Hamiltonian per parameter vector")
        hs = (A.PauliSum * b)()
        keep = []
        for k, (coeffs, codes) in enumerate(hamiltonians):
            h, kp = self._pauli(coeffs, codes)
            hs[k] = h
            keep.append(kp)
        e = np.zeros(b, dtype=np.float64)
        g = np.zeros((b, max(1, self.info.n_params)), dtype=np.float64)
        self.ctx.check(A.lib().qsv_expval_grad_each(self.ctx.handle, self.handle, _ptr(th), b, hs, _ptr(e),
                                                    _ptr(g)))
        return e, g[:, :self.info.n_params]

    def expval_grad_device(self, theta_ptr, batch, pauli_sum, energy_ptr, grad_ptr):
        """qsv_expval_grad with device pointers (context created with device_ptrs=True)."""
        self.ctx.check(A.lib().qsv_expval_grad(self.ctx.handle, self.handle, C.c_void_p(theta_ptr), batch,
                                               C.byref(pauli_sum), C.c_void_p(energy_ptr),
                                               C.c_void_p(grad_ptr)))
