"""Python binding of the C ABI in include/tron.h (argument marshalling only).

Every step of a solve runs in the HIP library; this module checks tensor shapes and types,
passes raw device pointers and the torch stream, and turns error codes into exceptions.
There is no CPU fallback: if the library is not built, loading it raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

from . import build as _build

QP4, BR6, HS45M, BR8L = 0, 1, 2, 3
CONVERGED, MAX_ITER, STALLED, NONFINITE, BAD_BOUNDS, AL_MAX_OUTER = 0, 1, 2, 3, 4, 5
FLAG_WARM = 1
FLAG_GRAPH = 2
ERRORS = {1: "invalid argument", 2: "out of memory", 3: "device error", 4: "unsupported",
          5: "busy"}


class TronError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Options(C.Structure):
    _fields_ = [("gtol", C.c_double), ("max_iter", C.c_int32), ("flags", C.c_uint32),
                ("cg_rtol", C.c_double), ("delta0", C.c_double)]


class AlOptions(C.Structure):
    _fields_ = [("ctol", C.c_double), ("outer_max", C.c_int32), ("rho_growth", C.c_double),
                ("decrease", C.c_double), ("rho_max", C.c_double)]


class PlanSpec(C.Structure):
    _fields_ = [("lane_max_n", C.c_int32), ("nedges", C.c_int32), ("edges", C.c_int32 * 16),
                ("streams", C.c_int32), ("lane_block", C.c_int32), ("pool_waves", C.c_int32),
                ("lane_group", C.c_int32), ("group16", C.c_int32), ("wave_global", C.c_int32)]

    def describe(self):
        return dict(lane_max_n=self.lane_max_n, edges=list(self.edges[:self.nedges]),
                    streams=self.streams, lane_block=self.lane_block, pool_waves=self.pool_waves,
                    lane_group=self.lane_group, group16=self.group16, wave_global=self.wave_global)


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("lds_budget", C.c_size_t), ("max_inflight", C.c_int32),
                ("streams", C.c_int32), ("coalesce", C.c_int32), ("max_group_instances", C.c_int32),
                ("opt", Options)]


class NetworkC(C.Structure):
    _fields_ = [("nbus", C.c_int32), ("nbranch", C.c_int32), ("ngen", C.c_int32),
                ("ref_bus", C.c_int32), ("rho", C.c_double), ("base_mva", C.c_double),
                ("br_from", C.c_void_p), ("br_to", C.c_void_p), ("br_adm", C.c_void_p),
                ("br_lo", C.c_void_p), ("br_hi", C.c_void_p), ("gen_bus", C.c_void_p),
                ("gen_cost", C.c_void_p), ("gen_lim", C.c_void_p), ("bus_load", C.c_void_p)]


_lib = None
EXPORTS = ("tron_default_options", "tron_last_error", "tron_param_size", "tron_batch_create",
           "tron_batch_solve", "tron_batch_get_state", "tron_batch_set_state",
           "tron_batch_set_options", "tron_batch_plan", "tron_batch_destroy",
           "admm_state_size", "admm_create", "admm_step", "admm_get_state", "admm_set_state",
           "admm_destroy", "tron_server_default_config", "tron_server_create", "tron_server_submit",
           "tron_server_poll", "tron_server_wait", "tron_server_result", "tron_server_close_session",
           "tron_server_cancel",
           "tron_server_stats", "tron_server_destroy", "tron_batch_set_timestamps", "tron_clock_rate_hz",
           "tron_default_plan_spec", "tron_batch_create_ex", "tron_autotune",
           "tron_default_al_options", "tron_al_solve", "tron_design_chol", "tron_design_trsv",
           "tron_design_fma_peak",
           "tron_solve_noalloc", "tron_noalloc_scratch_bytes")
CHOL_LEFT_LDS, CHOL_RIGHT_LDS, CHOL_LEFT_GLOBAL, CHOL_BLOCKED_MFMA = 0, 1, 2, 3
TRSV_IMPLICIT, TRSV_PADDED, TRSV_EXPLICIT, TRSV_GLOBAL = 0, 1, 2, 3


# Handles still open when the interpreter exits are closed by an exit hook, which runs
# before the HIP runtime's own teardown; destructors that run later (during module
# teardown) then do nothing instead of calling into a runtime that may be gone.
_live = weakref.WeakSet()
_at_exit = False


def _close_all():
    global _at_exit
    for h in list(_live):
        try:
            h.close()
        except Exception:
            pass
    _at_exit = True


atexit.register(_close_all)


def lib_path() -> str:
    return _build.LIB


def lib():
    """Open the HIP library (built by paper_2106_14995_amd.build / __graft_entry__.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise RuntimeError(f"HIP library missing at {_build.LIB}: run __graft_entry__.build()")
        L = C.CDLL(_build.LIB)
        P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
        L.tron_last_error.restype = C.c_char_p
        L.tron_last_error.argtypes = []
        L.tron_default_options.argtypes = [C.POINTER(Options)]
        L.tron_param_size.restype = I64
        L.tron_param_size.argtypes = [I32, I32]
        L.tron_batch_create.argtypes = [C.POINTER(P), I32, I64, P, I32, C.POINTER(Options), P]
        L.tron_batch_solve.argtypes = [P] * 10
        L.tron_batch_get_state.argtypes = [P, P, P]
        L.tron_batch_set_state.argtypes = [P, P, P]
        L.tron_batch_set_options.argtypes = [P, C.POINTER(Options)]
        L.tron_batch_plan.argtypes = [P, P, P, I32]
        L.tron_batch_destroy.argtypes = [P]
        L.tron_default_plan_spec.argtypes = [C.POINTER(PlanSpec)]
        L.tron_batch_create_ex.argtypes = [C.POINTER(P), I32, I64, P, I32, C.POINTER(Options),
                                           C.POINTER(PlanSpec), P]
        L.tron_autotune.argtypes = [I32, I64, P, P, P, P, P, P, P, P, P, I32, C.c_char_p,
                                    C.POINTER(PlanSpec), C.POINTER(C.c_double), P]
        L.tron_default_al_options.argtypes = [C.POINTER(AlOptions)]
        L.tron_al_solve.argtypes = [P, C.POINTER(AlOptions)] + [P] * 11
        L.tron_design_chol.argtypes = [I32, I64, I32, P, P, P, P]
        L.tron_design_trsv.argtypes = [I32, I64, I32, P, P, P, I32, P]
        L.tron_design_fma_peak.argtypes = [I64, I32, P, P]
        L.tron_clock_rate_hz.restype = I64
        L.tron_clock_rate_hz.argtypes = []
        L.tron_solve_noalloc.argtypes = [I32, I64, I32, C.POINTER(Options)] + [P] * 9
        L.tron_noalloc_scratch_bytes.restype = I64
        L.tron_noalloc_scratch_bytes.argtypes = []
        L.tron_batch_set_timestamps.argtypes = [P, P]
        L.tron_server_default_config.argtypes = [C.POINTER(ServerConfig)]
        L.tron_server_create.argtypes = [C.POINTER(P), I32, C.POINTER(ServerConfig)]
        L.tron_server_submit.argtypes = [P, I64, P, P, P, P, P, C.c_uint64, C.POINTER(I64)]
        L.tron_server_poll.argtypes = [P, I64, C.POINTER(I32)]
        L.tron_server_wait.argtypes = [P, I64, C.c_double]
        L.tron_server_result.argtypes = [P, I64, P, P, P, P, C.POINTER(C.c_double)]
        L.tron_server_close_session.argtypes = [P, C.c_uint64]
        L.tron_server_cancel.argtypes = [P, I64]
        L.tron_server_stats.argtypes = [P, P]
        L.tron_server_destroy.argtypes = [P]
        if hasattr(L, "admm_state_size"):
            L.admm_state_size.restype = I64
            L.admm_state_size.argtypes = [C.POINTER(NetworkC)]
            L.admm_create.argtypes = [C.POINTER(P), C.POINTER(NetworkC), C.POINTER(Options), P]
            L.admm_step.argtypes = [P, I32, P, P]
            L.admm_get_state.argtypes = [P, P, I64, P]
            L.admm_set_state.argtypes = [P, P, I64, P]
            L.admm_destroy.argtypes = [P]
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise TronError(rc, lib().tron_last_error().decode())


def options(gtol=1e-6, max_iter=500, cg_rtol=0.1, delta0=0.0, warm=False, graph=False) -> Options:
    o = Options()
    lib().tron_default_options(C.byref(o))
    o.gtol, o.max_iter, o.cg_rtol, o.delta0 = gtol, max_iter, cg_rtol, delta0
    o.flags = (FLAG_WARM if warm else 0) | (FLAG_GRAPH if graph else 0)
    return o


def param_size(family: int, n: int) -> int:
    return int(lib().tron_param_size(family, n))


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype, numel, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")
    return C.c_void_p(t.data_ptr())


class Batch:
    """A tron_batch handle: `batch` instances of `family` with sizes `n` (int or array)."""

    def __init__(self, family: int, n, batch: int | None = None, opts: Options | None = None,
                 stream=None, spec: "PlanSpec | None" = None):
        L = lib()
        if np.isscalar(n):
            if batch is None:
                raise ValueError("batch is required with a uniform n")
            self.n = np.full(int(batch), int(n), dtype=np.int32)
            nptr, nuni = None, int(n)
        else:
            self.n = np.ascontiguousarray(n, dtype=np.int32)
            nptr, nuni = self.n.ctypes.data_as(C.c_void_p), 0
        self.family = int(family)
        self.batch = int(self.n.shape[0])
        self.nsum = int(self.n.astype(np.int64).sum())
        vals, cnts = np.unique(self.n, return_counts=True)
        self.psum = int(sum(param_size(family, int(v)) * int(c) for v, c in zip(vals, cnts)))
        self._h = C.c_void_p()
        o = opts if opts is not None else options()
        _check(L.tron_batch_create_ex(C.byref(self._h), self.family, self.batch, nptr, nuni,
                                      C.byref(o), C.byref(spec) if spec is not None else None,
                                      _stream_ptr(stream)))
        _live.add(self)

    def solve(self, params, lo, hi, x0, x=None, f=None, status=None, iters=None, stream=None):
        import torch
        dev = lo.device
        if x is None:
            x = torch.empty(self.nsum, dtype=torch.float64, device=dev)
        if f is None:
            f = torch.empty(self.batch, dtype=torch.float64, device=dev)
        if status is None:
            status = torch.empty(self.batch, dtype=torch.int32, device=dev)
        if iters is None:
            iters = torch.empty(self.batch, dtype=torch.int32, device=dev)
        f64, i32 = torch.float64, torch.int32
        pp = _dev(params, f64, self.psum, "params") if self.psum else C.c_void_p(
            params.data_ptr() if params is not None and params.numel() else 0)
        args = [pp, _dev(lo, f64, self.nsum, "lo"), _dev(hi, f64, self.nsum, "hi"),
                _dev(x0, f64, self.nsum, "x0"), _dev(x, f64, self.nsum, "x"),
                _dev(f, f64, self.batch, "f"), _dev(status, i32, self.batch, "status"),
                _dev(iters, i32, self.batch, "iters")]
        _check(lib().tron_batch_solve(self._h, *args, _stream_ptr(stream)))
        return x, f, status, iters

    def al_solve(self, params, lo, hi, x0, ctol=1e-6, outer_max=50, rho_growth=10.0,
                 decrease=0.25, rho_max=1e6, x=None, stream=None):
        """Multiplier loop on a BR8L batch; `params` (device, batch x 40) is updated in place.
        Returns x, f, status, iters, outer, viol (device tensors)."""
        import torch
        dev = lo.device
        f64, i32 = torch.float64, torch.int32
        if x is None:
            x = torch.empty(self.nsum, dtype=f64, device=dev)
        f = torch.empty(self.batch, dtype=f64, device=dev)
        viol = torch.empty(self.batch, dtype=f64, device=dev)
        status, iters, outer = (torch.empty(self.batch, dtype=i32, device=dev) for _ in range(3))
        o = AlOptions()
        lib().tron_default_al_options(C.byref(o))
        o.ctol, o.outer_max, o.rho_growth, o.decrease, o.rho_max = ctol, outer_max, rho_growth, decrease, rho_max
        _check(lib().tron_al_solve(self._h, C.byref(o), _dev(params, f64, self.psum, "params"),
                                   _dev(lo, f64, self.nsum, "lo"), _dev(hi, f64, self.nsum, "hi"),
                                   _dev(x0, f64, self.nsum, "x0"), _dev(x, f64, self.nsum, "x"),
                                   _dev(f, f64, self.batch, "f"), _dev(status, i32, self.batch, "status"),
                                   _dev(iters, i32, self.batch, "iters"), _dev(outer, i32, self.batch, "outer"),
                                   _dev(viol, f64, self.batch, "viol"), _stream_ptr(stream)))
        return x, f, status, iters, outer, viol

    def get_state(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(2 * self.batch, dtype=torch.float64, device="cuda")
        _check(lib().tron_batch_get_state(self._h, _dev(out, torch.float64, 2 * self.batch, "state"),
                                          _stream_ptr(stream)))
        return out

    def set_state(self, state, stream=None):
        import torch
        _check(lib().tron_batch_set_state(self._h, _dev(state, torch.float64, 2 * self.batch, "state"),
                                          _stream_ptr(stream)))

    def set_options(self, opts: Options):
        _check(lib().tron_batch_set_options(self._h, C.byref(opts)))

    def plan(self):
        nb = C.c_int32()
        desc = (C.c_int32 * (3 * 256))()
        _check(lib().tron_batch_plan(self._h, C.byref(nb), desc, 256))
        return [dict(nmax=desc[3 * i], lanes=desc[3 * i + 1], count=desc[3 * i + 2])
                for i in range(min(nb.value, 256))]

    def close(self):
        if self._h:
            lib().tron_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        if _at_exit:
            return
        try:
            self.close()
        except Exception:
            pass


def solve_noalloc(family, n, batch, params, lo, hi, x0, x=None, f=None, status=None, iters=None,
                  opts: Options | None = None, stream=None):
    """tron_solve_noalloc: one cold-start solve of `batch` instances of uniform size n whose
    working memory is the library's fixed device array (no device allocation in the call).
    Outputs not passed in are allocated here by torch."""
    import torch
    dev = lo.device
    nsum = int(batch) * int(n)
    f64, i32 = torch.float64, torch.int32
    if x is None:
        x = torch.empty(nsum, dtype=f64, device=dev)
    if f is None:
        f = torch.empty(batch, dtype=f64, device=dev)
    if status is None:
        status = torch.empty(batch, dtype=i32, device=dev)
    if iters is None:
        iters = torch.empty(batch, dtype=i32, device=dev)
    psum = param_size(family, n) * int(batch)
    pp = _dev(params, f64, psum, "params") if psum > 0 else C.c_void_p(0)
    _check(lib().tron_solve_noalloc(int(family), int(batch), int(n), C.byref(opts) if opts is not None else None,
                                    pp, _dev(lo, f64, nsum, "lo"), _dev(hi, f64, nsum, "hi"),
                                    _dev(x0, f64, nsum, "x0"), _dev(x, f64, nsum, "x"),
                                    _dev(f, f64, batch, "f"), _dev(status, i32, batch, "status"),
                                    _dev(iters, i32, batch, "iters"), _stream_ptr(stream)))
    return x, f, status, iters


def design_chol(variant, a, l=None, info=None, stream=None):
    """Batched Cholesky of a (count, n, n) float64 device tensor of SPD blocks, in one of the
    design variants of include/tron_design.h. Returns (L, info)."""
    import torch
    count, n = int(a.shape[0]), int(a.shape[1])
    if l is None:
        l = torch.empty_like(a)
    if info is None:
        info = torch.empty(count, dtype=torch.int32, device=a.device)
    _check(lib().tron_design_chol(variant, count, n, _dev(a, torch.float64, count * n * n, "a"),
                                  _dev(l, torch.float64, count * n * n, "l"),
                                  _dev(info, torch.int32, count, "info"), _stream_ptr(stream)))
    return l, info


def design_trsv(variant, l, b, x=None, reps=1, stream=None):
    """Solve L L^T x = b for (count, n, n) factors and (count, n) right-hand sides."""
    import torch
    count, n = int(l.shape[0]), int(l.shape[1])
    if x is None:
        x = torch.empty_like(b)
    _check(lib().tron_design_trsv(variant, count, n, _dev(l, torch.float64, count * n * n, "l"),
                                  _dev(b, torch.float64, count * n, "b"), _dev(x, torch.float64, count * n, "x"),
                                  reps, _stream_ptr(stream)))
    return x


def design_fma_peak(blocks, iters, sink=None, stream=None):
    """tron_design_fma_peak: one launch of the FP64 FMA-rate kernel (blocks x 256 lanes, 8 chains
    of `iters` fused multiply-adds each); returns the per-lane sums. Flops issued:
    blocks x 256 x 8 x iters x 2."""
    import torch
    if sink is None:
        sink = torch.empty(int(blocks) * 256, dtype=torch.float64, device="cuda")
    _check(lib().tron_design_fma_peak(int(blocks), int(iters), _dev(sink, torch.float64, int(blocks) * 256, "sink"),
                                      _stream_ptr(stream)))
    return sink


def to_device(batch, device="cuda"):
    """Move a workloads.Batch's arrays to the GPU as float64 tensors."""
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)
    return t(batch.params), t(batch.lo), t(batch.hi), t(batch.x0)


class Admm:
    """An admm handle over a workloads.Network (host arrays are copied at creation)."""

    def __init__(self, net, branch_opts: Options | None = None, stream=None):
        L = lib()
        keep = [np.ascontiguousarray(a) for a in (net.br_from, net.br_to, net.br_adm, net.br_lo,
                                                    net.br_hi, net.gen_bus, net.gen_cost,
                                                    net.gen_lim, net.bus_load)]
        self._net = NetworkC(net.nbus, net.nbranch, net.ngen, net.ref_bus, net.rho, net.base_mva,
                             *[a.ctypes.data_as(C.c_void_p) for a in keep])
        self.state_size = int(L.admm_state_size(C.byref(self._net)))
        self._h = C.c_void_p()
        o = branch_opts if branch_opts is not None else options()
        _check(L.admm_create(C.byref(self._h), C.byref(self._net), C.byref(o), _stream_ptr(stream)))
        _live.add(self)
        del keep

    def step(self, iters: int, resid=None, stream=None):
        import torch
        if resid is None:
            resid = torch.empty(2 * max(iters, 1), dtype=torch.float64, device="cuda")
        _check(lib().admm_step(self._h, iters, _dev(resid, torch.float64, 2 * iters, "resid"),
                               _stream_ptr(stream)))
        return resid[:2 * iters].view(iters, 2) if iters else resid[:0]

    def get_state(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(self.state_size, dtype=torch.float64, device="cuda")
        _check(lib().admm_get_state(self._h, _dev(out, torch.float64, self.state_size, "state"),
                                    self.state_size, _stream_ptr(stream)))
        return out

    def set_state(self, state, stream=None):
        import torch
        _check(lib().admm_set_state(self._h, _dev(state, torch.float64, self.state_size, "state"),
                                    self.state_size, _stream_ptr(stream)))

    def close(self):
        if self._h:
            lib().admm_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        if _at_exit:
            return
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A tron_server: continuous batching of solve requests given as host arrays."""

    def __init__(self, family: int, hbm_budget=1 << 30, lds_budget=None, max_inflight=8, streams=4,
                 coalesce=True, max_group_instances=65536, opts: Options | None = None):
        L = lib()
        cfg = ServerConfig()
        L.tron_server_default_config(C.byref(cfg))
        cfg.hbm_budget = int(hbm_budget)
        if lds_budget is not None:
            cfg.lds_budget = int(lds_budget)
        cfg.max_inflight, cfg.streams = int(max_inflight), int(streams)
        cfg.coalesce, cfg.max_group_instances = int(bool(coalesce)), int(max_group_instances)
        if opts is not None:
            cfg.opt = opts
        self.family = int(family)
        self._h = C.c_void_p()
        self._sizes = {}
        _check(L.tron_server_create(C.byref(self._h), self.family, C.byref(cfg)))
        _live.add(self)

    def submit(self, n, params, lo, hi, x0=None, session=0) -> int:
        n = np.ascontiguousarray(n, dtype=np.int32)
        arr = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
        params, lo, hi, x0 = arr(params), arr(lo), arr(hi), arr(x0)
        p = lambda a: None if a is None or a.size == 0 else a.ctypes.data_as(C.c_void_p)
        t = C.c_int64()
        _check(lib().tron_server_submit(self._h, int(n.shape[0]), n.ctypes.data_as(C.c_void_p),
                                        p(params), p(lo), p(hi), p(x0), C.c_uint64(session), C.byref(t)))
        self._sizes[t.value] = (int(n.shape[0]), int(n.astype(np.int64).sum()))
        return t.value

    def submit_batch(self, batch, x0=True, session=0) -> int:
        return self.submit(batch.n, batch.params, batch.lo, batch.hi, batch.x0 if x0 else None, session)

    def poll(self, ticket) -> int:
        st = C.c_int32()
        _check(lib().tron_server_poll(self._h, ticket, C.byref(st)))
        return st.value

    def wait(self, ticket, timeout=-1.0):
        _check(lib().tron_server_wait(self._h, ticket, float(timeout)))

    def result(self, ticket):
        B, nsum = self._sizes.get(ticket, (0, 0))
        x = np.empty(nsum); f = np.empty(B)
        st = np.empty(B, dtype=np.int32); it = np.empty(B, dtype=np.int32)
        lat = C.c_double()
        p = lambda a: a.ctypes.data_as(C.c_void_p)
        try:
            _check(lib().tron_server_result(self._h, ticket, p(x), p(f), p(st), p(it), C.byref(lat)))
        except TronError as e:
            if "not finished" not in str(e):  # the library released the ticket
                self._sizes.pop(ticket, None)
            raise
        self._sizes.pop(ticket, None)
        return dict(x=x, f=f, status=st, iters=it, latency=lat.value)

    def cancel(self, ticket):
        """Take a queued request off the queue (TronError BUSY if it already reached the
        device); its result call then raises with the cancellation."""
        _check(lib().tron_server_cancel(self._h, ticket))

    def close_session(self, session):
        _check(lib().tron_server_close_session(self._h, C.c_uint64(session)))

    def stats(self):
        out = np.zeros(4, dtype=np.int64)
        _check(lib().tron_server_stats(self._h, out.ctypes.data_as(C.c_void_p)))
        return dict(requests=int(out[0]), instances=int(out[1]), device_bytes=int(out[2]),
                    lds_inflight=int(out[3]))

    def close(self):
        if self._h:
            lib().tron_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        if _at_exit:
            return
        try:
            self.close()
        except Exception:
            pass


DEFAULT_EDGES = (16, 24, 32, 40, 48, 56, 64, 80, 96, 112, 128)


def plan_spec(lane_max_n=8, edges=DEFAULT_EDGES, streams=4, lane_block=64, pool_waves=12,
              lane_group=0, group16=0, wave_global=0) -> PlanSpec:
    """A launch plan (the defaults are the library's default plan); pool_waves 8 or 12 selects
    the persistent launch for batches of mixed sizes up to n = 128 (0: the buckets); lane_group 1/2/4/8 puts each instance with n <= lane_max_n on that
    many lanes (0: automatic, 8 for uniform quartic batches of n = 7 or 8 up to 16,384
    instances, else 1); group16 8/16 puts lane_max_n < n <= 16 on groups of that width; wave_global 1
    keeps the quartic family's wavefront matrices in global memory instead of LDS."""
    p = PlanSpec()
    p.lane_max_n, p.nedges, p.streams, p.lane_block = lane_max_n, len(edges), streams, lane_block
    p.pool_waves, p.lane_group, p.group16, p.wave_global = pool_waves, lane_group, group16, wave_global
    for i, e in enumerate(edges):
        p.edges[i] = int(e)
    return p


def autotune(family, n, params, lo, hi, x0, x, f, status, iters, reps=3, cache_path=None,
             stream=None):
    """Time candidate plans on this batch (the C autotuner) and return (PlanSpec, ms per
    solve; -1 when read from the cache)."""
    import torch
    n = np.ascontiguousarray(n, dtype=np.int32)
    best = PlanSpec()
    ms = C.c_double()
    ptr = lambda t: C.c_void_p(t.data_ptr()) if t is not None and t.numel() else None
    _check(lib().tron_autotune(family, int(n.shape[0]), n.ctypes.data_as(C.c_void_p), ptr(params),
                               ptr(lo), ptr(hi), ptr(x0), ptr(x), ptr(f), ptr(status), ptr(iters),
                               int(reps), cache_path.encode() if cache_path else None,
                               C.byref(best), C.byref(ms), _stream_ptr(stream)))
    return best, ms.value
