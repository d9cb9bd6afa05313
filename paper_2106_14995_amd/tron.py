"""Python binding of the C ABI in include/tron.h (argument marshalling only).

Every step of a solve runs in the HIP library; this module checks tensor shapes and types,
passes raw device pointers and the torch stream, and turns error codes into exceptions.
There is no CPU fallback: if the library is not built, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

QP4, BR6, HS45M = 0, 1, 2
CONVERGED, MAX_ITER, STALLED, NONFINITE, BAD_BOUNDS = 0, 1, 2, 3, 4
FLAG_WARM = 1
ERRORS = {1: "invalid argument", 2: "out of memory", 3: "device error", 4: "unsupported",
          5: "busy"}


class TronError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Options(C.Structure):
    _fields_ = [("gtol", C.c_double), ("max_iter", C.c_int32), ("flags", C.c_uint32),
                ("cg_rtol", C.c_double), ("delta0", C.c_double)]


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
           "admm_destroy")


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


def options(gtol=1e-6, max_iter=500, cg_rtol=0.1, delta0=0.0, warm=False) -> Options:
    o = Options()
    lib().tron_default_options(C.byref(o))
    o.gtol, o.max_iter, o.cg_rtol, o.delta0 = gtol, max_iter, cg_rtol, delta0
    o.flags = FLAG_WARM if warm else 0
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
                 stream=None):
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
        _check(L.tron_batch_create(C.byref(self._h), self.family, self.batch, nptr, nuni,
                                   C.byref(o), _stream_ptr(stream)))

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
        try:
            self.close()
        except Exception:
            pass


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
        try:
            self.close()
        except Exception:
            pass
