"""ctypes binding of the CPU oracle (tron_oracle.c).

TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the benchmark's
CPU-baseline leg. The GPU library never imports this package, and this package imports
nothing from the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tron_oracle.c")
_SO = os.path.join(_HERE, "_tron_oracle.so")
# The planted-mistake check (tests/test_oracle_mutations.py) builds altered copies of the
# oracle and points this variable at one of them; nothing else sets it.
_SO_OVERRIDE = os.environ.get("TRON_ORACLE_SO_OVERRIDE")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11", "-Wall", "-Wextra",
          "-shared", "-fPIC"]

QP4, BR6, HS45M = 0, 1, 2
CONVERGED, MAX_ITER, STALLED, NONFINITE, BAD_BOUNDS = 0, 1, 2, 3, 4
NSTAT = 8
STAT_NAMES = ("flops", "iters", "cg_iters", "chol_tries", "cauchy_trials", "search_trials",
              "passes", "accepted")


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math)."""
    cmd = ["gcc", *CFLAGS, "-o", _SO, _SRC, "-lm", "-lpthread"]
    out = subprocess.run(cmd, capture_output=True, text=True)
    if out.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + out.stderr)
    if verbose and out.stderr:
        print(out.stderr)
    return _SO


class Opts(C.Structure):
    _fields_ = [("gtol", C.c_double), ("max_iter", C.c_int32), ("use_warm", C.c_int32),
                ("cg_rtol", C.c_double), ("delta0", C.c_double)]


class AlOpts(C.Structure):
    _fields_ = [("ctol", C.c_double), ("outer_max", C.c_int32), ("rho_growth", C.c_double),
                ("decrease", C.c_double), ("rho_max", C.c_double)]


class NetworkC(C.Structure):
    _fields_ = [("nbus", C.c_int32), ("nbranch", C.c_int32), ("ngen", C.c_int32),
                ("ref_bus", C.c_int32), ("rho", C.c_double), ("base_mva", C.c_double),
                ("br_from", C.c_void_p), ("br_to", C.c_void_p), ("br_adm", C.c_void_p),
                ("br_lo", C.c_void_p), ("br_hi", C.c_void_p), ("gen_bus", C.c_void_p),
                ("gen_cost", C.c_void_p), ("gen_lim", C.c_void_p), ("bus_load", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _SO_OVERRIDE:
            L = C.CDLL(_SO_OVERRIDE)
        else:
            if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
                build()
            L = C.CDLL(_SO)
        P = C.c_void_p
        L.or_param_size.restype = C.c_int64
        L.or_param_size.argtypes = [C.c_int32, C.c_int32]
        L.or_tron_batch.restype = C.c_int32
        L.or_tron_batch.argtypes = [C.c_int32, C.c_int64, P, C.c_int32, P, P, P, P, P, P, P, P,
                                    P, P, P, C.POINTER(Opts), C.c_int32]
        L.or_eval_f.restype = C.c_double
        L.or_eval_f.argtypes = [C.c_int32, C.c_int32, P, P]
        L.or_eval_g.argtypes = [C.c_int32, C.c_int32, P, P, P]
        L.or_eval_h.argtypes = [C.c_int32, C.c_int32, P, P, P]
        L.or_br6_flows.argtypes = [P, P, P]
        L.or_eval_batch.argtypes = [C.c_int32, C.c_int64, P, C.c_int32, P, P, P, P, P, P]
        L.or_ccf.restype = C.c_int32
        L.or_ccf.argtypes = [C.c_int32, P, C.c_double, P]
        L.or_trsv_lower.argtypes = [C.c_int32, P, P]
        L.or_trsv_lower_t.argtypes = [C.c_int32, P, P]
        L.or_trqsol.restype = C.c_double
        L.or_trqsol.argtypes = [C.c_int32, P, P, C.c_double]
        L.or_breakpt.argtypes = [C.c_int32, P, P, P, P, P, P, P]
        L.or_gpstep.argtypes = [C.c_int32, P, P, P, C.c_double, P, P]
        L.or_projgrad_inf.restype = C.c_double
        L.or_projgrad_inf.argtypes = [C.c_int32, P, P, P, P]
        L.or_subspace_cg.restype = C.c_int32
        L.or_subspace_cg.argtypes = [C.c_int32, P, P, C.c_double, C.c_double, P, P, P, P]
        L.or_radius_update.restype = C.c_double
        L.or_radius_update.argtypes = [C.c_double] * 6 + [C.c_int32]
        L.or_cauchy_step.restype = C.c_double
        L.or_cauchy_step.argtypes = [C.c_int32, P, P, P, P, P, C.c_double, C.c_double, P, P]
        L.or_projected_search.restype = C.c_int32
        L.or_projected_search.argtypes = [C.c_int32, P, P, P, P, P, P, P, P, P]
        L.or_step_norm.restype = C.c_double
        L.or_step_norm.argtypes = [C.c_int32, P, C.c_int32, P, P]
        L.or_actual_reduction.restype = C.c_double
        L.or_actual_reduction.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, P, P, P]
        L.or_family_flops.restype = C.c_double
        L.or_family_flops.argtypes = [C.c_int32, C.c_int32, C.c_int32]
        L.or_al_batch.restype = C.c_int32
        L.or_al_batch.argtypes = [C.c_int64, P, P, P, P, P, P, P, P, P, P, C.POINTER(Opts),
                                  C.POINTER(AlOpts), C.c_int32]
        L.or_admm_state_size.restype = C.c_int64
        L.or_admm_state_size.argtypes = [C.POINTER(NetworkC)]
        L.or_admm_init.argtypes = [C.POINTER(NetworkC), P]
        L.or_admm_run.restype = C.c_int32
        L.or_admm_run.argtypes = [C.POINTER(NetworkC), P, C.c_int32, P, C.POINTER(Opts),
                                  C.c_int32]
        L.or_admm_phase.restype = C.c_int32
        L.or_admm_phase.argtypes = [C.POINTER(NetworkC), P, C.c_int32, P, C.POINTER(Opts),
                                    C.c_int32]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def opts(gtol=1e-6, max_iter=500, cg_rtol=0.1, delta0=0.0, use_warm=0) -> Opts:
    return Opts(gtol, max_iter, use_warm, cg_rtol, delta0)


def al_solve(batch, ctol=1e-6, outer_max=50, rho_growth=10.0, decrease=0.25, rho_max=1e6,
             gtol=1e-6, max_iter=500, cg_rtol=0.1, delta0=0.0, nthreads=0):
    """Augmented-Lagrangian loop over a BR8L batch (n = 8, 40 parameters per instance).
    Returns a dict: x, f, status, iters, outer, viol, params (with the final multipliers and
    penalties)."""
    B = int(batch.n.shape[0])
    assert batch.family == 3 and np.all(batch.n == 8)
    params = _f64(batch.params).copy()
    lo, hi, x0 = _f64(batch.lo), _f64(batch.hi), _f64(batch.x0)
    x = np.zeros(8 * B)
    f, viol = np.zeros(B), np.zeros(B)
    status, iters, outer = (np.zeros(B, dtype=np.int32) for _ in range(3))
    o = opts(gtol, max_iter, cg_rtol, delta0, 0)
    a = AlOpts(ctol, outer_max, rho_growth, decrease, rho_max)
    lib().or_al_batch(B, _p(params), _p(lo), _p(hi), _p(x0), _p(x), _p(f), _p(status), _p(iters),
                      _p(outer), _p(viol), C.byref(o), C.byref(a), nthreads)
    return dict(x=x, f=f, status=status, iters=iters, outer=outer, viol=viol, params=params)


def param_size(family, n):
    return int(lib().or_param_size(family, n))


def solve(batch, gtol=1e-6, max_iter=500, cg_rtol=0.1, delta0=0.0, delta=None, alphac=None,
          use_warm=False, nthreads=0, with_stats=True):
    """Solve every instance of `batch` (attributes family, n, params, lo, hi, x0).
    Returns a dict: x, f, status, iters, delta, alphac, stats, threads."""
    n = np.ascontiguousarray(batch.n, dtype=np.int32)
    B = int(n.shape[0])
    nsum = int(n.astype(np.int64).sum())
    x = np.zeros(nsum)
    f = np.zeros(B)
    status = np.zeros(B, dtype=np.int32)
    iters = np.zeros(B, dtype=np.int32)
    d = _f64(delta).copy() if delta is not None else np.zeros(B)
    a = _f64(alphac).copy() if alphac is not None else np.zeros(B)
    stats = np.zeros(B * NSTAT) if with_stats else None
    params, lo, hi, x0 = (_f64(batch.params), _f64(batch.lo), _f64(batch.hi), _f64(batch.x0))
    o = opts(gtol, max_iter, cg_rtol, delta0, 1 if use_warm else 0)
    nt = lib().or_tron_batch(batch.family, B, _p(n), 0, _p(params), _p(lo), _p(hi), _p(x0),
                             _p(x), _p(f), _p(status), _p(iters), _p(d), _p(a), _p(stats),
                             C.byref(o), nthreads)
    out = dict(x=x, f=f, status=status, iters=iters, delta=d, alphac=a, threads=nt)
    if with_stats:
        out["stats"] = stats.reshape(B, NSTAT)
    return out


def eval_f(family, n, params, x):
    return lib().or_eval_f(family, n, _p(_f64(params)), _p(_f64(x)))


def eval_g(family, n, params, x):
    g = np.zeros(n)
    lib().or_eval_g(family, n, _p(_f64(params)), _p(_f64(x)), _p(g))
    return g


def eval_h(family, n, params, x):
    h = np.zeros(n * n)
    lib().or_eval_h(family, n, _p(_f64(params)), _p(_f64(x)), _p(h))
    return h.reshape(n, n)


def eval_batch(batch, x):
    """f and the infinity norm of the projected gradient of every instance of `batch` at
    the packed points x (one array, instances back to back)."""
    n = np.ascontiguousarray(batch.n, dtype=np.int32)
    B = int(n.shape[0])
    x = _f64(x)
    assert x.shape[0] == int(n.astype(np.int64).sum())
    f = np.zeros(B)
    pg = np.zeros(B)
    lib().or_eval_batch(batch.family, B, _p(n), 0, _p(_f64(batch.params)), _p(_f64(batch.lo)),
                        _p(_f64(batch.hi)), _p(x), _p(f), _p(pg))
    return f, pg


def br6_flows(params, x):
    out = np.zeros(4)
    lib().or_br6_flows(_p(_f64(params)), _p(_f64(x)), _p(out))
    return out


def ccf(a, alpha=0.0):
    a = _f64(a)
    m = a.shape[0]
    l = np.zeros((m, m))
    rc = lib().or_ccf(m, _p(a), alpha, _p(l))
    return rc, l


def trsv_lower(l, b):
    l = _f64(l); b = _f64(b).copy()
    lib().or_trsv_lower(l.shape[0], _p(l), _p(b))
    return b


def trsv_lower_t(l, b):
    l = _f64(l); b = _f64(b).copy()
    lib().or_trsv_lower_t(l.shape[0], _p(l), _p(b))
    return b


def trqsol(x, p, delta):
    x = _f64(x); p = _f64(p)
    return lib().or_trqsol(x.shape[0], _p(x), _p(p), delta)


def breakpt(x, lo, hi, w):
    x, lo, hi, w = map(_f64, (x, lo, hi, w))
    nb = np.zeros(1, dtype=np.int32)
    bmin = np.zeros(1); bmax = np.zeros(1)
    lib().or_breakpt(x.shape[0], _p(x), _p(lo), _p(hi), _p(w), _p(nb), _p(bmin), _p(bmax))
    return int(nb[0]), float(bmin[0]), float(bmax[0])


def gpstep(x, lo, hi, alpha, w):
    x, lo, hi, w = map(_f64, (x, lo, hi, w))
    s = np.zeros_like(x)
    lib().or_gpstep(x.shape[0], _p(x), _p(lo), _p(hi), alpha, _p(w), _p(s))
    return s


def projgrad_inf(x, lo, hi, g):
    x, lo, hi, g = map(_f64, (x, lo, hi, g))
    return lib().or_projgrad_inf(x.shape[0], _p(x), _p(lo), _p(hi), _p(g))


def subspace_cg(a, r, delta, cg_rtol=0.1):
    a = _f64(a); r = _f64(r)
    m = r.shape[0]
    w = np.zeros(m); sh = np.zeros(m)
    it = np.zeros(1, dtype=np.int32); shift = np.zeros(1)
    ex = lib().or_subspace_cg(m, _p(a), _p(r), delta, cg_rtol, _p(w), _p(sh), _p(it), _p(shift))
    return dict(exit=int(ex), w=w, shat=sh, iters=int(it[0]), shift=float(shift[0]))


def radius_update(delta, rho, f, ft, gts, snorm, finite=True):
    return lib().or_radius_update(delta, rho, f, ft, gts, snorm, 1 if finite else 0)


def cauchy_step(x, lo, hi, g, H, delta, alpha):
    """Returns (alpha, xs, trials)."""
    x, lo, hi, g = map(_f64, (x, lo, hi, g))
    H = _f64(H)
    xs = np.zeros_like(x)
    tr = np.zeros(1, dtype=np.int32)
    a = lib().or_cauchy_step(x.shape[0], _p(x), _p(lo), _p(hi), _p(g), _p(H), delta, alpha,
                             _p(xs), _p(tr))
    return a, xs, int(tr[0])


def projected_search(xs, lo, hi, w, r, H):
    """Returns (accepted, new xs, last beta tried, trials)."""
    xs, lo, hi, w, r = map(_f64, (xs, lo, hi, w, r))
    H = _f64(H)
    out = np.zeros_like(xs)
    beta = np.zeros(1)
    tr = np.zeros(1, dtype=np.int32)
    acc = lib().or_projected_search(xs.shape[0], _p(xs), _p(lo), _p(hi), _p(w), _p(r), _p(H),
                                    _p(out), _p(beta), _p(tr))
    return bool(acc), out, float(beta[0]), int(tr[0])


def step_norm(s, free_idx, L):
    s = _f64(s)
    idx = np.ascontiguousarray(free_idx, dtype=np.int32)
    L = _f64(L) if len(idx) else np.zeros(1)
    return lib().or_step_norm(s.shape[0], _p(s), len(idx), _p(idx), _p(L))


def actual_reduction(f, ft, pred, g, gt, s):
    g, gt, s = map(_f64, (g, gt, s))
    return lib().or_actual_reduction(s.shape[0], f, ft, pred, _p(g), _p(gt), _p(s))


def family_flops(family, n, which):
    return lib().or_family_flops(family, n, which)


# ---------------------------------------------------------------- component ADMM
def _net_struct(net):
    keep = [net.br_from, net.br_to, net.br_adm, net.br_lo, net.br_hi, net.gen_bus, net.gen_cost,
            net.gen_lim, net.bus_load]
    s = NetworkC(net.nbus, net.nbranch, net.ngen, net.ref_bus, net.rho, net.base_mva,
                 *[_p(np.ascontiguousarray(a)) for a in keep])
    return s, keep


def admm_init(net):
    s, keep = _net_struct(net)
    st = np.zeros(int(lib().or_admm_state_size(C.byref(s))))
    lib().or_admm_init(C.byref(s), _p(st))
    return st


def admm_run(net, state, iters, gtol=1e-6, max_iter=500, cg_rtol=0.1, nthreads=0):
    """Run `iters` ADMM iterations on a copy of `state`; returns (state, resid[iters, 2])."""
    s, keep = _net_struct(net)
    st = _f64(state).copy()
    res = np.zeros(2 * max(iters, 1))
    o = opts(gtol, max_iter, cg_rtol, 0.0, 1)
    rc = lib().or_admm_run(C.byref(s), _p(st), iters, _p(res), C.byref(o), nthreads)
    if rc != 0:
        raise ValueError("network has a bus with no branch")
    return st, res[:2 * iters].reshape(iters, 2)


def admm_phase(net, state, phase, gtol=1e-6, max_iter=500, cg_rtol=0.1, nthreads=0):
    """Apply one phase (0 generators, 1 branches, 2 buses, 3 multipliers) to a copy of
    `state`; returns (state, scalar) where the scalar is the squared dual change (buses)
    or the squared primal residual (multipliers)."""
    s, keep = _net_struct(net)
    st = _f64(state).copy()
    out = np.zeros(1)
    o = opts(gtol, max_iter, cg_rtol, 0.0, 1)
    rc = lib().or_admm_phase(C.byref(s), _p(st), phase, _p(out), C.byref(o), nthreads)
    if rc != 0:
        raise ValueError("bad phase")
    return st, float(out[0])


def admm_views(net, state):
    """Named views into a flat ADMM state (the layout of the C interface)."""
    G, L, B = net.ngen, net.nbranch, net.nbus
    s = state
    o = 6 * G
    v = dict(pg=s[0:G], qg=s[G:2 * G], pgt=s[2 * G:3 * G], qgt=s[3 * G:4 * G],
             lpg=s[4 * G:5 * G], lqg=s[5 * G:6 * G])
    v["x"] = s[o:o + 6 * L].reshape(L, 6); o += 6 * L
    v["y"] = s[o:o + 8 * L].reshape(L, 8); o += 8 * L
    v["yt"] = s[o:o + 4 * L].reshape(L, 4); o += 4 * L
    v["lam"] = s[o:o + 8 * L].reshape(L, 8); o += 8 * L
    v["mu"] = s[o:o + 2 * L].reshape(L, 2); o += 2 * L
    v["delta"] = s[o:o + L]; o += L
    v["alphac"] = s[o:o + L]; o += L
    v["wt"] = s[o:o + B]; o += B
    v["tht"] = s[o:o + B]; o += B
    return v
