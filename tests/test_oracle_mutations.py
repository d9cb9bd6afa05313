"""Planted mistakes in the oracle must fail its CPU pins.

Each case changes one spot of a copy of oracle/tron_oracle.c (a dropped term, a wrong
sign, index or constant, a transposed operand, a wrong flop charge), builds it with the
oracle's own flags, and runs the oracle's pin tests against that build in a child process
(TRON_ORACLE_SO_OVERRIDE). The case passes when at least one pin fails. The mistakes are
planted on the CPU only; nothing here touches the HIP library.
"""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "tron_oracle.c")
PIN_FILES = ["test_oracle_core.py", "test_oracle_steps.py", "test_oracle_tron.py",
             "test_oracle_families.py", "test_oracle_admm.py", "test_oracle_al.py"]

# (name, text in the oracle, replacement). Every text occurs exactly once.
MUTATIONS = [
    # core operations
    ("dot drops its first term", "for (int i = 0; i < n; i++) s += a[i] * b[i];",
     "for (int i = 1; i < n; i++) s += a[i] * b[i];"),
    ("Cholesky reads L transposed", "l[i * m + k] * l[j * m + k]", "l[k * m + i] * l[j * m + k]"),
    ("backward solve uses L instead of L^T", "s -= l[k * m + i] * b[k]", "s -= l[i * m + k] * b[k]"),
    ("trqsol sign", "(dsq - xtx) / (ptx + rad)", "(dsq + xtx) / (ptx + rad)"),
    ("projected gradient at the lower bound", "if (x <= lo) return g < 0.0 ? g : 0.0;",
     "if (x <= lo) return g > 0.0 ? g : 0.0;"),
    ("breakpoint uses the wrong bound", "b = (hi[i] - x[i]) / w[i]", "b = (lo[i] - x[i]) / w[i]"),
    ("gpstep direction sign", "proj1(x[i] + alpha * w[i]", "proj1(x[i] - alpha * w[i]"),
    # families
    ("QP4 gradient drops a power", "kap4 * x[i] * x[i] * x[i]", "kap4 * x[i] * x[i]"),
    ("BR6 flow admittance sign", "double be[4] = {p[1], -p[0], -p[5], p[4]};",
     "double be[4] = {p[1], p[0], -p[5], p[4]};"),
    ("BR6 copy-coupling gradient sign", "g[i] -= coef * dy[pk][i]", "g[i] += coef * dy[pk][i]"),
    ("BR6 copy-coupling Hessian sign", "h[i * 6 + j] -= coef", "h[i * 6 + j] += coef"),
    # conjugate gradients and the subspace step
    ("CG direction coefficient inverted", "double bet = rrn / rr;", "double bet = rr / rrn;"),
    ("CG right-hand side sign", "w->rh[a] = -w->rF[a];", "w->rh[a] = w->rF[a];"),
    ("model gradient sign", "w->r[i] += w->g[i]", "w->r[i] -= w->g[i]"),
    ("negative-curvature test skipped", "if (!(kap > 0.0)) {", "if (kap < -1e300) {"),
    # readings S2, S4, S13, S30, S31
    ("sigma1 and sigma2 swapped", "SIG1 = 0.25, SIG2 = 0.5,", "SIG1 = 0.5, SIG2 = 0.25,"),
    ("eta1 and eta2 swapped", "ETA1 = 0.25, ETA2 = 0.75;", "ETA1 = 0.75, ETA2 = 0.25;"),
    ("mu0 0.01 -> 0.1", "MU0 = 0.01;", "MU0 = 0.1;"),
    ("Cauchy extrapolation x10 -> x2", "double a2 = 10.0 * alpha;", "double a2 = 2.0 * alpha;"),
    ("Cauchy interpolation x0.1 -> x0.5", "alpha = 0.1 * alpha;", "alpha = 0.5 * alpha;"),
    ("Cauchy ignores the largest breakpoint", "if (!(alpha < bmax)) break;", "if (0) break;"),
    ("alpha* on gamma <= 0", "if (gam <= 0.0) astar = SIG3;", "if (gam <= 0.0) astar = SIG1;"),
    ("alpha* formula sign", "astar = -0.5 * gts / gam;", "astar = 0.5 * gts / gam;"),
    ("search halving -> quartering", "beta *= 0.5;", "beta *= 0.25;"),
    ("step norm with L instead of L^T",
     "for (int b = a; b < m; b++) t += w->L[b * m + a] * w->s[w->lidx[b]];",
     "for (int b = 0; b <= a; b++) t += w->L[a * m + b] * w->s[w->lidx[b]];"),
    ("rounding switch without max(1, |f|)", "ARED_SWITCH * (fabs(f) > 1.0 ? fabs(f) : 1.0)",
     "ARED_SWITCH * fabs(f)"),
    ("trapezoid reduction sign", "return -0.5 * sg;", "return 0.5 * sg;"),
    # flop counter
    ("gemv charged m^2", "*fl += 2.0 * n * n;", "*fl += 1.0 * n * n;"),
    ("trqsol charge dropped", "    *fl += 9.0;\n", "    *fl += 0.0;\n"),
    ("QP4 gradient charge", "if (which == 1) return 4.0 * n + 1.0;", "if (which == 1) return 5.0 * n + 1.0;"),
    # ADMM closed forms
    ("generator update drops the linear cost", "- v->lpg[g] - c1) / (2.0 * c2 + rho)",
     "- v->lpg[g]) / (2.0 * c2 + rho)"),
    ("multiplier update sign", "la[k] += rho * r;", "la[k] -= rho * r;"),
]


def _build(tmp, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, (name, src.count(old))
    mut = src.replace(old, new)
    c = os.path.join(tmp, "m.c")
    so = os.path.join(tmp, "m.so")
    with open(c, "w") as fh:
        fh.write(mut)
    sys.path.insert(0, ROOT)
    import oracle
    flags = [f for f in oracle.CFLAGS if not f.startswith("-W")]
    hdr = os.path.join(ROOT, "oracle")
    out = subprocess.run(["gcc", *flags, "-I" + hdr, "-o", so, c, "-lm", "-lpthread"],
                         capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    return so


def _run(case):
    name, old, new = case
    with tempfile.TemporaryDirectory() as tmp:
        so = _build(tmp, name, old, new)
        env = dict(os.environ, TRON_ORACLE_SO_OVERRIDE=so, OMP_NUM_THREADS="1")
        cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
               "-m", "not gpu", *[os.path.join(HERE, f) for f in PIN_FILES]]
        out = subprocess.run(cmd, capture_output=True, text=True, env=env, cwd=ROOT, timeout=600)
        return name, out.returncode, out.stdout[-400:]


def test_every_planted_mistake_fails_a_pin():
    workers = max(1, min(6, (os.cpu_count() or 2) - 1))
    with cf.ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(_run, MUTATIONS))
    survived = [(n, tail) for n, rc, tail in results if rc == 0]
    assert not survived, "planted mistakes that no pin caught: " + "; ".join(n for n, _ in survived)
    # a return code other than "tests failed" (1) means the run itself broke
    broken = [(n, rc, tail) for n, rc, tail in results if rc not in (0, 1)]
    assert not broken, broken


def test_unaltered_copy_passes():
    """The harness itself: an identity 'mutation' must pass every pin."""
    name, rc, tail = _run(("identity", "MU0 = 0.01;", "MU0 = 0.01;"))
    assert rc == 0, tail
