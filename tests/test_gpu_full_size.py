"""GPU runs at the benchmark's full size (n = 65535, M = 2048, the bench
recipe and launch configuration), checked level by level against the direct
scheme: at sampled levels m the right-hand side of eq. (4.1),
    g [a_1 u^0 + sum_{k=1}^{m-1} (a_{k+1} - a_k) u^k] + f^m,
is rebuilt from the GPU's own earlier states with the oracle's graded-L1
weights, and u^m must satisfy
    g a_m u^m + kappa^m .* (A u^m) = that right-hand side
up to the SOE tolerance and the Krylov tolerance (A u^m by scipy's Toeplitz
product with the oracle's IFL column).  The oracle cannot solve this size,
but each level's equation it can evaluate; a dropped history term, a wrong
weight, sign or scaling anywhere in the path leaves an O(1) residual.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_2002_11978_amd import workloads as W

from gpu_util import gpu_solve, say

pytestmark = pytest.mark.gpu

N, M = 65535, 2048
LEVELS = [1, 2, 3, 100, 1024, 2047, 2048]

FORMS = [
    pytest.param(dict(solver=2, precision=0, x0_mode=3), 1e-8, id="headline-pcg-fp64-x0cubic"),
    pytest.param(dict(solver=1, precision=0, x0_mode=3), 1e-8, id="fgmres-fp64-x0cubic"),
    pytest.param(dict(solver=1, precision=1, x0_mode=3), 1e-7, id="mixed-fgmres-fp32pc"),
    pytest.param(dict(solver=0, precision=0, x0_mode=0), 1e-8, id="plain-bicgstab-fp64"),
]


@pytest.fixture(scope="module")
def recipe():
    pb = W.seeded(1.5, 0.4, N, M, r=4.0, kappa_seed=3, f_seed=4, name="bench")
    col = oracle.ifl_column(N, pb.alpha)
    return pb, col


@pytest.mark.parametrize("kw,gate", FORMS)
def test_full_size_levels_satisfy_direct_scheme(recipe, kw, gate):
    pb, col = recipe
    U, reps = gpu_solve(pb, soe_tol=1e-10, krylov_tol=1e-10, krylov_maxit=500, **kw)
    assert U.shape == (M + 1, N) and np.isfinite(U).all()
    g = 1.0 / math.gamma(1.0 - pb.gamma)
    worst = 0.0
    for m in LEVELS:
        a = oracle.l1_weights(pb.T, M, pb.r, pb.gamma, m)
        rhs = g * a[0] * U[0] + pb.f[m - 1]
        if m > 1:
            rhs = rhs + g * (np.diff(a)[: m - 1] @ U[1:m])
        lhs = g * a[m - 1] * U[m] + pb.kappa[m - 1] * sla.matmul_toeplitz(col, U[m])
        rel = float(np.linalg.norm(rhs - lhs) / np.linalg.norm(rhs))
        worst = max(worst, rel)
        say(f"  level {m}: relative residual of the direct scheme {rel:.2e} ({reps[m - 1].iters} its)")
        assert rel <= gate, m
    say(f"  worst {worst:.2e}")


def _rounding_level(pb, m, col, um, rhs_norm):
    """Rounding level of a level's FP64 residual relative to ||b||, from the
    same analysis as the library's acceptance bound: a product with A through
    length-L FFTs is exact to about u log2(L) ||A||_inf ||x|| (u = 2^-53),
    scaled by kappa <= kmax, plus u g a_m ||x|| from the shift and u ||b||."""
    u = 2.0 ** -53
    L = 1 << int(math.ceil(math.log2(2 * pb.n)))
    anorm = abs(col[0]) + 2.0 * np.abs(col[1:]).sum()
    g = 1.0 / math.gamma(1.0 - pb.gamma)
    beta = g * oracle.l1_weights(pb.T, pb.M, pb.r, pb.gamma, m)[m - 1]
    kmax = float(np.max(pb.kappa[m - 1]))
    return u * ((math.log2(L) * kmax * anorm + beta) * float(np.linalg.norm(um)) / rhs_norm + 1.0)


def _check_levels(pb, U, reps, col, levels, tol):
    g = 1.0 / math.gamma(1.0 - pb.gamma)
    for m in levels:
        a = oracle.l1_weights(pb.T, pb.M, pb.r, pb.gamma, m)
        rhs = g * a[0] * U[0] + pb.f[m - 1]
        if m > 1:
            rhs = rhs + g * (np.diff(a)[: m - 1] @ U[1:m])
        lhs = g * a[m - 1] * U[m] + pb.kappa[m - 1] * sla.matmul_toeplitz(col, U[m])
        rel = float(np.linalg.norm(rhs - lhs) / np.linalg.norm(rhs))
        e = _rounding_level(pb, m, col, U[m], float(np.linalg.norm(rhs)))
        accept = max(4.0 * tol, e)            # what the solver may accept (fids.h)
        # this evaluation differs from the solver's own true residual by the
        # SOE tolerance (1e-10 relative on the history) and by its own
        # rounding (scipy's FFTs, the same level e)
        gate = accept + e + 1e-9
        rep = reps[m - 1]
        say(f"  level {m}: direct-scheme residual {rel:.2e}, reported {rep.relres:.2e}, rounding level {e:.2e}, "
            f"gate {gate:.2e}, flags {rep.flags}")
        assert rep.relres <= accept, m
        assert bool(rep.flags & 1) == (rep.relres > tol), m
        assert rel <= gate, m


# The largest problems the library accepts.  There the attainable FP64
# residual of a level is no longer the Krylov tolerance: a matvec through
# FFTs of length L is exact to about u log2(L) kmax ||A||_inf ||u|| (||A||
# grows like h^{-alpha}); at n = 2^20 - 1 and 2^21 - 1 with alpha = 1.3 that
# rounding level is 1e-8 - 1e-7 of ||b|| for these states (PCG measured
# 1.99e-8 at n = 2^20 - 1).  The solvers accept a level at its floor only
# within max(4 tol, that level) and flag it; the gate of this check is that
# acceptance bound plus the check's own rounding and the SOE tolerance,
# computed per level.
LARGEST = [
    pytest.param(dict(solver=2, precision=0, x0_mode=3), id="pcg-fp64-x0cubic"),
    pytest.param(dict(solver=1, precision=0, x0_mode=3), id="fgmres-fp64-x0cubic"),
    pytest.param(dict(solver=1, precision=1, x0_mode=3), id="mixed-fgmres-fp32pc"),
]


@pytest.mark.parametrize("kw", LARGEST)
@pytest.mark.parametrize("n", [(1 << 20) - 1, (1 << 21) - 1])
def test_largest_sizes_satisfy_direct_scheme(n, kw):
    """n <= 2^21: embedding 2^22, longest column FFT 2048 points, one column
    per tile, twiddle tables partly in global memory; six levels."""
    pb = W.seeded(1.3, 0.6, n, 6, kappa_seed=11, f_seed=12)
    U, reps = gpu_solve(pb, soe_tol=1e-10, krylov_tol=1e-10, krylov_maxit=500, **kw)
    assert np.isfinite(U).all()
    _check_levels(pb, U, reps, oracle.ifl_column(n, pb.alpha), range(1, 7), 1e-10)
