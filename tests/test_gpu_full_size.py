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


def _check_levels(pb, U, reps, col, levels, gate):
    g = 1.0 / math.gamma(1.0 - pb.gamma)
    for m in levels:
        a = oracle.l1_weights(pb.T, pb.M, pb.r, pb.gamma, m)
        rhs = g * a[0] * U[0] + pb.f[m - 1]
        if m > 1:
            rhs = rhs + g * (np.diff(a)[: m - 1] @ U[1:m])
        lhs = g * a[m - 1] * U[m] + pb.kappa[m - 1] * sla.matmul_toeplitz(col, U[m])
        rel = float(np.linalg.norm(rhs - lhs) / np.linalg.norm(rhs))
        rep = reps[m - 1].relres
        say(f"  level {m}: relative residual of the direct scheme {rel:.2e}, true residual the GPU reports {rep:.2e}")
        assert rel <= gate, m
        # the solver's own true residual (FIDS system, GPU FFTs) and this one
        # (direct history, scipy FFTs) agree up to the SOE tolerance and the
        # rounding of two FP64 evaluations at the floor (measured ratio about 3.4)
        assert rel <= 5.0 * rep + 1e-9, m


# The largest problems the library accepts.  There the attainable FP64
# residual of a level is no longer the Krylov tolerance: a matvec through
# FFTs of length L is exact to about eps log2(L) ||kappa|| ||A|| ||u|| (||A||
# grows like h^{-alpha}), a few 1e-9 of ||b|| at n = 2^20 for these smooth
# states, so the solvers accept a level at that floor (reported) and the gate
# is 5e-8 (FP64) / 1e-7 (FP32 preconditioner).
LARGEST = [
    pytest.param(dict(solver=2, precision=0, x0_mode=3), 5e-8, id="pcg-fp64-x0cubic"),
    pytest.param(dict(solver=1, precision=0, x0_mode=3), 5e-8, id="fgmres-fp64-x0cubic"),
    pytest.param(dict(solver=1, precision=1, x0_mode=3), 1e-7, id="mixed-fgmres-fp32pc"),
]


@pytest.mark.parametrize("kw,gate", LARGEST)
@pytest.mark.parametrize("n", [(1 << 20) - 1, (1 << 21) - 1])
def test_largest_sizes_satisfy_direct_scheme(n, kw, gate):
    """n <= 2^21: embedding 2^22, longest column FFT 2048 points, one column
    per tile, twiddle tables partly in global memory; six levels."""
    pb = W.seeded(1.3, 0.6, n, 6, kappa_seed=11, f_seed=12)
    U, reps = gpu_solve(pb, soe_tol=1e-10, krylov_tol=1e-10, krylov_maxit=500, **kw)
    assert np.isfinite(U).all()
    _check_levels(pb, U, reps, oracle.ifl_column(n, pb.alpha), range(1, 7), gate)
