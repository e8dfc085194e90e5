"""Pins of the 2-D operator of ``oracle.ifl2d`` (the 2-D form of the paper's
IFL matrix, eq. (3.16x); the paper names the multi-dimensional case in Sec. 6
without writing it out).  Every expected value here is fixed by mathematics,
not by the oracle:

* cell integrals of |eta|^beta against brute-force Gauss-Legendre quadrature;
* the splitting exponent: the same cell-error condition in 1-D is satisfied
  exactly by the paper's mu = 1 + alpha/2, and mu_star is a root of the 2-D
  one;
* Dyda's closed form: (-Delta)^{alpha/2} (1 - |x|^2)_+^{alpha/2} =
  2^alpha Gamma(1 + alpha/2)^2 inside the unit disk (d = 2);
* the Gaussian: (-Delta)^{alpha/2} e^{-|x|^2/s^2} =
  (2/s)^alpha Gamma(1 + alpha/2) 1F1(1 + alpha/2; 1; -|x|^2/s^2), with the
  second-order convergence the construction is designed for;
* symmetry, sign pattern and positive definiteness of the BTTB matrix.
A wrong constant c_{2,alpha}, exterior term, weight or exponent moves the
Dyda and Gaussian values by O(1).
"""
import math
import warnings

import numpy as np
import pytest
import scipy.special as sps

import oracle
from oracle import ifl2d

warnings.filterwarnings("ignore", category=UserWarning)


def _gl_cell(a, b, c, d, beta, pts=40, sub=1):
    x, w = np.polynomial.legendre.leggauss(pts)
    tot = 0.0
    for i in range(sub):
        for j in range(sub):
            a0, b0 = a + (b - a) * i / sub, a + (b - a) * (i + 1) / sub
            c0, d0 = c + (d - c) * j / sub, c + (d - c) * (j + 1) / sub
            xs = (a0 + b0) / 2 + (b0 - a0) / 2 * x
            ys = (c0 + d0) / 2 + (d0 - c0) / 2 * x
            f = (xs[:, None] ** 2 + ys[None, :] ** 2) ** (beta / 2)
            tot += (b0 - a0) * (d0 - c0) / 4 * float((w[:, None] * w[None, :] * f).sum())
    return tot


@pytest.mark.parametrize("beta", [-1.9, -1.25, -0.4])
@pytest.mark.parametrize("cell", [(1, 0), (2, 3), (10, 7), (40, 1), (150, 149)])
def test_cell_integrals_against_gauss_legendre(beta, cell):
    I = ifl2d.cell_integrals(max(cell) + 1, beta)
    k1, k2 = cell
    sub = 8 if max(cell) < 5 else 1
    ref = _gl_cell(k1, k1 + 1, k2, k2 + 1, beta, sub=sub)
    # the closed form is a difference of four corner integrals F of the size
    # of F(k1+1, k2+1), each good to about 1e-14 relative (hypergeometric
    # evaluation): that cancellation bounds the cell's error
    bound = 1e-14 * 4 * float(ifl2d.corner_integral(k1 + 1.0, k2 + 1.0, beta))
    assert abs(I[k1, k2] - ref) <= bound + 1e-13 * ref


@pytest.mark.parametrize("beta", [-1.8, -1.0, -0.3])
def test_origin_cell_against_polar_quadrature(beta):
    """The cell with a corner at the singular point: int_{[0,1]^2} r^beta =
    2 int_0^{pi/4} (1/cos t)^{beta+2} / (beta+2) dt."""
    import scipy.integrate as spi
    ref, _ = spi.quad(lambda t: (1.0 / math.cos(t)) ** (beta + 2) / (beta + 2), 0.0, math.pi / 4,
                      epsabs=1e-15, epsrel=1e-14)
    got = float(ifl2d.corner_integral(1.0, 1.0, beta))
    assert got == pytest.approx(2 * ref, rel=1e-13)


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.9, 1.5])
def test_splitting_condition_gives_the_paper_exponent_in_1d(alpha):
    """The cell-error condition behind mu_star, written for 1-D intervals,
    holds on every interval at mu = 1 + alpha/2 (the paper's choice, Sec. 2.2)
    and fails elsewhere."""
    def err1(mu, K=512):
        k = np.arange(K + 1, dtype=np.float64)
        Pb = k ** (mu - alpha) / (mu - alpha)           # int eta^{mu-1-alpha}
        Pa = k ** (2 - alpha) / (2 - alpha)             # int eta^{1-alpha}
        g = k ** (2 - mu)
        g[0] = 0.0
        return (0.5 * (g[1:] + g[:-1])) * (Pb[1:] - Pb[:-1]) - (Pa[1:] - Pa[:-1])
    e = err1(1 + alpha / 2)
    assert np.max(np.abs(e)) <= 1e-12 * (512 ** (2 - alpha))
    assert abs(err1(1 + alpha / 2 + 0.05).sum()) > 1e-2


@pytest.mark.parametrize("alpha", [0.1, 0.5, 1.0, 1.5, 1.9])
def test_mu_star_is_a_root_in_range(alpha):
    mu = oracle.mu_star(alpha)
    assert alpha < mu < 2.0
    assert abs(oracle.lattice_error(mu, alpha)) <= 1e-9
    # brute-force partial sums approach zero at the rate of the tail
    e256 = ifl2d._lattice_error(mu, alpha, 256)
    e128 = ifl2d._lattice_error(mu, alpha, 128)
    assert abs(e256) < abs(e128) or abs(e256) < 1e-9


@pytest.mark.parametrize("alpha,tol", [(0.5, 1e-4), (1.0, 5e-5), (1.5, 1e-5), (1.9, 5e-6)])
def test_dyda_disk_constant(alpha, tol):
    """(1 - |x|^2)_+^{alpha/2} on Omega = (-1, 1)^2: the discrete operator at
    the centre tends to 2^alpha Gamma(1 + alpha/2)^2."""
    target = 2.0 ** alpha * math.gamma(1 + alpha / 2) ** 2
    errs = []
    for n in (63, 127):
        a = oracle.ifl2d_coefficients(n, alpha, 1.0)
        X, Y = oracle.grid2d(n, 1.0)
        U = np.clip(1 - X ** 2 - Y ** 2, 0, None) ** (alpha / 2)
        c = n // 2
        errs.append(abs(oracle.ifl2d_apply_at(a, U, c, c) - target) / target)
    assert errs[1] < errs[0]
    assert errs[1] <= tol


@pytest.mark.parametrize("alpha", [0.1, 0.5, 1.0, 1.9])
def test_gaussian_second_order(alpha):
    """e^{-|x|^2/s^2}, s = 0.2, on Omega = (-1, 1)^2 (u < 2e-11 on the
    boundary): relative error at the centre and at x = (1/4, 0) against the
    closed form, falling by at least 3.5x when h is halved."""
    s = 0.2
    scale = (2 / s) ** alpha * math.gamma(1 + alpha / 2)
    errs = []
    for n in (63, 127):
        a = oracle.ifl2d_coefficients(n, alpha, 1.0)
        X, Y = oracle.grid2d(n, 1.0)
        U = np.exp(-(X ** 2 + Y ** 2) / s ** 2)
        c = n // 2
        i2 = c + (n + 1) // 8
        e = []
        for (i, j) in ((c, c), (i2, c)):
            exact = scale * sps.hyp1f1(1 + alpha / 2, 1, -(X[j, i] ** 2 + Y[j, i] ** 2) / s ** 2)
            e.append(abs(oracle.ifl2d_apply_at(a, U, i, j) - exact) / scale)
        errs.append(e)
    for k in range(2):
        assert errs[1][k] * 3.5 <= errs[0][k]
        assert errs[1][k] <= 4e-3


@pytest.mark.parametrize("alpha", [0.5, 1.5])
def test_bttb_structure(alpha):
    n = 15
    a = oracle.ifl2d_coefficients(n, alpha, 1.0)
    assert np.allclose(a, a.T, rtol=1e-14, atol=0)             # x <-> y symmetry of the kernel
    off = a.copy()
    off[0, 0] = -1.0
    assert np.all(off < 0)                                      # neighbours enter with a minus sign
    assert a[0, 0] > -(off.sum() + 1.0)                         # diagonal dominance of the generating row
    A = oracle.ifl2d_matrix(n, alpha, 1.0)
    assert np.array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 0
    # block-Toeplitz ordering: entry ((x,y),(x',y')) = a[|x-x'|, |y-y'|]
    assert A[3 + n * 5, 6 + n * 1] == a[3, 4]


def test_dids2d_level_equations():
    """dids2d_solve runs the direct scheme (4.1) with the 2-D matrix: each
    level satisfies (g a_m I + K A) u^m = rhs."""
    rng = np.random.default_rng(5)
    n, M, alpha, gamma, r = 7, 4, 1.4, 0.6, 2.0
    kappa = 1 + 0.5 * rng.random((M, n * n))
    f = rng.standard_normal((M, n * n))
    phi = rng.standard_normal(n * n)
    U = oracle.dids2d_solve(alpha, gamma, n, M, r, kappa, f, phi)
    A = oracle.ifl2d_matrix(n, alpha, 1.0)
    g = 1.0 / math.gamma(1.0 - gamma)
    for m in range(1, M + 1):
        a = oracle.l1_weights(1.0, M, r, gamma, m)
        rhs = g * a[0] * U[0] + f[m - 1]
        if m > 1:
            rhs = rhs + g * (np.diff(a)[: m - 1] @ U[1:m])
        lhs = g * a[m - 1] * U[m] + kappa[m - 1] * (A @ U[m])
        assert np.max(np.abs(lhs - rhs)) <= 1e-10 * np.max(np.abs(rhs))
