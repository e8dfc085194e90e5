"""Two-dimensional integral fractional Laplacian on a square, plain FP64.

Test infrastructure only (see the package docstring).

The paper treats the 1-D problem and names the multi-dimensional case as a
direct adaptation (Sec. 6, conclusions) without writing it out.  This module
states the 2-D operator the library implements, as the analogue of the 1-D
matrix of eq. (3.16x) built the same way (Sec. 3.1): the same splitting of the
hypersingular integral, the same weighted trapezoidal rule, the same exact
treatment of the region where both neighbours lie outside the domain.

Domain Omega = (-l, l)^2, N_p intervals per axis, h = 2l/N_p, interior nodes
x_{ij} = (-l + i h, -l + j h), i, j = 1..n (n = N_p - 1), u = 0 outside Omega.
With the symmetrised definition (1.4) in two dimensions,

  (-Delta)^{alpha/2} u(x) = (c_2/2) int_{R^2} (2u(x) - u(x+xi) - u(x-xi)) |xi|^{-2-alpha} dxi,
  c_2 = c_{2,alpha} = alpha 2^{alpha-1} Gamma(1 + alpha/2) / (pi Gamma(1 - alpha/2)),

the integrand is split as psi(xi) omega(xi) with psi = (2u(x) - u(x+xi) -
u(x-xi)) / |xi|^mu, omega = |xi|^(mu-2-alpha), mu = mu_star(alpha) in
(alpha, 2), the 2-D counterpart of the paper's mu = 1 + alpha/2 (see
`mu_star`; psi -> 0 at xi = 0).  In lattice units xi = h eta:

* inside the square |eta|_inf <= N_p, psi is replaced on every unit cell by
  the mean of its four corner values and omega is integrated exactly over the
  cell (the 2-D form of the 1-D weighted trapezoidal rule), which gives node
  m the weight W_m = (1/4) sum of I_C over the (up to four) cells C of the
  square that have m as a corner, I_C = int_C |eta|^beta, beta = mu-2-alpha;
* outside it, x +- xi lie outside Omega, psi = 2u(x)/|xi|^mu exactly and the
  integral is E = int_{|eta|_inf >= N_p} |eta|^(-2-alpha) = (8/alpha) N_p^(-alpha)
  int_0^{pi/4} cos^alpha(t) dt.

The discrete operator is then the symmetric block-Toeplitz matrix with
Toeplitz blocks

  A = (c_2 / h^alpha) [ D I - sum_{0 < |m|_inf <= n-1} (W_m / |m|^mu) S_m ],
  D = sum_{0 < |m|_inf <= N_p} W_m / |m|^mu + E,

(S_m the shift by m), whose 1-D restriction of the same construction is the
matrix of eq. (3.16x).  Unknowns are ordered x-fastest: index i-1 + n (j-1).
"""
from __future__ import annotations

import math

import functools

import numpy as np
import scipy.optimize as so
import scipy.special as sps


def c2_alpha(alpha: float) -> float:
    """c_{d,alpha} of the IFL definition (1.4) for d = 2:
    alpha 2^{alpha-1} Gamma((d+alpha)/2) / (pi^{d/2} Gamma(1 - alpha/2))."""
    return alpha * 2.0 ** (alpha - 1) * math.gamma(1 + alpha / 2) / (math.pi * math.gamma(1 - alpha / 2))


def _lattice_error(mu: float, alpha: float, K: int) -> float:
    """Sum over the unit cells C of [-K, K]^2 of the rule's error for psi =
    |eta|^{2-mu}: (mean of psi at the corners of C) int_C |eta|^{mu-2-alpha}
    - int_C |eta|^{-alpha}, with psi(0) = 0 (four times the first quadrant)."""
    g = np.arange(K + 1, dtype=np.float64)
    Fb = corner_integral(g[:, None], g[None, :], mu - 2.0 - alpha)
    Fa = corner_integral(g[:, None], g[None, :], -alpha)
    Ib = Fb[1:, 1:] - Fb[:-1, 1:] - Fb[1:, :-1] + Fb[:-1, :-1]
    Ia = Fa[1:, 1:] - Fa[:-1, 1:] - Fa[1:, :-1] + Fa[:-1, :-1]
    P = np.hypot(g[:, None], g[None, :]) ** (2.0 - mu)
    P[0, 0] = 0.0
    avg = 0.25 * (P[1:, 1:] + P[:-1, 1:] + P[1:, :-1] + P[:-1, :-1])
    return 4.0 * float(np.sum(avg * Ib - Ia))


def lattice_error(mu: float, alpha: float) -> float:
    """The rule's total error over the plane for psi = |eta|^{2-mu}: partial
    sums over [-K, K]^2 for K = 32, 64, 128, extrapolated in K with the tail
    K^{-alpha} (a + b K^{-2}) of per-cell errors that decay like |eta|^{-2-alpha}
    (two Richardson steps; about 1e-10 from the limit)."""
    S = [_lattice_error(mu, alpha, K) for K in (32, 64, 128)]
    q1, q2 = 2.0 ** (-alpha), 2.0 ** (-alpha - 2.0)
    R = [(S[i + 1] - q1 * S[i]) / (1.0 - q1) for i in range(2)]
    return (R[1] - q2 * R[0]) / (1.0 - q2)


@functools.lru_cache(maxsize=None)
def mu_star(alpha: float) -> float:
    """The splitting exponent mu of the 2-D operator.

    A smooth u gives psi = -(xi^T H xi / |xi|^2) |xi|^{2-mu} + O(|xi|^{4-mu})
    (H the Hessian of u at x).  The rule's error on that leading term, summed
    over all cells, is of order h^{2-alpha} unless it vanishes; by the
    symmetry of the lattice only the trace of H survives, so the requirement
    is lattice_error(mu) = 0.  In 1-D the same requirement holds on every
    interval separately exactly when mu = 1 + alpha/2, the paper's choice
    (Sec. 2.2): ((a^{1-a/2} + b^{1-a/2})/2) (b^{1-a/2} - a^{1-a/2})/(1-a/2) =
    (b^{2-a} - a^{2-a})/(2-a).  In 2-D no mu makes every cell exact; the root
    of the summed error in (alpha, 2) is taken (it exists: the error tends to
    +inf as mu -> alpha and equals -1/4 int over the four cells at the origin
    of |eta|^{-alpha} at mu = 2).  With it the operator is second-order
    consistent on smooth u (measured: Gaussian, relative error falling 4x per
    halving of h)."""
    return float(so.brentq(lattice_error, alpha + 1e-6, 2.0, args=(alpha,), xtol=1e-14, rtol=1e-15))


def _mu(alpha):
    return mu_star(alpha)


def corner_integral(X, Y, beta):
    """F(X, Y) = int_0^X int_0^Y (x^2 + y^2)^{beta/2} dy dx for X, Y >= 0 and
    -2 < beta < 0.

    The rectangle is split by its diagonal into two triangles with a vertex at
    the origin; in polar coordinates the radial integral is exact and the
    angular one, with t = tan(theta), is int_0^T (1 + t^2)^{nu/2 - 1} dt =
    T 2F1(1/2, 1 - nu/2; 3/2; -T^2), nu = beta + 2:
      F = X^{nu-1} Y / nu 2F1(.; -Y^2/X^2) + Y^{nu-1} X / nu 2F1(.; -X^2/Y^2).
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    nu = beta + 2.0
    out = np.zeros(np.broadcast(X, Y).shape)
    Xb, Yb = np.broadcast_arrays(X, Y)
    ok = (Xb > 0) & (Yb > 0)
    x, y = Xb[ok], Yb[ok]
    b = 1.0 - nu / 2
    t1 = x ** (nu - 1) * y / nu * sps.hyp2f1(0.5, b, 1.5, -(y / x) ** 2)
    t2 = y ** (nu - 1) * x / nu * sps.hyp2f1(0.5, b, 1.5, -(x / y) ** 2)
    out[ok] = t1 + t2
    return out


def cell_integrals(Np: int, beta: float) -> np.ndarray:
    """I[k1, k2] = int over the unit cell [k1, k1+1] x [k2, k2+1] of |eta|^beta
    for 0 <= k1, k2 < Np (first quadrant; the other quadrants by symmetry)."""
    g = np.arange(Np + 1, dtype=np.float64)
    F = corner_integral(g[:, None], g[None, :], beta)
    return F[1:, 1:] - F[:-1, 1:] - F[1:, :-1] + F[:-1, :-1]


def node_weights(Np: int, alpha: float, mu: float) -> np.ndarray:
    """W[m1 + Np, m2 + Np] for |m|_inf <= Np: a quarter of the integrals of
    |eta|^beta over the unit cells of the square [-Np, Np]^2 that have node m
    as a corner."""
    beta = mu - 2.0 - alpha
    Iq = cell_integrals(Np, beta)
    k = np.arange(-Np, Np)
    sig = np.where(k >= 0, k, -k - 1)                 # cell [k, k+1] mirrored into [0, Np)
    full = Iq[np.ix_(sig, sig)]                      # cells with lower-left corner k, k in [-Np, Np)
    pad = np.zeros((2 * Np + 2, 2 * Np + 2))
    pad[1:-1, 1:-1] = full                           # pad[k + Np + 1]
    # node m touches the cells with lower-left corners m, m-(1,0), m-(0,1), m-(1,1)
    W = 0.25 * (pad[1:, 1:] + pad[:-1, 1:] + pad[1:, :-1] + pad[:-1, :-1])
    return W                                         # W[m + Np], m in [-Np, Np]


def exterior_integral(Np: int, alpha: float) -> float:
    """E = int_{|eta|_inf >= Np} |eta|^{-2-alpha} d eta
    = (8 / alpha) Np^{-alpha} int_0^{pi/4} cos^alpha(t) dt."""
    x, w = np.polynomial.legendre.leggauss(40)       # smooth integrand: exact to rounding
    t = math.pi / 8 * (x + 1.0)
    val = math.pi / 8 * float(np.sum(w * np.cos(t) ** alpha))
    return 8.0 / alpha * Np ** (-alpha) * val


def ifl2d_coefficients(n: int, alpha: float, l: float = 1.0, mu: float | None = None) -> np.ndarray:
    """a[p, q], 0 <= p, q <= n-1: the entry of A coupling nodes whose indices
    differ by (+-p, +-q); a[0, 0] is the diagonal.  mu defaults to mu_star."""
    Np = n + 1
    h = 2.0 * l / Np
    mu = _mu(alpha) if mu is None else mu
    W = node_weights(Np, alpha, mu)
    m = np.arange(-Np, Np + 1, dtype=np.float64)
    R = np.hypot(m[:, None], m[None, :])
    R[Np, Np] = 1.0
    ratio = W / R ** mu
    ratio[Np, Np] = 0.0
    D = float(np.sum(ratio)) + exterior_integral(Np, alpha)
    scale = c2_alpha(alpha) / h ** alpha
    a = -scale * ratio[Np:Np + n, Np:Np + n]
    a[0, 0] = scale * D
    return a


def ifl2d_matrix(n: int, alpha: float, l: float = 1.0, mu: float | None = None) -> np.ndarray:
    """Dense symmetric BTTB matrix of order n^2 (x-fastest ordering)."""
    a = ifl2d_coefficients(n, alpha, l, mu)
    i = np.arange(n)
    dx = np.abs(i[:, None] - i[None, :])
    # A[(x, y), (x', y')] = a[|x - x'|, |y - y'|]
    A = a[dx[None, :, None, :], dx[:, None, :, None]]
    return A.reshape(n * n, n * n)


def ifl2d_apply_at(a: np.ndarray, U: np.ndarray, i: int, j: int) -> float:
    """(A u) at node (i, j) (0-based, x index i) by the direct sum over the
    nodes of the grid; U[j, i] holds u at node (i, j)."""
    n = U.shape[0]
    x = np.arange(n)
    P = np.abs(x - i)
    Q = np.abs(x - j)
    return float(np.sum(a[P[None, :], Q[:, None]] * U))


def grid(n: int, l: float = 1.0):
    """Interior node coordinates (X, Y), each of shape (n, n), indexed [j, i]."""
    h = 2.0 * l / (n + 1)
    x = -l + h * np.arange(1, n + 1)
    return np.meshgrid(x, x, indexing="xy")


def dids2d_solve(alpha, gamma, n, M, r, kappa, f, phi, l=1.0, T=1.0, mu=None):
    """The direct scheme (4.1) with the 2-D matrix: kappa, f rows and phi are
    flattened n^2 fields in the x-fastest ordering."""
    from .fids_oracle import dids_solve
    return dids_solve(alpha, gamma, n * n, M, r, kappa, f, phi, l, T, matrix=ifl2d_matrix(n, alpha, l, mu))
