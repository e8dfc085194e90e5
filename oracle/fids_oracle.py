"""Direct implicit difference scheme (DIDS) in plain FP64 NumPy/LAPACK.

Test infrastructure only (see the package docstring).  Notation follows the
paper: N_p = number of spatial intervals (the paper's N), n = N_p - 1 interior
unknowns, h = 2l/N_p, x_i = -l + i h; t_m = T (m/M)^r, tau_m = t_m - t_{m-1}
(Sec. 2.1); g = 1/Gamma(1-gamma) is the Caputo prefactor (the printed
1/Gamma(gamma-1) in (1.2) is read as 1/Gamma(1-gamma), as in the discrete L1
formula of Sec. 2.1).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla


# ---------------------------------------------------------------- constants
def c1_alpha(alpha: float) -> float:
    """Normalisation constant c_{1,alpha} of the IFL definition (1.4)."""
    return (2.0 ** (alpha - 1) * alpha * math.gamma((alpha + 1) / 2)
            / (math.sqrt(math.pi) * math.gamma(1 - alpha / 2)))


# ---------------------------------------------------------------- time mesh
def graded_mesh(T: float, M: int, r: float) -> np.ndarray:
    """Graded time levels t_m = T (m/M)^r, m = 0..M (Sec. 2.1)."""
    return T * (np.arange(M + 1, dtype=np.float64) / M) ** r


def _gap(T, M, r, m, j):
    """t_m - t_j for 0 <= j < m, without cancellation.

    t_m - t_j = T (m/M)^r (1 - (j/m)^r) and 1 - (j/m)^r is evaluated as
    -expm1(r log1p(-(m-j)/m)); the naive difference of two nearby t values
    loses log10(t_m / (t_m - t_j)) digits, which is 13 digits for the first
    interval of a strongly graded mesh.
    """
    if j == 0:
        return T * (m / M) ** r
    return -T * (m / M) ** r * math.expm1(r * math.log1p(-(m - j) / m))


def step_sizes(T: float, M: int, r: float) -> np.ndarray:
    """tau_m = t_m - t_{m-1}, m = 1..M (index m-1)."""
    return np.array([_gap(T, M, r, m, m - 1) for m in range(1, M + 1)])


def l1_weights(T: float, M: int, r: float, gamma: float, m: int) -> np.ndarray:
    """Graded-L1 weights a_k^{(m)} = (1/tau_k) int_{t_{k-1}}^{t_k} (t_m - s)^{-gamma} ds
    for k = 1..m (eq. (2.8)); returned with index k-1.

    The integral is (A^{1-g} - B^{1-g}) / (1-g) with A = t_m - t_{k-1},
    B = t_m - t_k = A - tau_k; it is evaluated as
    A^{1-g} (1 - (1 - tau_k/A)^{1-g}) / ((1-g) tau_k) with expm1/log1p so that
    short intervals far from t_m keep full relative accuracy.
    """
    g1 = 1.0 - gamma
    out = np.empty(m)
    for k in range(1, m + 1):
        tau_k = _gap(T, M, r, k, k - 1)
        A = _gap(T, M, r, m, k - 1)
        if k == m:
            out[k - 1] = tau_k ** (-gamma) / g1
        else:
            frac = -math.expm1(g1 * math.log1p(-tau_k / A))
            out[k - 1] = A ** g1 * frac / (g1 * tau_k)
    return out


# ---------------------------------------------------------------- IFL matrix
def _mu_params(alpha, mu):
    mu = 1.0 + alpha / 2 if (mu is None or mu <= 0) else mu
    kmu = 2.0 if mu == 2.0 else 1.0
    return mu, mu - alpha, kmu


def ifl_column(n: int, alpha: float, l: float = 1.0, mu: float | None = None) -> np.ndarray:
    """First column (a_{11}, a_{21}, ..., a_{n1}) of the IFL matrix A, eq. (3.16x).

    C^h = c_{1,alpha} / (nu h^alpha), nu = mu - alpha, kappa_mu = 2 if mu = 2
    else 1 (Sec. 2.1, after (2.11)).  Diagonal:
      C^h [ sum_{l=2}^{N_p-1} ((l+1)^nu - (l-1)^nu)/l^mu + (N_p^nu - (N_p-1)^nu)/N_p^mu
            + (2^nu + kappa_mu - 1) + 2 nu / (alpha N_p^alpha) ],
    first off-diagonal -C^h (2^nu + kappa_mu - 1)/2, and distance d >= 2:
    -C^h ((d+1)^nu - (d-1)^nu) / (2 d^mu).
    """
    Np = n + 1
    h = 2.0 * l / Np
    mu, nu, kmu = _mu_params(alpha, mu)
    Ch = c1_alpha(alpha) / (nu * h ** alpha)
    ell = np.arange(2, Np, dtype=np.float64)
    diag = (np.sum(((ell + 1) ** nu - (ell - 1) ** nu) / ell ** mu)
            + (Np ** nu - (Np - 1) ** nu) / Np ** mu
            + (2.0 ** nu + kmu - 1.0)
            + 2.0 * nu / (alpha * Np ** alpha))
    col = np.empty(n)
    col[0] = Ch * diag
    if n > 1:
        col[1] = -Ch * (2.0 ** nu + kmu - 1.0) / 2.0
    if n > 2:
        d = np.arange(2, n, dtype=np.float64)
        col[2:] = -Ch * ((d + 1) ** nu - (d - 1) ** nu) / (2.0 * d ** mu)
    return col


def ifl_matrix(n: int, alpha: float, l: float = 1.0, mu: float | None = None) -> np.ndarray:
    """Dense symmetric Toeplitz A of eq. (3.16x)."""
    return sla.toeplitz(ifl_column(n, alpha, l, mu))


def strang_column(col: np.ndarray) -> np.ndarray:
    """First column c_S of Strang's circulant s(A) (Sec. 4.1, after (4.3)).

    The n-periodic circulant keeps the central diagonals of A: entry j of c_S
    is a_{1,j+1} for j <= floor(n/2) and a_{1,n-j+1} otherwise, i.e. the
    distance min(j, n-j) diagonal.
    """
    n = col.shape[0]
    j = np.arange(n)
    return col[np.minimum(j, n - j)]


# ---------------------------------------------------------------- DIDS solve
def _kappa_row(kappa, m):
    return kappa[m - 1] if kappa.ndim == 2 else kappa


def dids_solve(alpha, gamma, n, M, r, kappa, f, phi, l=1.0, T=1.0, mu=None, matrix=None):
    """Direct implicit difference scheme, matrix form (4.1), dense LU per level.

    For m = 1..M:
      rhs = g [a_1^{(m)} u^0 + sum_{k=1}^{m-1} (a_{k+1}^{(m)} - a_k^{(m)}) u^k] + f^m
      (g a_m^{(m)} I + K^{(m)} A) u^m = rhs,   K^{(m)} = diag(kappa(x_i, t_m)).
    The solve is LAPACK gesv (the paper's direct solver is MATLAB's backslash).
    A is the matrix of eq. (3.16x), or `matrix` when given (the 2-D operator of
    ``oracle.ifl2d``, n then being the number of unknowns).
    Returns U with U[m] = u^m, m = 0..M.
    """
    A = ifl_matrix(n, alpha, l, mu) if matrix is None else matrix
    g = 1.0 / math.gamma(1.0 - gamma)
    U = np.empty((M + 1, n))
    U[0] = phi
    for m in range(1, M + 1):
        a = l1_weights(T, M, r, gamma, m)
        rhs = g * a[0] * U[0]
        if m > 1:
            rhs = rhs + g * (np.diff(a)[: m - 1] @ U[1:m])
        rhs = rhs + f[m - 1]
        Mm = _kappa_row(kappa, m)[:, None] * A
        Mm[np.diag_indices(n)] += g * a[m - 1]
        U[m] = sla.solve(Mm, rhs)
    return U


def dids_adjoint(alpha, gamma, n, M, r, kappa, f, phi, dJ_duM, U=None,
                 l=1.0, T=1.0, mu=None, matrix=None):
    """Exact discrete adjoint of ``dids_solve`` for a loss J(u^M).

    Backward over m = M..1 with ubar^m complete on arrival:
      lambda^m = (M^{(m)})^{-T} ubar^m
      dJ/df^m    = lambda^m
      dJ/dkappa^m_i = -lambda^m_i (A u^m)_i     (summed over m if kappa is [n])
      ubar^0 += g a_1^{(m)} lambda^m,  ubar^k += g (a_{k+1}^{(m)} - a_k^{(m)}) lambda^m
    and dJ/dphi = ubar^0.  Returns (g_kappa, g_f, g_phi).  `matrix` as in
    ``dids_solve``.
    """
    if U is None:
        U = dids_solve(alpha, gamma, n, M, r, kappa, f, phi, l, T, mu, matrix)
    A = ifl_matrix(n, alpha, l, mu) if matrix is None else matrix
    g = 1.0 / math.gamma(1.0 - gamma)
    ubar = np.zeros((M + 1, n))
    ubar[M] = dJ_duM
    g_f = np.zeros((M, n))
    g_k = np.zeros_like(kappa)
    for m in range(M, 0, -1):
        a = l1_weights(T, M, r, gamma, m)
        Mm = _kappa_row(kappa, m)[:, None] * A
        Mm[np.diag_indices(n)] += g * a[m - 1]
        lam = sla.solve(Mm.T, ubar[m])
        g_f[m - 1] = lam
        contrib = -lam * (A @ U[m])
        if kappa.ndim == 2:
            g_k[m - 1] = contrib
        else:
            g_k += contrib
        ubar[0] += g * a[0] * lam
        if m > 1:
            ubar[1:m] += g * np.outer(np.diff(a)[: m - 1], lam)
    return g_k, g_f, ubar[0].copy()


# ---------------------------------------------------------------- errors
def errors(U: np.ndarray, exact: np.ndarray, l: float = 1.0):
    """Err_inf = max_m ||E^m||_inf and Err_2 = max_m (h sum_i (E^m_i)^2)^{1/2}
    over m = 0..M (Sec. 5); the boundary nodes carry zero error."""
    n = U.shape[1]
    h = 2.0 * l / (n + 1)
    E = U - exact
    return float(np.max(np.abs(E))), float(np.max(np.sqrt(h * np.sum(E * E, axis=1))))


# ---------------------------------------------------------------- SOE checks
def soe_relative_error(s, w, gamma, delta, T, npts=4000):
    """max over a log grid of [delta, T] of |t^gamma sum_j w_j e^{-s_j t} - 1|
    (Lemma 2.2, read as a relative bound; the grid includes both ends)."""
    t = np.exp(np.linspace(math.log(delta), math.log(T), npts))
    approx = np.exp(-np.outer(t, s)) @ w
    return float(np.max(np.abs(approx * t ** gamma - 1.0)))


def fids_history_weights(s, w, T, M, r, m):
    """b_k^{(m)} for k = 1..m-1 from its definition in Sec. 2.1 (after (2.9)):
    b_k^{(m)} = sum_j w_j (1/tau_k) int_{t_{k-1}}^{t_k} e^{-s_j (t_m - s)} ds,
    evaluated in closed form e^{-s_j (t_m - t_k)} (1 - e^{-s_j tau_k}) / (s_j tau_k)."""
    out = np.empty(m - 1)
    for k in range(1, m):
        tau_k = _gap(T, M, r, k, k - 1)
        B = _gap(T, M, r, m, k) if k < m else 0.0
        x = s * tau_k
        out[k - 1] = np.sum(w * np.exp(-s * B) * (-np.expm1(-x)) / x)
    return out
