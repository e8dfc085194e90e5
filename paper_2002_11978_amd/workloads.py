"""Seeded synthetic inputs for the time-space fractional diffusion problem (1.1).

This module only evaluates problem data -- the diffusivity kappa(x, t), the
source f(x, t), the initial value phi(x) and, where one exists, the exact
solution -- at the spatial nodes x_i = -l + i h (i = 1..n, h = 2l/(n+1)) and
the time levels t_m = T (m/M)^r where the equation is sampled (Sec. 2.1).
It holds none of the scheme's arithmetic (no L1 weights, no IFL matrix, no
solver): both the CPU oracle and the GPU path take the arrays it returns.

Array conventions (shared by every consumer):
  kappa  : [M, n] with row m-1 = kappa(x_i, t_m)   (time dependent), or [n]
  f      : [M, n] with row m-1 = f(x_i, t_m)
  phi    : [n]
  exact  : [M+1, n] with row m = u(x_i, t_m)     (when a closed form exists)

Workloads:
  * ``example1`` / ``example2``: the manufactured solutions of Sec. 5,
    u = (1-x^2)_+^{s+alpha/2} (t^gamma + 1), with the closed-form fractional
    Laplacian of (1-x^2)_+^{s+alpha/2} (a terminating 2F1 for integer s).
  * ``closed_form_s0``: the s = 0 member of that family, whose fractional
    Laplacian is the constant 2^alpha Gamma(1+alpha/2) Gamma((1+alpha)/2) /
    Gamma(1/2) on (-1, 1).
  * ``seeded``: smooth random fields -- kappa from 8 random Fourier modes
    (clipped below at 0.1), f from 16 random modes, phi = (1-x^2)^{alpha/2}.
    These are a stand-in recipe, not taken from the paper.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def node_coords(n: int, l: float = 1.0) -> np.ndarray:
    """Interior nodes x_i = -l + i h, i = 1..n, h = 2l/(n+1)."""
    h = 2.0 * l / (n + 1)
    return -l + h * np.arange(1, n + 1, dtype=np.float64)


def time_levels(T: float, M: int, r: float) -> np.ndarray:
    """Graded time levels t_m = T (m/M)^r, m = 0..M."""
    return T * (np.arange(M + 1, dtype=np.float64) / M) ** r


def default_grading(gamma: float) -> float:
    """r = (2-gamma)/gamma, which makes min{r gamma, 2-gamma} = 2-gamma."""
    return (2.0 - gamma) / gamma


def ifl_of_bump(x: np.ndarray, alpha: float, s: int) -> np.ndarray:
    """Closed form of (-Delta)^{alpha/2} (1-x^2)_+^{s+alpha/2} on |x| < 1.

    Equals 2^alpha Gamma((alpha+1)/2) Gamma(s+1+alpha/2) / (sqrt(pi) Gamma(s+1))
    times 2F1((alpha+1)/2, -s; 1/2; x^2); for integer s >= 0 the 2F1 series
    stops after s+1 terms.
    """
    pref = (2.0 ** alpha * math.gamma((alpha + 1) / 2) * math.gamma(s + 1 + alpha / 2)
            / (math.sqrt(math.pi) * math.gamma(s + 1)))
    a, b, c = (alpha + 1) / 2, -s, 0.5
    z = x * x
    total = np.zeros_like(x)
    term = np.ones_like(x)
    for k in range(s + 1):
        total = total + term
        term = term * (a + k) * (b + k) / ((c + k) * (k + 1)) * z
    return pref * total


@dataclass
class Problem:
    """One instance of (1.1) sampled on the grid, plus its discretisation knobs."""
    alpha: float
    gamma: float
    n: int
    M: int
    r: float
    l: float = 1.0
    T: float = 1.0
    mu: float = 0.0            # 0 selects mu = 1 + alpha/2
    kappa: np.ndarray | None = None
    f: np.ndarray | None = None
    phi: np.ndarray | None = None
    exact: np.ndarray | None = None
    kappa_time_dependent: bool = True
    name: str = ""
    dims: int = 1              # 2: n nodes per axis of (-l, l)^2, fields flattened x-fastest (i + n j)

    @property
    def mu_eff(self) -> float:
        return self.mu if self.mu > 0 else 1.0 + self.alpha / 2


def _manufactured(alpha, gamma, n, M, r, s, kappa_fn, mu=0.0, name=""):
    x = node_coords(n, 1.0)
    t = time_levels(1.0, M, r)
    bump = np.maximum(1.0 - x * x, 0.0) ** (s + alpha / 2)
    lap = ifl_of_bump(x, alpha, s)
    X, Tm = np.meshgrid(x, t[1:], indexing="xy")          # [M, n]
    kap = kappa_fn(X, Tm)
    f = math.gamma(1 + gamma) * bump[None, :] + kap * lap[None, :] * (Tm ** gamma + 1.0)
    exact = bump[None, :] * (t[:, None] ** gamma + 1.0)
    return Problem(alpha, gamma, n, M, r, 1.0, 1.0, mu, np.ascontiguousarray(kap),
                   np.ascontiguousarray(f), bump.copy(), exact, True, name)


def example1(alpha, gamma, r, Np, M, s=3, mu=0.0) -> Problem:
    """Example 1: kappa = (1+t) e^{0.8x+1}, s = 3; Np = number of intervals."""
    return _manufactured(alpha, gamma, Np - 1, M, r, s,
                         lambda X, Tm: (1.0 + Tm) * np.exp(0.8 * X + 1.0), mu, "example1")


def example2(alpha, gamma, r, Np, M, s=1, mu=0.0) -> Problem:
    """Example 2: kappa = 7 [ln(5+2x+t) + cos(xt)] / 4, s = 1."""
    return _manufactured(alpha, gamma, Np - 1, M, r, s,
                         lambda X, Tm: 7.0 * (np.log(5.0 + 2.0 * X + Tm) + np.cos(X * Tm)) / 4.0,
                         mu, "example2")


def closed_form_s0(alpha=1.5, gamma=0.5, n=255, M=64, r=None) -> Problem:
    """kappa = 1 + 0.5 sin(pi x) e^{-t}; exact u = (1+t^gamma)(1-x^2)^{alpha/2}."""
    r = default_grading(gamma) if r is None else r
    return _manufactured(alpha, gamma, n, M, r, 0,
                         lambda X, Tm: 1.0 + 0.5 * np.sin(np.pi * X) * np.exp(-Tm), 0.0,
                         "closed_form_s0")


def _kappa_modes(seed: int, time_dependent: bool):
    g = np.random.Generator(np.random.PCG64(seed))
    A = g.normal(0.0, 0.2, 8)
    k = g.integers(1, 5, 8)
    w = g.integers(0, 3, 8) if time_dependent else np.zeros(8, dtype=np.int64)
    th = g.uniform(0.0, 2 * np.pi, 8)
    return A, k, w, th


def _f_modes(seed: int):
    g = np.random.Generator(np.random.PCG64(seed))
    k = g.integers(1, 9, 16)
    B = g.normal(0.0, 1.0, 16) / k
    w = g.integers(0, 4, 16)
    ps = g.uniform(0.0, 2 * np.pi, 16)
    return B, k, w, ps


def seeded_kappa(x, t_levels, seed, time_dependent=True):
    """kappa = max(0.1, 1 + 0.5 sum_q A_q cos(pi k_q x + pi w_q t + theta_q)).

    Evaluated as a sum of separable products so that [M, n] fields cost one
    small matrix product.  Returns [M, n] (rows t_1..t_M) or [n].
    """
    A, k, w, th = _kappa_modes(seed, time_dependent)
    cx = np.cos(np.pi * np.outer(k, x))                  # [8, n]
    sx = np.sin(np.pi * np.outer(k, x))
    if not time_dependent:
        val = 1.0 + 0.5 * ((A * np.cos(th)) @ cx - (A * np.sin(th)) @ sx)
        return np.maximum(val, 0.1)
    ph = np.pi * np.outer(t_levels, w) + th[None, :]      # [M, 8]
    val = 1.0 + 0.5 * ((np.cos(ph) * A) @ cx - (np.sin(ph) * A) @ sx)
    return np.maximum(val, 0.1)


def seeded_source(x, t_levels, seed):
    """f = sum_q B_q sin(pi k_q (x+1)/2) cos(pi w_q t + psi_q), [M, n]."""
    B, k, w, ps = _f_modes(seed)
    sx = np.sin(np.pi * np.outer(k, x + 1.0) / 2.0)          # [16, n]
    ct = np.cos(np.pi * np.outer(t_levels, w) + ps[None, :])  # [M, 16]
    return (ct * B) @ sx


def seeded(alpha, gamma, n, M, r=None, kappa_seed=1, f_seed=2,
           time_dependent=True, name="seeded") -> Problem:
    """Seeded smooth-field workload; phi = (1-x^2)^{alpha/2}."""
    r = default_grading(gamma) if r is None else r
    x = node_coords(n, 1.0)
    t = time_levels(1.0, M, r)[1:]
    kap = seeded_kappa(x, t, kappa_seed, time_dependent)
    f = seeded_source(x, t, f_seed)
    phi = np.maximum(1.0 - x * x, 0.0) ** (alpha / 2)
    return Problem(alpha, gamma, n, M, r, 1.0, 1.0, 0.0, np.ascontiguousarray(kap),
                   np.ascontiguousarray(f), phi, None, time_dependent, name)


def seeded2d(alpha, gamma, n, M, r=None, kappa_seed=1, f_seed=2,
             time_dependent=True, name="seeded2d") -> Problem:
    """Seeded smooth fields on the square (-1, 1)^2, n nodes per axis
    (dims = 2), flattened x-fastest (node (i, j) at i + n j):
    kappa(x, y, t) = (k_a(x, t) + k_b(y, t)) / 2 from two seeded 1-D kappa
    fields (>= 0.1), f(x, y, t) = s_a(x, t) g(y) + g(x) s_b(y, t) with two
    seeded 1-D sources and g(z) = sin(pi (z + 1)/2), and the non-smooth
    initial datum phi = (1 - x^2 - y^2)_+^{alpha/2}."""
    r = default_grading(gamma) if r is None else r
    x = node_coords(n, 1.0)
    t = time_levels(1.0, M, r)[1:]
    ka = seeded_kappa(x, t, kappa_seed, time_dependent)
    kb = seeded_kappa(x, t, kappa_seed + 7919, time_dependent)
    if time_dependent:
        kap = 0.5 * (ka[:, None, :] + kb[:, :, None])            # [M, y, x]
        kap = kap.reshape(M, n * n)
    else:
        kap = (0.5 * (ka[None, :] + kb[:, None])).reshape(n * n)
    g = np.sin(np.pi * (x + 1.0) / 2.0)
    sa = seeded_source(x, t, f_seed)
    sb = seeded_source(x, t, f_seed + 7919)
    f = (sa[:, None, :] * g[None, :, None] + g[None, None, :] * sb[:, :, None]).reshape(M, n * n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    phi = (np.maximum(1.0 - X * X - Y * Y, 0.0) ** (alpha / 2)).reshape(n * n)
    return Problem(alpha, gamma, n, M, r, 1.0, 1.0, 0.0, np.ascontiguousarray(kap),
                   np.ascontiguousarray(f), phi, None, time_dependent, name, dims=2)


def batch_shapes(count=256, seed0=1000, n_lo=511, n_hi=16383):
    """Per-problem (n, alpha, gamma) for a heterogeneous batch.

    n is drawn log-uniformly in [n_lo, n_hi] and rounded to an integer,
    alpha ~ U(1.1, 1.9), gamma ~ U(0.2, 0.8), one generator per problem.
    """
    out = []
    for p in range(count):
        g = np.random.Generator(np.random.PCG64(seed0 + p))
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        alpha = float(g.uniform(1.1, 1.9))
        gamma = float(g.uniform(0.2, 0.8))
        out.append((n, alpha, gamma))
    return out


def batch_member(p: int, M: int = 256, count_seed0: int = 1000, kappa_seed0: int = 2000,
                 f_seed0: int = 3000, n_lo: int = 511, n_hi: int = 16383) -> Problem:
    """Member p of the heterogeneous batch: (n, alpha, gamma) from
    batch_shapes, grading r = (2 - gamma)/gamma, kappa seed 2000 + p, f seed
    3000 + p."""
    g = np.random.Generator(np.random.PCG64(count_seed0 + p))
    n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
    alpha = float(g.uniform(1.1, 1.9))
    gamma = float(g.uniform(0.2, 0.8))
    return seeded(alpha, gamma, n, M, kappa_seed=kappa_seed0 + p, f_seed=f_seed0 + p,
                  name=f"batch[{p}]")
