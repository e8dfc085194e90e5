"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/fids.h, validates parameters, and its host-side set-up
tables agree with the oracle's definitions (IFL column of eq. (3.16x), level
coefficients g a_m^{(m)} of Sec. 2.1, Strang eigenvalues of eq. (4.3), SOE
accuracy of Lemma 2.2)."""
import ctypes
import math

import numpy as np
import pytest

import oracle
from paper_2002_11978_amd import fids

ROOT = __import__("os").path.dirname(__import__("os").path.dirname(__import__("os").path.abspath(__file__)))


def test_library_exports_every_declared_function():
    L = fids.lib()
    names = fids.header_functions()
    assert len(names) >= 19 and "fids_strerror" in names
    for name in names:
        assert hasattr(L, name), name


def test_strerror_and_defaults():
    assert fids.strerror(0) == "ok"
    p = fids.default_params()
    assert p.alpha == 1.5 and p.n == 255 and p.solver == fids.FIDS_BICGSTAB


@pytest.mark.parametrize("field,value", [
    ("alpha", 0.0), ("alpha", 2.0), ("gamma", 0.0), ("gamma", 1.0), ("r", 0.5), ("n", 0), ("M", 0),
    ("l", 0.0), ("T", -1.0), ("krylov_tol", 0.0), ("soe_tol", 1.5), ("restart", 0), ("restart", 33),
    ("mu", 1.4), ("solver", 7), ("precision", 3), ("precond", 9), ("x0_mode", 4), ("soe_helpers", -2),
    ("n", (1 << 21) + 1),
])
def test_invalid_parameters_rejected(field, value):
    p = fids.default_params(**{field: value})
    sz = ctypes.c_size_t(0)
    assert fids.lib().fids_workspace_size(ctypes.byref(p), ctypes.byref(sz)) == fids.FIDS_EINVAL


def test_solver_precision_combinations():
    sz = ctypes.c_size_t(0)
    for solver, precision, ok in [(0, 0, True), (1, 0, True), (2, 0, True), (1, 1, True),
                                  (0, 1, False), (2, 1, False), (3, 0, False)]:
        p = fids.default_params(solver=solver, precision=precision)
        st = fids.lib().fids_workspace_size(ctypes.byref(p), ctypes.byref(sz))
        assert (st == fids.FIDS_OK) == ok, (solver, precision, st)


def test_null_pointers_rejected():
    L = fids.lib()
    p = fids.default_params()
    h = ctypes.c_void_p(0)
    assert L.fids_init_problem(ctypes.byref(p), None, None, None, None, 0, None, ctypes.byref(h)) == fids.FIDS_EINVAL
    assert L.fids_workspace_size(None, None) == fids.FIDS_EINVAL
    assert L.fids_step(None, None, None) == fids.FIDS_EINVAL
    assert L.fids_destroy(None) == fids.FIDS_OK


def test_workspace_size_grows_with_problem():
    a = fids.workspace_size(fids.default_params(n=255, M=64))
    b = fids.workspace_size(fids.default_params(n=4095, M=512))
    assert a % 256 == 0 and b > a


@pytest.mark.parametrize("alpha,mu", [(0.5, 0.0), (1.5, 0.0), (1.9, 0.0), (1.6, 2.0)])
@pytest.mark.parametrize("n", [1, 2, 7, 255, 1000])
def test_ifl_column_matches_oracle(alpha, mu, n):
    got = fids.ifl_column(n, alpha, 1.0, mu)
    ref = oracle.ifl_column(n, alpha, 1.0, mu or None)
    # The oracle forms (d+1)^nu - (d-1)^nu as the plain difference of eq.
    # (3.16x); the library uses d^nu (expm1(nu log1p(1/d)) - expm1(nu log1p(-1/d))).
    # The two powers are about d^nu and differ by about 2 nu d^(nu-1), so the
    # plain difference carries a relative rounding error of about
    # u d^nu / (2 nu d^(nu-1)) = u d / (2 nu) (u = 2^-53): at nu = mu - alpha
    # = 0.05 (alpha = 1.9) that is 1.1e-15 d.  The tolerance 1e-13 max(1, d)
    # covers it with a margin of 90 for every nu >= 0.05 tested here.
    tol = 1e-13 * np.maximum(1.0, np.arange(n))
    assert np.all(np.abs(got - ref) <= tol * np.abs(ref) + 1e-15 * abs(ref[0]))


@pytest.mark.parametrize("gamma,r,M", [(0.5, 3.0, 64), (0.4, 4.0, 2048), (0.3, (2 - 0.3) / 0.3, 512)])
def test_level_coefficients_match_l1_weights(gamma, r, M):
    beta = fids.level_coefficients(gamma, 1.0, M, r)
    g = 1.0 / math.gamma(1 - gamma)
    for m in (1, 2, M // 2, M):
        a = oracle.l1_weights(1.0, M, r, gamma, m)
        assert beta[m - 1] == pytest.approx(g * a[m - 1], rel=1e-13)


@pytest.mark.parametrize("n", [1, 3, 63, 255, 1000, 4095])
@pytest.mark.parametrize("alpha", [0.5, 1.5, 1.9])
def test_strang_eigs_match_fft(n, alpha):
    lam = fids.strang_eigs(n, alpha)
    ref = np.fft.fft(oracle.strang_column(oracle.ifl_column(n, alpha))).real
    assert np.max(np.abs(lam - ref)) <= 1e-12 * np.max(np.abs(ref))
    col0 = oracle.ifl_column(n, alpha)[0]
    assert np.all(lam > 0) and np.all(lam < 2 * col0)          # Lemma 4.1


@pytest.mark.parametrize("gamma,delta,tol", [
    (0.5, (1 / 64) ** 3, 1e-10),        # closed-form workload, M = 64, r = 3
    (0.4, 2048.0 ** -4, 1e-10),         # M = 2048, r = 4
    (0.2, 256.0 ** -9, 1e-10),          # strongest grading of the batch recipe
    (0.8, 1e-3, 1e-12),
    (0.5, 1.0, 1e-10),                  # M = 1: the interval is the single point T
])
def test_soe_nodes_accuracy(gamma, delta, tol):
    s, w = fids.soe_nodes(gamma, delta, 1.0, tol)
    assert np.all(s > 0) and np.all(w > 0)
    err = oracle.soe_relative_error(s, w, gamma, min(delta, 1.0), 1.0, npts=20000)
    assert err <= tol * 1.05, err
    assert len(s) < 400


def test_single_hip_runtime_in_process():
    """The binding loads torch's HIP runtime before the library, so only one
    HIP (and HSA) runtime is mapped into the process."""
    import subprocess
    import sys
    code = ("from paper_2002_11978_amd import fids; fids.default_params();"
            "maps = open('/proc/self/maps').read();"
            "print(len({l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, check=True)
    assert out.stdout.strip() == "1"


def _batch_params(count=256, M=256):
    from paper_2002_11978_amd import workloads as W
    return [fids.default_params(alpha=a, gamma=g, n=n, M=M, r=(2 - g) / g)
            for n, a, g in W.batch_shapes(count)]


def _embed(n):
    L = 4
    while L < 2 * n:
        L *= 2
    return L


@pytest.mark.parametrize("resident", [1, 7, 64, 256, 1024])
def test_batch_plan_is_a_valid_placement(resident):
    """Every member is placed once; groups of more than one workgroup hold one
    member; the workgroups used fit `resident`; the modelled makespan is at
    least the obvious lower bounds and within 1.5x of the larger one."""
    ps = _batch_params()
    ng, slot, mk = fids.batch_plan(ps, resident)
    slots = {}
    for i, s in enumerate(slot):
        slots.setdefault(s, []).append(i)
    used = 0
    for s, members in slots.items():
        sizes = {ng[i] for i in members}
        assert len(sizes) == 1
        k = sizes.pop()
        if k > 1:
            assert len(members) == 1
        used += k
    assert used <= max(resident, 1)
    cost = [_embed(p.n) for p in ps]
    if resident >= 2:
        assert mk >= sum(cost) / resident - 1e-9
    assert mk >= max(c / 64 for c in cost)
    if resident >= 64:
        lower = max(sum(cost) / resident, max(min(c / k + (260 + 12 * k if k > 1 else 0)
                                                  for k in (1, 2, 4, 8, 16, 32, 64) if k * 1024 <= c // 2 or k == 1)
                                              for c in cost))
        assert mk <= 1.5 * lower


def test_batch_plan_single_workgroup_packs_everything():
    ps = _batch_params(12)
    ng, slot, mk = fids.batch_plan(ps, 1)
    assert ng == [1] * 12 and len(set(slot)) == 1
    assert mk == pytest.approx(sum(_embed(p.n) for p in ps))


@pytest.mark.parametrize("M,r,gamma,m", [(25268, 3.0, 0.8, 25268), (25268, 3.0, 0.8, 9000),
                                         (12855, 2.0, 0.5, 12855), (64, 1.0, 0.3, 40)])
def test_direct_weights_against_extended_precision(M, r, gamma, m):
    """Direct-scheme weights (eq. 4.1) against the L1 integrals evaluated in
    40-digit arithmetic, on the strongest gradings of the paper's Table 11,
    where a naive t_m - t_k - tau_k residue would spoil the last interval."""
    import mpmath
    mpmath.mp.dps = 40
    w = fids.direct_weights(gamma, 1.0, M, r, m)
    t = lambda j: (mpmath.mpf(j) / M) ** r
    nu = 1 - mpmath.mpf(gamma)
    g = 1 / mpmath.gamma(1 - mpmath.mpf(gamma))
    a = lambda k: ((t(m) - t(k - 1)) ** nu - (t(m) - t(k)) ** nu) / (nu * (t(k) - t(k - 1)))
    # w_k = g (a_{k+1} - a_k) of two nearly equal integrals is exact to the
    # rounding of a_k itself (about 1e-16 of g a_k, far below the sum of the row)
    scale = float(g * a(m))
    for k in sorted({0, 1, 2, m // 2, m - 2, m - 1}):
        if k < 0 or k >= m:
            continue
        exact = g * a(1) if k == 0 else g * (a(k + 1) - a(k))
        ak = float(g * a(max(k, 1)))
        assert abs(w[k] - float(exact)) <= 1e-9 * abs(float(exact)) + 1e-14 * ak, (k, w[k], float(exact))
    assert abs(float(np.sum(w)) - float(g * a(m))) <= 1e-12 * scale + 1e-12


# ---------------------------------------------------------------- 2-D operator
@pytest.mark.parametrize("alpha", [0.1, 0.7, 1.3, 1.9])
def test_ifl2d_mu_matches_oracle(alpha):
    """The library's splitting exponent mu*(alpha) (its own cell quadrature and
    root finding) against the oracle's (closed-form cell integrals)."""
    assert fids.ifl2d_mu(alpha) == pytest.approx(oracle.mu_star(alpha), abs=1e-9)


@pytest.mark.parametrize("n", [1, 2, 15, 64])
@pytest.mark.parametrize("alpha", [0.4, 1.5, 1.95])
def test_ifl2d_coefficients_match_oracle(n, alpha):
    """Block-Toeplitz coefficients a[p, q] of the 2-D matrix at the same mu:
    the two sides integrate the cells differently (Gauss-Legendre against
    hypergeometric closed forms), so agreement is to quadrature accuracy."""
    mu = oracle.mu_star(alpha)
    got = fids.ifl2d_coefficients(n, alpha, 1.3, mu)
    ref = oracle.ifl2d_coefficients(n, alpha, 1.3, mu)
    assert np.max(np.abs(got - ref)) <= 1e-11 * abs(ref[0, 0])
    # default mu: the library's own mu*, within its root's tolerance
    d = fids.ifl2d_coefficients(n, alpha, 1.3, 0.0)
    assert np.max(np.abs(d - ref)) <= 1e-8 * abs(ref[0, 0])


@pytest.mark.parametrize("field,value", [("dims", 0), ("dims", 3), ("mu", 2.0), ("mu", 0.5), ("n", 2049)])
def test_invalid_2d_parameters_rejected(field, value):
    kw = dict(dims=2, n=31, alpha=1.5)
    kw[field] = value
    p = fids.default_params(**kw)
    sz = ctypes.c_size_t(0)
    assert fids.lib().fids_workspace_size(ctypes.byref(p), ctypes.byref(sz)) == fids.FIDS_EINVAL


def test_2d_layout_lengths():
    p = fids.default_params(dims=2, n=255)
    assert fids.natural_len(p) == 255 * 255
    assert fids.toeplitz_len(p) == 512 * 254 + 255
    assert fids.workspace_size(p) > fids.workspace_size(fids.default_params(n=255))
