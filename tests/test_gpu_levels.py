"""GPU tests of stepping through windows of levels (fids_solve_levels) and of
the per-level acceptance flags, and of the per-level symbols built on a
second stream while the levels run.

Advancing a problem in windows of levels runs the same kernels over the same
levels as one launch over all of them, so the states and level reports must
agree bit for bit.  A level whose FP64 true residual stalls above the
tolerance is accepted only within the residual's rounding level (flag
FIDS_LEVEL_ABOVE_TOL); with that allowance switched off from the host
(FIDS_FLOOR_SCALE=0) the same level reports FIDS_ENOCONV.
"""
import os

import numpy as np
import pytest

from paper_2002_11978_amd import fids
from paper_2002_11978_amd import workloads as W

from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

FORMS = [
    pytest.param(dict(solver=2, x0_mode=3), id="pcg-x0cubic"),
    pytest.param(dict(solver=1, x0_mode=3), id="fgmres-x0cubic"),
    pytest.param(dict(solver=0, x0_mode=0), id="bicgstab-x0zero"),
    pytest.param(dict(solver=1, x0_mode=3, precision=1), id="mixed-x0cubic"),
]


def _problem(pb, **kw):
    params = fids.default_params(alpha=pb.alpha, gamma=pb.gamma, n=pb.n, M=pb.M, r=pb.r,
                                 kappa_time_dependent=1, krylov_maxit=500)
    for k, v in kw.items():
        setattr(params, k, v)
    return fids.Problem(params, to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi))


def _key(r):
    return (r.m, r.iters, r.matvecs, r.relres, r.pc_fp64_iters, r.flags)


@pytest.mark.parametrize("kw", FORMS)
def test_windows_equal_one_launch(kw):
    pb = W.seeded(1.5, 0.4, 4095, 40, r=4.0, kappa_seed=3, f_seed=4)
    say(f"[levels] windows n={pb.n} M={pb.M} {kw}")
    prob = _problem(pb, krylov_tol=1e-10, **kw)
    uT, _, reps = prob.solve_all()
    ref = uT.cpu().numpy()
    ref_keys = [_key(r) for r in reps]
    for split in ([1] * 5 + [35], [7, 13, 20], [39, 1]):
        prob.reset()
        got = []
        for c in split:
            u, rs = prob.solve_levels(c)
            got += [_key(r) for r in rs]
        assert np.array_equal(u.cpu().numpy(), ref), split
        assert got == ref_keys, split
    # single steps through fids_step give the same states and reports too
    prob.reset()
    got = []
    for _ in range(pb.M):
        u, r = prob.step()
        got.append(_key(r))
    assert np.array_equal(u.cpu().numpy(), ref)
    assert got == ref_keys
    # out-of-range counts and stepping past level M
    prob.reset()
    assert fids.lib().fids_solve_levels(prob.h, 0, None, None) == fids.FIDS_EINVAL
    assert fids.lib().fids_solve_levels(prob.h, pb.M + 1, None, None) == fids.FIDS_EINVAL
    assert prob.solve_levels_raw(pb.M) == fids.FIDS_OK
    assert prob.solve_levels_raw(1) == fids.FIDS_ESTATE
    prob.close()


@pytest.mark.parametrize("kw", FORMS)
def test_flags_mark_levels_above_tolerance(kw):
    pb = W.seeded(1.5, 0.4, 4095, 24, r=4.0, kappa_seed=3, f_seed=4)
    tol = 1e-10
    prob = _problem(pb, krylov_tol=tol, **kw)
    _, _, reps = prob.solve_all()
    for r in reps:
        above = bool(r.flags & fids.FIDS_LEVEL_ABOVE_TOL)
        assert above == (r.relres > tol), (r.m, r.relres, r.flags)
    prob.close()


@pytest.mark.parametrize("solver", [2, 1], ids=["pcg", "fgmres"])
def test_stalled_residual_accepted_only_within_rounding_level(solver):
    # a tolerance below the FP64 floor of these systems: the true residual
    # stalls above it, so each level is accepted at its rounding level
    pb = W.seeded(1.5, 0.4, 4095, 6, r=4.0, kappa_seed=3, f_seed=4)
    tol = 1e-16
    prob = _problem(pb, krylov_tol=tol, solver=solver, x0_mode=3)
    _, _, reps = prob.solve_all()
    say("[levels] floor relres", [f"{r.relres:.2e}" for r in reps])
    assert all(r.flags & fids.FIDS_LEVEL_ABOVE_TOL for r in reps)
    assert max(r.relres for r in reps) < 1e-10
    prob.close()
    # the allowance switched off from the host: the first level fails
    os.environ["FIDS_FLOOR_SCALE"] = "0"
    try:
        prob = _problem(pb, krylov_tol=tol, solver=solver, x0_mode=3)
    finally:
        del os.environ["FIDS_FLOOR_SCALE"]
    info = (fids.StepInfo * pb.M)()
    st = prob.solve_all_raw(None, None, info)
    assert st == fids.FIDS_ENOCONV
    assert info[0].m == 1 and info[0].relres > 4 * tol
    # the level was not accepted: the state stays at level 0 until a reset
    assert prob.solve_levels_raw(1) == fids.FIDS_ESTATE
    prob.reset()
    prob.close()


@pytest.mark.parametrize("kw", FORMS[:2])
def test_symbols_built_alongside_equal_built_before(kw, monkeypatch):
    """A solve from level 0 builds the per-level symbols (kbar, kmax and the
    preconditioner of each level) on a second stream while its levels run,
    each level waiting for its own; the solution and every level report are
    bit-identical to a solve whose symbols were all built before the launch
    (FIDS_SYM_OVERLAP=0), and to runs of levels that build their own levels'
    symbols alongside."""
    pb = W.seeded(1.4, 0.4, 4095, 64, kappa_seed=91, f_seed=92)
    prob = _problem(pb, krylov_tol=1e-10, **kw)
    try:
        monkeypatch.setenv("FIDS_SYM_OVERLAP", "0")
        u0, _, reps0 = prob.solve_all()
        u0 = u0.cpu().numpy()
        monkeypatch.setenv("FIDS_SYM_OVERLAP", "1")
        prob.reset()
        u1, _, reps1 = prob.solve_all()
        u1 = u1.cpu().numpy()
        prob.reset()
        got = []
        for c in (1, 9, 30, 24):
            u2, r2 = prob.solve_levels(c)
            got += r2
        u2 = u2.cpu().numpy()
    finally:
        prob.close()
    say(f"  overlap vs before: max diff {np.max(np.abs(u1 - u0)):.3e}, windows {np.max(np.abs(u2 - u0)):.3e}")
    assert np.array_equal(u1, u0) and np.array_equal(u2, u0)
    assert [_key(r) for r in reps1] == [_key(r) for r in reps0]
    assert [_key(r) for r in got] == [_key(r) for r in reps0]
