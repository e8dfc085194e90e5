"""GPU parity of the discrete adjoint (dJ/dkappa, dJ/df, dJ/dphi of J(u^M)).

Reference values come from the oracle's exact adjoint of the direct scheme
(dense transposed LU per level, full L1 history).  The fast scheme's adjoint
differs from it by the SOE and Krylov tolerances only, so the gates are those
of the forward parity: relative max-norm <= 1e-8 (FP64), <= 1e-7 (FP32
preconditioner).  Checkpointed runs (segments recomputed from snapshots)
must reproduce the stored-states run bit for bit, and central finite
differences of the GPU forward check the gradients independently of the
oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2002_11978_amd import fids
from paper_2002_11978_amd import workloads as W

from gpu_util import rel_maxnorm, say, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-8
TOL_MIXED = 1e-7

VARIANTS = [
    pytest.param(dict(solver=0, precision=0, x0_mode=0), id="bicgstab-fp64-x0zero"),
    pytest.param(dict(solver=0, precision=0, x0_mode=1), id="bicgstab-fp64-x0extrap"),
    pytest.param(dict(solver=1, precision=0, x0_mode=0), id="fgmres-fp64-x0zero"),
    pytest.param(dict(solver=1, precision=0, x0_mode=1), id="fgmres-fp64-x0extrap"),
    pytest.param(dict(solver=1, precision=1, x0_mode=1), id="fgmres-mixed-x0extrap"),
    pytest.param(dict(solver=2, precision=0, x0_mode=3), id="pcg-fp64-x0cubic"),
]


def _gate(kw):
    return TOL_MIXED if kw.get("precision", 0) == 1 else TOL


def _params(pb, **kw):
    td = int(pb.kappa.ndim == 2)
    p = fids.default_params(alpha=pb.alpha, gamma=pb.gamma, n=pb.n, M=pb.M, r=pb.r, mu=pb.mu,
                            l=pb.l, T=pb.T, kappa_time_dependent=td)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _target(pb, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    return g.normal(0.0, 1.0, pb.n)


def _gpu_grads(pb, ustar, **kw):
    """Forward to u^M, then the adjoint of J = ||u^M - u*||^2; numpy outputs."""
    import torch
    p = _params(pb, **kw)
    say(f"[gpu adjoint] n={pb.n} M={pb.M} td={p.kappa_time_dependent} solver={p.solver} "
        f"prec={p.precision} x0={p.x0_mode} store={p.store_states} ckpt={p.checkpoint_every}")
    prob = fids.Problem(p, to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi))
    uT, _, _ = prob.solve_all()
    dJ = 2.0 * (uT - to_dev(ustar))
    gk, gf, gphi = prob.adjoint(dJ.contiguous())
    reps = prob.adjoint_reports()
    torch.cuda.synchronize()
    out = (gk.cpu().numpy(), gf.cpu().numpy(), gphi.cpu().numpy(), uT.cpu().numpy())
    prob.close()
    return out, reps


def _oracle_grads(pb, ustar):
    U = oracle.dids_solve(pb.alpha, pb.gamma, pb.n, pb.M, pb.r, pb.kappa, pb.f, pb.phi,
                          l=pb.l, T=pb.T, mu=pb.mu or None)
    dJ = 2.0 * (U[-1] - ustar)
    return oracle.dids_adjoint(pb.alpha, pb.gamma, pb.n, pb.M, pb.r, pb.kappa, pb.f, pb.phi, dJ, U=U,
                               l=pb.l, T=pb.T, mu=pb.mu or None)


SIZES = [(1, 3), (4, 2), (5, 1), (100, 12), (257, 9), (1000, 16)]


@pytest.mark.parametrize("kw", VARIANTS)
@pytest.mark.parametrize("td", [True, False], ids=["kappa_xt", "kappa_x"])
@pytest.mark.parametrize("n,M", SIZES)
def test_adjoint_matches_oracle(n, M, td, kw):
    pb = W.seeded(1.5, 0.4, n, M, kappa_seed=11, f_seed=12, time_dependent=td)
    ustar = _target(pb, 13)
    (gk, gf, gphi, _), reps = _gpu_grads(pb, ustar, store_states=1, **kw)
    rk, rf, rphi = _oracle_grads(pb, ustar)
    errs = (rel_maxnorm(gk, rk), rel_maxnorm(gf, rf), rel_maxnorm(gphi, rphi))
    say(f"  rel err kappa {errs[0]:.3e} f {errs[1]:.3e} phi {errs[2]:.3e} "
        f"adj its {np.mean([r.iters for r in reps]):.2f}")
    assert gk.shape == rk.shape and gf.shape == rf.shape
    assert max(errs) <= _gate(kw)
    assert [r.m for r in reps] == list(range(1, M + 1))


@pytest.mark.parametrize("kw", [VARIANTS[0], VARIANTS[3], VARIANTS[4],
                                pytest.param(dict(solver=1, precision=0, x0_mode=2), id="fgmres-fp64-x0quad"),
                                pytest.param(dict(solver=1, precision=0, x0_mode=3), id="fgmres-fp64-x0cubic"),
                                pytest.param(dict(solver=2, precision=0, x0_mode=3), id="pcg-fp64-x0cubic")])
@pytest.mark.parametrize("C", [1, 3, 5, 16, 40])
def test_checkpointed_equals_stored_states(C, kw):
    """Segments recomputed from snapshots give the stored-states gradients
    exactly (the recomputation is the same deterministic computation; both
    forward runs stream the history in the solver group, as snapshots
    require, so that the history sums share their rounding order)."""
    pb = W.seeded(1.3, 0.6, 2047, 33, kappa_seed=21, f_seed=22, time_dependent=True)
    ustar = _target(pb, 23)
    full, _ = _gpu_grads(pb, ustar, store_states=1, wg_count=4, soe_helpers=0, **kw)
    ck, _ = _gpu_grads(pb, ustar, store_states=0, checkpoint_every=C, wg_count=4, soe_helpers=0, **kw)
    for a, b in zip(full, ck):
        assert np.array_equal(a, b)


def test_checkpoint_snapshots_do_not_change_the_forward():
    pb = W.seeded(1.5, 0.4, 1023, 20, kappa_seed=31, f_seed=32)
    outs = []
    # without helper workgroups in all three (snapshots turn them off; they
    # change the history sums' rounding order)
    for kw in (dict(), dict(checkpoint_every=3), dict(store_states=1)):
        p = _params(pb, solver=1, x0_mode=3, soe_helpers=0, **kw)
        prob = fids.Problem(p, to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi))
        uT, _, _ = prob.solve_all()
        outs.append(uT.cpu().numpy())
        prob.close()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_adjoint_state_errors():
    import torch
    pb = W.seeded(1.5, 0.4, 63, 6)
    dJ = torch.ones(pb.n, dtype=torch.float64, device="cuda")
    # no stored states and no snapshots
    prob = fids.Problem(_params(pb), to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi))
    prob.solve_all()
    with pytest.raises(fids.FidsError) as e:
        prob.adjoint(dJ)
    assert e.value.status == fids.FIDS_ESTATE
    prob.close()
    # forward not complete
    prob = fids.Problem(_params(pb, checkpoint_every=2), to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi))
    prob.step()
    with pytest.raises(fids.FidsError) as e:
        prob.adjoint(dJ)
    assert e.value.status == fids.FIDS_ESTATE
    # stepping level by level then the adjoint works; afterwards the forward
    # state is at level min(C, M) and solve_all returns it to M
    for _ in range(pb.M - 1):
        prob.step()
    gk, gf, gphi = prob.adjoint(dJ)
    assert torch.isfinite(gk).all() and torch.isfinite(gf).all() and torch.isfinite(gphi).all()
    uT, _, _ = prob.solve_all()
    gk2, gf2, gphi2 = prob.adjoint(dJ)
    assert torch.equal(gk, gk2) and torch.equal(gf, gf2) and torch.equal(gphi, gphi2)
    prob.close()


def test_outputs_may_be_null():
    import torch
    pb = W.seeded(1.2, 0.3, 300, 7)
    ustar = _target(pb, 41)
    (gk, gf, gphi, uT), _ = _gpu_grads(pb, ustar, store_states=1)
    p = _params(pb, store_states=1)
    prob = fids.Problem(p, to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi))
    prob.solve_all()
    dJ = 2.0 * (to_dev(uT) - to_dev(ustar))
    only_phi = torch.empty(pb.n, dtype=torch.float64, device="cuda")
    prob.adjoint(dJ, g_phi=only_phi, allocate=False)
    assert np.array_equal(only_phi.cpu().numpy(), gphi)
    prob.close()


def _fd_check(pb, ustar, ndir, seed, rel_gate, tol=1e-13, **kw):
    """Central differences of J along unit directions d over (kappa, f, phi).

    Step: the kappa part of the perturbation has norm 1e-4 ||kappa||, so the
    O(step^2) truncation error along kappa is about 1e-8 relative; J is
    quadratic in (f, phi), where central differences are exact for any step.
    What remains is the noise of J from the Krylov tolerance divided by the
    step.  The error of each direction is measured relative to
    max(|<g, d>|, ||g|| / sqrt(dim)): the second term is the typical size of a
    random unit direction's derivative, so that a direction nearly orthogonal
    to g (where that noise is the whole of both numbers) does not read as a
    relative error of order one.
    """
    import torch
    p = _params(pb, krylov_tol=tol, **kw)
    kap, f, phi = to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi)
    k0, f0, p0 = kap.clone(), f.clone(), phi.clone()
    us = to_dev(ustar)
    prob = fids.Problem(p, kap, f, phi)

    def J():
        prob.reset()
        uT, _, _ = prob.solve_all()
        return float(((uT - us) ** 2).sum())

    prob.reset()
    uT, _, _ = prob.solve_all()
    gk, gf, gphi = prob.adjoint((2.0 * (uT - us)).contiguous())
    g = torch.cat([gk.flatten(), gf.flatten(), gphi.flatten()])
    scale = float(torch.linalg.norm(g)) / g.numel() ** 0.5
    gen = np.random.Generator(np.random.PCG64(seed))
    nk, nf = k0.numel(), f0.numel()
    worst = 0.0
    for d_i in range(ndir):
        d = to_dev(gen.normal(0.0, 1.0, g.numel()))
        d /= torch.linalg.norm(d)
        dk, df, dp = d[:nk].view_as(k0), d[nk:nk + nf].view_as(f0), d[nk + nf:]
        eps = 1e-4 * float(torch.linalg.norm(k0)) / float(torch.linalg.norm(dk))
        jp = []
        for sgn in (1.0, -1.0):
            kap.copy_(k0 + sgn * eps * dk)
            f.copy_(f0 + sgn * eps * df)
            phi.copy_(p0 + sgn * eps * dp)
            jp.append(J())
        fd = (jp[0] - jp[1]) / (2 * eps)
        ad = float((g * d).sum())
        rel = abs(fd - ad) / max(abs(ad), scale)
        worst = max(worst, rel)
        say(f"  dir {d_i}: adjoint {ad:.10e} fd {fd:.10e} rel {rel:.2e} (|g|/sqrt(dim) {scale:.3e})")
    prob.close()
    assert worst <= rel_gate


@pytest.mark.parametrize("kw", [VARIANTS[0], VARIANTS[3], VARIANTS[4]])
def test_finite_differences_reduced(kw):
    pb = W.seeded(1.6, 0.5, 1023, 48, r=3.0, kappa_seed=5, f_seed=7, time_dependent=False)
    ustar = _target(pb, 6)
    _fd_check(pb, ustar, 16, 8, 1e-6, checkpoint_every=8, **kw)


@pytest.mark.parametrize("kw", [pytest.param(dict(solver=1, x0_mode=1), id="fgmres-x0linear"),
                                pytest.param(dict(solver=2, x0_mode=3), id="pcg-x0cubic")])
def test_finite_differences_adjoint_workload(kw):
    """n = 16383, M = 1024, alpha 1.6, gamma 0.5, r 3, time-independent kappa
    (seed 5); target u* = u^M of a second kappa (seed 6); f seed 7; snapshots
    every 32 levels; 16 unit directions (seed 8) over (kappa, f, phi); the
    FGMRES form and the benchmark's conjugate-gradient form."""
    import torch
    pb = W.seeded(1.6, 0.5, 16383, 1024, r=3.0, kappa_seed=5, f_seed=7, time_dependent=False)
    tgt = W.seeded(1.6, 0.5, 16383, 1024, r=3.0, kappa_seed=6, f_seed=7, time_dependent=False)
    p = _params(tgt, solver=1, x0_mode=1)
    prob = fids.Problem(p, to_dev(tgt.kappa), to_dev(tgt.f), to_dev(tgt.phi))
    ustar, _, _ = prob.solve_all()
    ustar = ustar.cpu().numpy()
    prob.close()
    torch.cuda.synchronize()
    _fd_check(pb, ustar, 16, 8, 1e-6, checkpoint_every=32, **kw)


def test_autograd_function_matches_adjoint():
    import torch
    from paper_2002_11978_amd import autograd as AG
    pb = W.seeded(1.5, 0.4, 511, 24, kappa_seed=51, f_seed=52, time_dependent=True)
    ustar = _target(pb, 53)
    # the wrapper checkpoints (no helper workgroups): so does the reference
    (gk, gf, gphi, uT), _ = _gpu_grads(pb, ustar, store_states=1, solver=1, x0_mode=1, soe_helpers=0)
    p = _params(pb, solver=1, x0_mode=1, soe_helpers=0)
    kap = to_dev(pb.kappa).requires_grad_(True)
    f = to_dev(pb.f).requires_grad_(True)
    phi = to_dev(pb.phi).requires_grad_(True)
    u = AG.solve(p, kap, f, phi, checkpoint_every=5)
    J = ((u - to_dev(ustar)) ** 2).sum()
    J.backward()
    assert np.array_equal(u.detach().cpu().numpy(), uT)
    assert np.array_equal(kap.grad.cpu().numpy(), gk)
    assert np.array_equal(f.grad.cpu().numpy(), gf)
    assert np.array_equal(phi.grad.cpu().numpy(), gphi)
