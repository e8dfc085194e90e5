"""GPU tests of the batched form: independent problems of (1.1) with uneven n,
(alpha, gamma), kappa and f advanced together, one workgroup per problem.

The batch gives large members a group of several workgroups and packs small
ones into shared one-workgroup slots.  A member runs the same arithmetic as a
single problem whose plan targets the member's group size (wg_count =
fids_batch_groups), so the two agree bit for bit; members small enough for
the oracle are also checked against it.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2002_11978_amd import fids
from paper_2002_11978_amd import workloads as W

from gpu_util import rel_maxnorm, say, to_dev

pytestmark = pytest.mark.gpu

MIXED = dict(solver=1, precision=1, x0_mode=1)


def _params(pb, **kw):
    p = fids.default_params(alpha=pb.alpha, gamma=pb.gamma, n=pb.n, M=pb.M, r=pb.r, mu=pb.mu,
                            kappa_time_dependent=int(pb.kappa.ndim == 2), dims=getattr(pb, "dims", 1))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _batch(pbs, **kw):
    say(f"[gpu batch] count={len(pbs)} M={pbs[0].M} n={[pb.n for pb in pbs][:8]}... kw={kw}")
    params = [_params(pb, **kw) for pb in pbs]
    return fids.Batch(params, [to_dev(pb.kappa) for pb in pbs], [to_dev(pb.f) for pb in pbs],
                      [to_dev(pb.phi) for pb in pbs])


def _solo(pb, wg=1, **kw):
    # batch members stream their history themselves (no helper workgroups):
    # so does the solo run it is compared with bit for bit
    kw.setdefault("soe_helpers", 0)
    prob = fids.Problem(_params(pb, wg_count=wg, **kw), to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi))
    uT, _, reps = prob.solve_all()
    out = uT.cpu().numpy()
    prob.close()
    return out, reps


def _mixed_members(M):
    shapes = [(1, 1.5, 0.5), (4, 1.2, 0.3), (100, 1.8, 0.7), (257, 1.5, 0.4), (511, 1.3, 0.6),
              (1000, 1.7, 0.25), (2047, 1.1, 0.8), (3000, 1.5, 0.5)]
    return [W.seeded(a, g, n, M, kappa_seed=100 + i, f_seed=200 + i, time_dependent=(i % 2 == 0))
            for i, (n, a, g) in enumerate(shapes)]


@pytest.mark.parametrize("kw", [dict(solver=0, precision=0, x0_mode=0), dict(solver=1, precision=0, x0_mode=1),
                                MIXED, dict(solver=2, precision=0, x0_mode=3)],
                         ids=["bicgstab-fp64", "fgmres-fp64", "fgmres-mixed", "pcg-fp64"])
def test_batch_members_equal_solo_and_oracle(kw):
    pbs = _mixed_members(12)
    b = _batch(pbs, **kw)
    groups = b.groups()
    say(f"  groups {groups}")
    assert max(groups) > 1          # the largest members run on several workgroups
    outs, reps = b.solve_all()
    gate = 1e-7 if kw.get("precision") == 1 else 1e-8
    for i, pb in enumerate(pbs):
        u = outs[i].cpu().numpy()
        solo, solo_reps = _solo(pb, wg=groups[i], **kw)
        assert np.array_equal(u, solo), f"member {i} differs from its solo run"
        assert [r.iters for r in reps[i]] == [r.iters for r in solo_reps]
        if pb.n <= 1000:
            R = oracle.dids_solve(pb.alpha, pb.gamma, pb.n, pb.M, pb.r, pb.kappa, pb.f, pb.phi)
            err = rel_maxnorm(u, R[-1])
            say(f"  member {i} n={pb.n}: rel err vs oracle {err:.3e}")
            assert err <= gate
    st, last = b.status()
    assert st == [0] * len(pbs) and last == [12] * len(pbs)
    b.close()


def test_batch_step_equals_solve_all_and_reset():
    pbs = _mixed_members(9)
    b = _batch(pbs, **MIXED)
    outs, _ = b.solve_all()
    ref = [o.cpu().numpy() for o in outs]
    b.reset()
    for m in range(1, 10):
        reps = b.step()
        assert all(r.m == m for r in reps)
    st, last = b.status()
    assert last == [9] * len(pbs)
    with pytest.raises(fids.FidsError) as e:
        b.step()
    assert e.value.status == fids.FIDS_ESTATE
    b.reset()
    outs2, _ = b.solve_all()
    for a, o in zip(ref, outs2):
        assert np.array_equal(a, o.cpu().numpy())
    b.close()


def test_batch_graph_mode_equals_persistent():
    # equal members: every one fits a one-workgroup slot, the launch is an
    # ordinary one and may be captured
    pbs = [W.seeded(1.5, 0.4, 100, 10, kappa_seed=300 + i, f_seed=400 + i) for i in range(6)]
    b = _batch(pbs, **MIXED)
    ref = [o.cpu().numpy() for o in b.solve_all()[0]]
    b.close()
    os.environ["FIDS_BATCH_MODE"] = "graph"
    try:
        g = _batch(pbs, **MIXED)
    finally:
        del os.environ["FIDS_BATCH_MODE"]
    assert g.groups() == [1] * len(pbs)
    for rep in range(3):           # the captured graph is replayed after each reset
        outs, _ = g.solve_all()
        for a, o in zip(ref, outs):
            assert np.array_equal(a, o.cpu().numpy())
        g.reset()
    g.close()


def test_batch_graph_mode_tuned_after_capture():
    """A solve in graph mode captures the level launches with the plan's tile
    shape and LDS size; tuning afterwards changes both, so the next solve
    must capture again rather than replay the old graph.  Its answer is
    compared with a persistent-mode batch tuned the same way (the tuner may
    pick another tiling there, so the comparison allows summation-order
    differences), and with the untuned graph-mode answer."""
    pbs = [W.seeded(1.5, 0.4, 1000, 10, kappa_seed=320 + i, f_seed=420 + i) for i in range(4)]
    p = _batch(pbs, **MIXED)
    p.tune()
    ref = [o.cpu().numpy() for o in p.solve_all()[0]]
    p.close()
    # the graph-mode batch starts from 4 column tiles of 8 columns (N_c = 1024
    # = 32 x 32), which the tuner is expected to replace
    os.environ["FIDS_BATCH_MODE"] = "graph"
    os.environ["FIDS_TILES"] = "4"
    try:
        g = _batch(pbs, **MIXED)
    finally:
        del os.environ["FIDS_BATCH_MODE"]
        del os.environ["FIDS_TILES"]
    first = [o.cpu().numpy() for o in g.solve_all()[0]]   # captured with the untuned plan
    g.reset()
    ct = g.tune()
    say(f"graph-mode batch tuned after capture: columns per tile 8 -> {list(ct)}")
    for rep in range(2):
        outs = [o.cpu().numpy() for o in g.solve_all()[0]]
        for a, b0, o in zip(ref, first, outs):
            assert np.isfinite(o).all()
            assert rel_maxnorm(o, a) <= 1e-10
            assert rel_maxnorm(o, b0) <= 1e-10
        g.reset()
    g.close()


def test_failing_member_does_not_stop_the_others():
    pbs = _mixed_members(6)
    params = [_params(pb, **MIXED) for pb in pbs]
    params[3].krylov_maxit = 1
    params[3].krylov_tol = 1e-15
    b = fids.Batch(params, [to_dev(pb.kappa) for pb in pbs], [to_dev(pb.f) for pb in pbs],
                   [to_dev(pb.phi) for pb in pbs])
    with pytest.raises(fids.FidsError) as e:
        b.solve_all()
    assert e.value.status == fids.FIDS_ENOCONV
    st, last = b.status()
    assert st[3] == fids.FIDS_ENOCONV and last[3] == 0
    assert all(st[i] == 0 and last[i] == 6 for i in range(len(pbs)) if i != 3)
    b.close()


def test_batch_rejects_bad_input():
    pbs = _mixed_members(5)
    params = [_params(pb) for pb in pbs]
    params[2].M = 6
    with pytest.raises(fids.FidsError):
        fids.Batch(params, [to_dev(pb.kappa) for pb in pbs], [to_dev(pb.f) for pb in pbs],
                   [to_dev(pb.phi) for pb in pbs])


def test_heterogeneous_batch_full_size_sampled():
    """256 members, n log-uniform in [511, 16383], M = 256, FP32-preconditioned
    FGMRES: every member finishes with a finite state; sampled members (the
    smallest, the largest and a few between) equal their solo one-workgroup
    runs bit for bit."""
    import torch
    M = 256
    pbs = [W.batch_member(p, M=M) for p in range(256)]
    b = _batch(pbs, krylov_tol=1e-10, **MIXED)
    groups = b.groups()
    say(f"  group sizes used: {sorted(set(groups))}, workgroups {sum(g for g in groups if g > 1)} in groups")
    try:
        outs, reps = b.solve_all()
    finally:
        st, last = b.status()
        bad = [(i, pbs[i].n, round(pbs[i].alpha, 3), round(pbs[i].gamma, 3), st[i], last[i])
               for i in range(256) if st[i] != 0]
        say(f"  failing members (i, n, alpha, gamma, status, last level): {bad}")
    assert st == [0] * 256 and last == [M] * 256
    assert all(bool(torch.isfinite(o).all()) for o in outs)
    ns = [pb.n for pb in pbs]
    sample = sorted({int(np.argmin(ns)), int(np.argmax(ns)), 17, 101, 200})
    for i in sample:
        solo, _ = _solo(pbs[i], wg=groups[i], krylov_tol=1e-10, **MIXED)
        assert np.array_equal(outs[i].cpu().numpy(), solo), f"member {i} (n={ns[i]})"
    its = np.mean([[r.iters for r in rr] for rr in reps])
    say(f"  mean FGMRES iterations {its:.2f}")
    b.close()


def test_batch_tune_keeps_results():
    """The autotuner may change every class's tiling; results stay within
    rounding of the untuned batch and match the oracle; a tuned batch is
    deterministic."""
    pbs = _mixed_members(10)
    b = _batch(pbs, solver=1, precision=0, x0_mode=3)
    ref = [o.cpu().numpy() for o in b.solve_all()[0]]
    b.reset()
    ct = b.tune(levels=3)
    say(f"  tuned columns per tile {ct}")
    assert all(c >= 1 for c in ct)
    outs1 = [o.cpu().numpy() for o in b.solve_all()[0]]
    b.reset()
    outs2 = [o.cpu().numpy() for o in b.solve_all()[0]]
    for a, c, d in zip(ref, outs1, outs2):
        assert np.array_equal(c, d)
        assert rel_maxnorm(c, a) <= 1e-10
    for i, pb in enumerate(pbs):
        if pb.n <= 1000:
            R = oracle.dids_solve(pb.alpha, pb.gamma, pb.n, pb.M, pb.r, pb.kappa, pb.f, pb.phi)
            assert rel_maxnorm(outs1[i], R[-1]) <= 1e-8
    b.close()


def test_batch_tune_class_with_uneven_soe_sizes():
    """Members of one class (equal embedding length and group) have different
    SOE node counts, so different LDS needs; the tuned tiling must fit the
    largest of them (a too-small LDS allocation corrupts results silently).
    Tuned results stay within rounding of the untuned batch."""
    M = 24
    pbs = [pb for pb in (W.batch_member(p, M=M) for p in range(256)) if 4096 < pb.n <= 8192][:24]
    assert len(pbs) >= 8
    b = _batch(pbs, solver=1, precision=0, x0_mode=3, precond=2, krylov_tol=1e-10)
    ref = [o.cpu().numpy() for o in b.solve_all()[0]]
    b.reset()
    ct = b.tune(levels=2)
    say(f"  tuned columns per tile {sorted(set(ct))}")
    outs, reps = b.solve_all()
    st, last = b.status()
    assert st == [0] * len(pbs)
    for a, o in zip(ref, outs):
        assert rel_maxnorm(o.cpu().numpy(), a) <= 1e-9
    b.close()


@pytest.mark.parametrize("kw", [dict(solver=2, precision=0, x0_mode=3), MIXED], ids=["pcg-fp64", "fgmres-mixed"])
def test_batch_with_2d_members(kw):
    """1-D and 2-D members (dims = 2, the padded-row layout) in one persistent
    launch: each equals its solo run bit for bit, and the 2-D members match
    the oracle's 2-D direct scheme."""
    M = 8
    pbs = [W.seeded2d(1.5, 0.5, 15, M, kappa_seed=400, f_seed=401),
           W.seeded(1.3, 0.6, 300, M, kappa_seed=402, f_seed=403),
           W.seeded2d(1.1, 0.3, 31, M, kappa_seed=404, f_seed=405),
           W.seeded2d(1.8, 0.7, 63, M, kappa_seed=406, f_seed=407)]
    for pb in pbs:
        if pb.dims == 2:
            pb.mu = oracle.mu_star(pb.alpha)
    b = _batch(pbs, **kw)
    groups = b.groups()
    outs, reps = b.solve_all()
    gate = 1e-7 if kw.get("precision") == 1 else 1e-8
    for i, pb in enumerate(pbs):
        u = outs[i].cpu().numpy()
        solo, solo_reps = _solo(pb, wg=groups[i], **kw)
        assert np.array_equal(u, solo), f"member {i} differs from its solo run"
        if pb.dims == 2:
            R = oracle.dids2d_solve(pb.alpha, pb.gamma, pb.n, M, pb.r, pb.kappa, pb.f, pb.phi, mu=pb.mu)
        else:
            R = oracle.dids_solve(pb.alpha, pb.gamma, pb.n, M, pb.r, pb.kappa, pb.f, pb.phi)
        err = rel_maxnorm(u, R[-1])
        say(f"  member {i} dims={pb.dims} n={pb.n} group {groups[i]}: rel err vs oracle {err:.3e}")
        assert err <= gate
    b.close()
