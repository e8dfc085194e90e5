"""GPU test of the allocation-free entry point fids_solve_static.

It must give the same u^M and level reports as fids_init_problem +
fids_solve_all on a caller's workspace (the same kernels run on the same
plan; only the workspace's address and the symbol batch size differ), on two
calls in a row with the second on a smaller problem (the fixed array keeps
the first call's contents), and it must reject a problem that does not fit.
"""
import ctypes

import numpy as np
import pytest
import torch

from paper_2002_11978_amd import fids
from paper_2002_11978_amd import workloads as W

from gpu_util import rel_maxnorm, say, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-8


def _params(pb, **kw):
    p = fids.default_params(alpha=pb.alpha, gamma=pb.gamma, n=pb.n, M=pb.M, r=pb.r, kappa_time_dependent=1,
                            krylov_tol=1e-10, krylov_maxit=500)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _static(params, k, f, phi):
    """fids_solve_static through the C ABI (ctypes), on the current stream."""
    uT = torch.empty(int(params.n), dtype=torch.float64, device=k.device)
    infos = (fids.StepInfo * int(params.M))()
    stream = torch.cuda.current_stream(k.device).cuda_stream
    st = fids.lib().fids_solve_static(ctypes.byref(params), ctypes.c_void_p(k.data_ptr()),
                                      ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(phi.data_ptr()),
                                      ctypes.c_void_p(uT.data_ptr()), infos, ctypes.c_void_p(stream))
    return st, uT.cpu().numpy(), [fids.LevelReport.of(i) for i in infos]


CASES = [
    (W.seeded(1.5, 0.4, 4095, 96, r=4.0, kappa_seed=3, f_seed=4), dict(solver=2, x0_mode=3)),
    (W.seeded(1.2, 0.3, 1000, 40, kappa_seed=1, f_seed=2), dict(solver=1, x0_mode=3)),
    (W.seeded(1.8, 0.7, 257, 24, kappa_seed=5, f_seed=6), dict(solver=0, x0_mode=0)),
]


@pytest.mark.parametrize("forms", [[0, 1], [1, 2], [0, 2]], ids=["large-then-mid", "mid-then-small", "large-then-small"])
def test_static_solve_matches_workspace_solve(forms):
    for i in forms:
        pb, kw = CASES[i]
        params = _params(pb, **kw)
        k, f, phi = to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi)
        say(f"[no-alloc] n={pb.n} M={pb.M} {kw}")
        st, u_s, reps_s = _static(params, k, f, phi)
        assert st == fids.FIDS_OK, fids.strerror(st)
        prob = fids.Problem(params, k, f, phi)
        uT, _, reps = prob.solve_all()
        prob.close()
        u_w = uT.cpu().numpy()
        err = rel_maxnorm(u_s, u_w)
        say(f"[no-alloc] rel diff {err:.3e}")
        assert err <= TOL
        assert np.array_equal(u_s, u_w)
        assert [(r.m, r.iters, r.matvecs, r.relres, r.flags) for r in reps_s] == \
               [(r.m, r.iters, r.matvecs, r.relres, r.flags) for r in reps]


def test_static_solve_rejects_problems_beyond_the_array():
    pb = W.seeded(1.5, 0.4, 16383, 1024, r=4.0, kappa_seed=3, f_seed=4)
    params = _params(pb, solver=2, x0_mode=3)
    k, f, phi = to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi)
    st, _, _ = _static(params, k, f, phi)
    assert st == fids.FIDS_EINVAL
    assert "static array" in fids.lib().fids_last_error().decode()
    # the array is still usable afterwards
    pb, kw = CASES[2]
    st, u_s, _ = _static(_params(pb, **kw), to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi))
    assert st == fids.FIDS_OK and np.all(np.isfinite(u_s))
