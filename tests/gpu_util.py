"""Helpers shared by the GPU tests: run a workload through the HIP library."""
import sys

import numpy as np

from paper_2002_11978_amd import fids


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def gpu_solve(pb, return_all=True, **kw):
    """Solve workload `pb` (workloads.Problem) on the GPU; returns (U or uT, reports)."""
    import torch
    td = int(pb.kappa.ndim == 2)
    params = fids.default_params(alpha=pb.alpha, gamma=pb.gamma, n=pb.n, M=pb.M, r=pb.r, mu=pb.mu,
                                 l=pb.l, T=pb.T, kappa_time_dependent=td,
                                 store_states=int(return_all), dims=getattr(pb, "dims", 1))
    for k, v in kw.items():
        setattr(params, k, v)
    say(f"[gpu] n={pb.n} M={pb.M} alpha={pb.alpha} gamma={pb.gamma} r={pb.r:.4g} "
        f"solver={params.solver} prec={params.precision} pc={params.precond} tol={params.krylov_tol}")
    prob = fids.Problem(params, to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi))
    uT, U, reps = prob.solve_all(return_all=return_all)
    torch.cuda.synchronize()
    out = U.cpu().numpy() if return_all else uT.cpu().numpy()
    prob.close()
    return out, reps


def rel_maxnorm(U, R):
    return float(np.max(np.abs(U - R)) / np.max(np.abs(R)))
