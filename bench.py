"""Benchmark: solved time levels per second of the fast implicit difference
scheme on one MI355X, at n = 65535 interior nodes and M = 2048 graded levels
(alpha = 1.5, gamma = 0.4, r = (2-gamma)/gamma = 4, seeded smooth kappa(x,t)
and f(x,t), phi = (1-x^2)^{alpha/2}).

A bench "step" is one time level: the SOE history update and right-hand side,
the level's Strang preconditioner symbol, and the preconditioned Krylov solve.
The timed region starts from level 0 (inputs resident in HBM, tables built)
and runs exactly --steps levels, restarting from level 0 after level M.

Prints one JSON line.  Extra fields:
  roofline      algorithmic HBM bytes of the level kernel / its measured time
  cpu_baseline  the CPU oracle (direct scheme, dense LU) on a bounded sample
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2048)
    ap.add_argument("--warmup", type=int, default=2048)
    ap.add_argument("--n", type=int, default=65535)
    ap.add_argument("--M", type=int, default=2048)
    ap.add_argument("--solver", default="bicgstab", choices=["bicgstab", "fgmres"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-levels", type=int, default=24)
    ap.add_argument("--cpu-n", type=int, default=4095)
    return ap.parse_args()


def workload(n, M):
    from paper_2002_11978_amd import workloads as W
    return W.seeded(1.5, 0.4, n, M, r=4.0, kappa_seed=3, f_seed=4, name="c2")


def algorithmic_bytes_per_level(n, nexp, matvecs):
    """Compulsory HBM bytes of one level (FP64 = 8 B; each vector read or
    written once per use in the method, symbols counted as n values):
      SOE update + rhs: read/write F (16 n nexp), read u^{m-1}, u^{m-2}, f^m,
                        kappa^m and write b (40 n)
      per BiCGSTAB iteration (two matvecs): 280 n
    """
    return 16.0 * n * nexp + 40.0 * n + 140.0 * n * matvecs


def cpu_baseline(args):
    """Oracle (direct scheme, dense LU per level, full history) on the first
    levels of the same recipe at n = cpu_n; reported in levels/s."""
    import oracle
    import torch
    t_threads = torch.get_num_threads()
    pb = workload(args.cpu_n, args.M)
    K = args.cpu_levels
    kap = pb.kappa[:K]
    f = pb.f[:K]
    t0 = time.perf_counter()
    # run the direct scheme over the first K levels of the M-level mesh
    A = oracle.ifl_matrix(pb.n, pb.alpha)
    g = 1.0 / math.gamma(1.0 - pb.gamma)
    U = np.empty((K + 1, pb.n))
    U[0] = pb.phi
    import scipy.linalg as sla
    for m in range(1, K + 1):
        a = oracle.l1_weights(1.0, pb.M, pb.r, pb.gamma, m)
        rhs = g * a[0] * U[0] + f[m - 1]
        if m > 1:
            rhs = rhs + g * (np.diff(a)[: m - 1] @ U[1:m])
        Mm = kap[m - 1][:, None] * A
        Mm[np.diag_indices(pb.n)] += g * a[m - 1]
        U[m] = sla.solve(Mm, rhs)
    dt = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"value": K / dt, "unit": "levels/s", "cores": cores, "kind": "oracle",
            "sample": f"direct scheme + LAPACK dense LU, first {K} of M={pb.M} levels of the same recipe "
                      f"at n={pb.n} (n=65535 does not fit a dense LU in a bounded time); "
                      f"{dt:.1f} s; torch threads {t_threads}"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "independent problems shard across GPUs without communication, see DESIGN.md", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2002_11978_amd import fids

    dev = torch.device("cuda:0")
    pb = workload(args.n, args.M)
    solver = fids.FIDS_FGMRES if args.solver == "fgmres" else fids.FIDS_BICGSTAB
    prec = fids.FIDS_MIXED if args.precision == "mixed" else fids.FIDS_FP64
    params = fids.default_params(alpha=pb.alpha, gamma=pb.gamma, n=pb.n, M=pb.M, r=pb.r,
                                 soe_tol=1e-10, krylov_tol=1e-12, krylov_maxit=500,
                                 solver=solver, precision=prec, kappa_time_dependent=1)
    kappa = torch.from_numpy(pb.kappa).to(dev)
    f = torch.from_numpy(pb.f).to(dev)
    phi = torch.from_numpy(pb.phi).to(dev)
    prob = fids.Problem(params, kappa, f, phi)
    stream = prob.stream
    M = pb.M
    infos = (fids.StepInfo * M)()

    def run_levels(K):
        """Exactly K levels from level 0, wrapping at M."""
        done = 0
        while done < K:
            prob.reset()
            if K - done >= M:
                st = prob.solve_all_raw(None, None, infos)
                if st != 0:
                    raise fids.FidsError(st, "fids_solve_all")
                done += M
            else:
                for _ in range(K - done):
                    prob.step()
                done = K

    print(f"[bench] n={pb.n} M={M} ws={prob.ws_bytes / 2**20:.1f} MiB warmup={args.warmup} steps={args.steps}",
          file=sys.stderr, flush=True)
    if args.warmup > 0:
        run_levels(args.warmup)
    torch.cuda.synchronize()
    # ---- timed region: exactly K levels
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    run_levels(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    value = args.steps / wall
    print(f"[bench] {args.steps} levels in {wall:.3f} s wall ({ms_total:.1f} ms events)", file=sys.stderr, flush=True)

    # ---- level kernel alone: symbols prepared first, one launch for all M levels
    prob.reset()
    prob.prepare()
    torch.cuda.synchronize()
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    k0.record(stream)
    st = prob.solve_all_raw(None, None, infos)
    k1.record(stream)
    torch.cuda.synchronize()
    if st != 0:
        raise fids.FidsError(st, "fids_solve_all")
    kern_ms = k0.elapsed_time(k1)
    mv = [infos[i].matvecs for i in range(M)]
    nexp = int(fids.soe_nodes(pb.gamma, (1.0 / M) ** pb.r, 1.0, params.soe_tol)[0].size)
    bytes_launch = sum(algorithmic_bytes_per_level(pb.n, nexp, v) for v in mv)
    achieved = bytes_launch / (kern_ms * 1e-3) / 1e9
    print(f"[bench] level kernel {kern_ms:.1f} ms for {M} levels; nexp={nexp}; "
          f"avg its {np.mean(mv) / 2:.2f}; {bytes_launch / 1e9:.2f} GB algorithmic", file=sys.stderr, flush=True)

    out = {
        "metric": "solved time steps/s at N=65535,M=2048",
        "value": value,
        "unit": "time steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == fids.FIDS_FP64 else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"fractional diffusion, n={pb.n} interior nodes, M={M} graded levels, "
                               f"alpha=1.5, gamma=0.4, r=4, seeded kappa(x,t) and f(x,t)",
                   "n": pb.n, "M": M, "solver": args.solver, "precision": args.precision,
                   "krylov_tol": params.krylov_tol, "soe_tol": params.soe_tol, "nexp": nexp,
                   "avg_iterations": float(np.mean(mv) / 2), "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_levels", "kernel_ms_per_launch": kern_ms,
                     "bytes_per_launch": bytes_launch},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args)
    prob.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
