"""Benchmark: solved time levels per second of the fast implicit difference
scheme on one MI355X, at n = 65535 interior nodes and M = 2048 graded levels
(alpha = 1.5, gamma = 0.4, r = (2-gamma)/gamma = 4, seeded smooth kappa(x,t)
and f(x,t), phi = (1-x^2)^{alpha/2}; SOE tolerance 1e-10, Krylov tolerance
1e-10 relative to ||b||, the tolerance of the paper's Table 11).

A bench "step" is one full solve of the problem: all M = 2048 graded time
levels from level 0, each level being the SOE history update and right-hand
side, the level's Strang preconditioner symbol and the preconditioned Krylov
solve (inputs resident in HBM, set-up tables built before timing; the
per-level symbols are built inside the timed region).  `value` is time
levels solved per second over --steps such solves after --warmup untimed
ones (headline form; the other forms are timed over min(steps, 2) solves
after one untimed solve).  A level's cost varies about 3x over the graded
mesh (Krylov iterations per level go from 4 to 11), so a window of a few
levels would measure a position in the solve rather than the method; the
paper's Table 11 also times whole solves.  Every form covers the same levels
1..M, so `speedup_vs_plain_fp64` compares identical work.  Each form also
reports the level kernel's time for one launch over all M levels with the
symbols prepared (`kernel_ms`), and `window_levels_per_s` gives the rate of
the first --window levels after the first 5 (fids_solve_levels, one launch)
for comparison.

Four forms of the same scheme are measured (more with --forms):
  headline  preconditioned conjugate gradients on the symmetrised system
            K^{-1} M (Sec. 4.2), FP64, initial guess by cubic extrapolation
  fgmres    flexible GMRES(20), FP64, the same initial guess
  plain     BiCGSTAB, FP64, zero initial guess (the paper's solver settings)
  mixed     flexible GMRES(20) with the preconditioner FFTs in FP32
  linear_x0, quad_x0  the fgmres form with linear / quadratic extrapolation
`value` is the headline form; the others are reported beside it together with
the relative difference of their u(T) from the headline's.

Extra JSON fields:
  roofline      algorithmic HBM bytes of the level kernel / its measured time
  cpu_baseline  the CPU oracle (direct scheme, dense LU) on a bounded sample
  adjoint       adj/fwd wall-time ratio of the discrete adjoint at n = 16383,
                M = 1024 (alpha 1.6, gamma 0.5, r 3, time-independent kappa),
                snapshots every 32 levels (the adjoint recomputes each segment)
                and with all states kept
  batch         256 independent problems (n log-uniform in [511, 16383],
                alpha ~ U(1.1, 1.9), gamma ~ U(0.2, 0.8), M = 256), one
                workgroup each, all levels in one launch: problem-levels/s
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

FORMS = {
    "headline": dict(solver=2, precision=0, x0_mode=3, label="pcg-symmetrised-fp64-x0cubic"),
    "fgmres": dict(solver=1, precision=0, x0_mode=3, label="fgmres(20)-fp64-x0cubic"),
    "linear_x0": dict(solver=1, precision=0, x0_mode=1, label="fgmres(20)-fp64-x0linear"),
    "quad_x0": dict(solver=1, precision=0, x0_mode=2, label="fgmres(20)-fp64-x0quad"),
    "plain": dict(solver=0, precision=0, x0_mode=0, label="bicgstab-fp64-x0zero"),
    "mixed": dict(solver=1, precision=1, x0_mode=3, label="fgmres(20)-fp64/fp32pc-x0cubic"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed full solves (M levels each)")
    ap.add_argument("--warmup", type=int, default=1, help="untimed full solves before them")
    ap.add_argument("--window", type=int, default=20, help="levels of the reported early window")
    ap.add_argument("--n", type=int, default=65535)
    ap.add_argument("--M", type=int, default=2048)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--forms", default="headline,fgmres,plain,mixed")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-levels", type=int, default=100)
    ap.add_argument("--cpu-n", type=int, default=4095)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2-D extension's leg")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--table11", action="store_true",
                    help="Table 11 rows (Example 2) on the GPU: fast/direct history, with/without preconditioner")
    ap.add_argument("--profile-pass", nargs="?", const="headline", choices=["headline", "batch", "2d"],
                    help="a 256 MiB device copy, then one launch of the level kernel over all levels: the "
                         "headline form (default) or the 256-problem batch in its PCG form (for counters)")
    return ap.parse_args()


def workload(n, M):
    from paper_2002_11978_amd import workloads as W
    return W.seeded(1.5, 0.4, n, M, r=4.0, kappa_seed=3, f_seed=4, name="bench")


def level_bytes(form, n, nexp, iters, matvecs, restart=20, cfg=None):
    """Compulsory HBM bytes of one level (FP64 8 B per value; every vector is
    read or written once per use in the method; symbols count n values):
      SOE update + right-hand side: F read and written (16 n nexp), u^{m-1},
        u^{m-2}, f^m, kappa^m read and b written (40 n);
      BiCGSTAB, per iteration (2 matvecs, 2 preconditioner applications, 7
        dot products, 4 vector updates): 280 n;
      PCG, per iteration: P^{-1} on K^{-1} r (r, kbar/kappa, symbol read, u
        written) 32 n, matvec with the two dots (symbol, kappa, u, r read, w
        written) 40 n, updates of p, s, x, r (u, w, p, s, x, r read, p, s,
        x, r written) 80 n; per level the true residual of the result (x,
        symbol, kappa, b read, r and A x written) 48 n, and with an initial
        guess the same for its initial residual;
      FGMRES, Arnoldi step j (0-based within a cycle): matvec 32 n, P^{-1}
        apply 24 n, dots with v_0..v_j 8 n (j+1), forming z_{j+1} and v_{j+1}
        from z_0..z_j, v_0..v_j 16 n (j+1) + 24 n, re-orthogonalisation dots
        8 n (j+2); plus per level the update x += Z y (8 n (it+2)) and the
        true residual (48 n).
    """
    cfg = cfg if cfg is not None else FORMS[form]
    b = 16.0 * n * nexp + 40.0 * n
    if cfg["solver"] == 0:
        return b + 140.0 * n * matvecs
    if cfg["solver"] == 2:
        checks = max(1, matvecs - iters - (1 if cfg["x0_mode"] else 0))   # true-residual passes
        return b + (48.0 * n if cfg["x0_mode"] else 0.0) + 48.0 * n * checks + 152.0 * n * iters
    zb = 4.0 if cfg["precision"] == 1 else 8.0
    for i in range(iters):
        j = i % restart
        b += 32 * n + 24 * n + 8 * n * (j + 1) + (8 + zb) * n * (j + 1) + 24 * n + 8 * n * (j + 2)
    b += zb * n * (min(iters, restart) + 2) + 48.0 * n
    return b


def cpu_baseline(args):
    """Oracle (direct scheme, dense LU per level, full history) on the first
    levels of the same recipe at n = cpu_n; reported in levels/s."""
    import scipy.linalg as sla

    import oracle
    pb = workload(args.cpu_n, args.M)
    K = args.cpu_levels
    t0 = time.perf_counter()
    A = oracle.ifl_matrix(pb.n, pb.alpha)
    g = 1.0 / math.gamma(1.0 - pb.gamma)
    U = np.empty((K + 1, pb.n))
    U[0] = pb.phi
    for m in range(1, K + 1):
        a = oracle.l1_weights(1.0, pb.M, pb.r, pb.gamma, m)
        rhs = g * a[0] * U[0] + pb.f[m - 1]
        if m > 1:
            rhs = rhs + g * (np.diff(a)[: m - 1] @ U[1:m])
        Mm = pb.kappa[m - 1][:, None] * A
        Mm[np.diag_indices(pb.n)] += g * a[m - 1]
        U[m] = sla.solve(Mm, rhs)
    dt = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"value": K / dt, "unit": "levels/s", "cores": cores, "kind": "oracle",
            "sample": f"direct scheme + LAPACK dense LU (all host threads), first {K} of M={pb.M} levels of the "
                      f"same recipe at n={pb.n}; a dense LU at n=65535 does not fit a bounded run; {dt:.1f} s"}


def adjoint_leg(tol):
    """Forward solve and discrete adjoint of J = ||u^M||^2 at n = 16383, M = 1024."""
    import torch

    from paper_2002_11978_amd import fids
    from paper_2002_11978_amd import workloads as W
    pb = W.seeded(1.6, 0.5, 16383, 1024, r=3.0, kappa_seed=5, f_seed=7, time_dependent=False)
    dev = torch.device("cuda:0")
    k, f, phi = (torch.from_numpy(a).to(dev) for a in (pb.kappa, pb.f, pb.phi))
    out = {"workload": "n=16383, M=1024, alpha=1.6, gamma=0.5, r=3, time-independent kappa (seed 5), f seed 7",
           "form": FORMS["headline"]["label"]}
    for name, extra in (("checkpoint_32", dict(checkpoint_every=32)), ("stored_states", dict(store_states=1))):
        prm = fids.default_params(alpha=pb.alpha, gamma=pb.gamma, n=pb.n, M=pb.M, r=pb.r, soe_tol=1e-10,
                                  krylov_tol=tol, krylov_maxit=500, kappa_time_dependent=0,
                                  solver=FORMS["headline"]["solver"], x0_mode=3, **extra)
        prob = fids.Problem(prm, k, f, phi)
        best = None
        for _ in range(2):
            prob.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            uT, _, _ = prob.solve_all()
            torch.cuda.synchronize()
            tf = time.perf_counter() - t0
            dJ = (2.0 * uT).contiguous()
            t0 = time.perf_counter()
            prob.adjoint(dJ)
            torch.cuda.synchronize()
            ta = time.perf_counter() - t0
            if best is None or tf + ta < best[0] + best[1]:
                best = (tf, ta)
        reps = prob.adjoint_reports()
        out[name] = {"fwd_ms": best[0] * 1e3, "adj_ms": best[1] * 1e3, "adj_over_fwd": best[1] / best[0],
                     "adj_avg_iters": float(np.mean([r.iters for r in reps]))}
        print(f"[bench] adjoint {name}: fwd {best[0] * 1e3:.1f} ms, adjoint {best[1] * 1e3:.1f} ms, "
              f"ratio {best[1] / best[0]:.2f}", file=sys.stderr, flush=True)
        prob.close()
    out["adj_over_fwd"] = out["checkpoint_32"]["adj_over_fwd"]
    return out


def leg_2d(tol, n=255, M=256, forms=("headline", "fgmres"), kernel_only=False):
    """The 2-D extension (dims = 2) on (-1, 1)^2 with n nodes per axis: full
    solves of M levels (symbols built inside) and one kernel-only launch of
    the level kernel over all levels, in the headline's PCG form and FGMRES.
    Algorithmic bytes use the n^2 unknowns (the padded rows the library
    streams hold about twice as many slots, see `padded_len`)."""
    import torch

    from paper_2002_11978_amd import fids
    from paper_2002_11978_amd import workloads as W
    pb = W.seeded2d(1.5, 0.4, n, M, r=4.0, kappa_seed=61, f_seed=62)
    dev = torch.device("cuda:0")
    k, f, phi = (torch.from_numpy(a).to(dev) for a in (pb.kappa, pb.f, pb.phi))
    out = {"workload": f"2-D square (-1,1)^2, n={n} nodes per axis ({n * n} unknowns), M={M}, alpha=1.5, "
                       f"gamma=0.4, r=4, seeded kappa(x,y,t), f(x,y,t), phi=(1-|x|^2)_+^(alpha/2)"}
    for form in forms:
        cfg = {kk: v for kk, v in FORMS[form].items() if kk != "label"}
        prm = fids.default_params(alpha=pb.alpha, gamma=pb.gamma, n=n, M=M, r=pb.r, soe_tol=1e-10,
                                  krylov_tol=tol, krylov_maxit=500, kappa_time_dependent=1, dims=2, **cfg)
        prob = fids.Problem(prm, k, f, phi)
        infos = (fids.StepInfo * M)()
        best = None
        for rep in range(0 if kernel_only else 3):
            prob.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = prob.solve_all_raw(None, None, infos)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if st != 0:
                raise fids.FidsError(st, "fids_solve_all")
            if rep > 0 and (best is None or dt < best):
                best = dt
        prob.reset()
        prob.prepare()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(prob.stream)
        st = prob.solve_all_raw(None, None, infos)
        e1.record(prob.stream)
        torch.cuda.synchronize()
        kern = e0.elapsed_time(e1)
        if kernel_only:                 # the counter pass: one launch, handle closed
            prob.close()
            if st != 0:
                raise fids.FidsError(st, "fids_solve_all")
            return kern
        its = np.array([infos[i].iters for i in range(M)])
        mvs = np.array([infos[i].matvecs for i in range(M)])
        rr = max(infos[i].relres for i in range(M))
        nexp = len(fids.soe_nodes(pb.gamma, pb.T * (1.0 / M) ** pb.r, pb.T, 1e-10)[0])   # delta = tau_1
        byts = sum(level_bytes(form, n * n, nexp, int(its[i]), int(mvs[i])) for i in range(M))
        ach = byts / (kern * 1e-3) / 1e9
        out[form] = {"form": FORMS[form]["label"], "levels_per_s": M / best, "solve_ms": best * 1e3,
                     "kernel_ms": kern, "avg_iters": float(its.mean()), "relres_max": rr,
                     "padded_len": fids.toeplitz_len(prm),
                     "roofline": {"bound": "hbm", "achieved": ach, "peak": 8000.0, "unit": "GB/s",
                                  "frac": ach / 8000.0, "bytes_per_launch": byts, "traffic": None}}
        tr = measured_traffic(n, M, TRAFFIC_2D_FILE, "2-D " + FORMS[form]["label"]) if form == "headline" else None
        if tr is not None:
            out[form]["roofline"]["traffic"] = tr["traffic_bytes_per_launch"]
            out[form]["roofline"]["traffic_source"] = os.path.relpath(TRAFFIC_2D_FILE,
                                                                    os.path.dirname(os.path.abspath(__file__)))
        print(f"[bench] 2-D {form}: n={n}^2 M={M}: {M / best:.0f} levels/s ({best * 1e3:.1f} ms per solve), "
              f"kernel {kern:.1f} ms, its {its.mean():.2f}, relres_max {rr:.2e}, {ach:.0f} GB/s algorithmic",
              file=sys.stderr, flush=True)
        prob.close()
    return out


def batch_leg(tol, count):
    """256 heterogeneous problems advanced together; problem-levels/s."""
    import torch

    from paper_2002_11978_amd import fids
    from paper_2002_11978_amd import workloads as W
    M = 256
    pbs = [W.batch_member(p, M=M) for p in range(count)]
    nexps = [int(fids.soe_nodes(pb.gamma, (1.0 / M) ** pb.r, 1.0, 1e-10)[0].size) for pb in pbs]
    dev = torch.device("cuda:0")
    arrs = [[torch.from_numpy(getattr(pb, a)).to(dev) for pb in pbs] for a in ("kappa", "f", "phi")]
    out = {"workload": f"{count} problems, n log-uniform in [511, 16383] (sum {sum(pb.n for pb in pbs)}), "
                       f"alpha~U(1.1,1.9), gamma~U(0.2,0.8), r=(2-gamma)/gamma, M={M}, seeded kappa(x,t), f(x,t)",
           "count": count, "M": M}
    for name, cfg in (("fp64", dict(solver=1, precision=0, x0_mode=3, precond=2)),
                      ("mixed", dict(solver=1, precision=1, x0_mode=3, precond=2)),
                      ("pcg", dict(solver=2, precision=0, x0_mode=3, precond=2)),
                      ("pcg_graph", dict(solver=2, precision=0, x0_mode=3, precond=2))):
        params = [fids.default_params(alpha=pb.alpha, gamma=pb.gamma, n=pb.n, M=M, r=pb.r, soe_tol=1e-10,
                                      krylov_tol=tol, krylov_maxit=500, **cfg) for pb in pbs]
        t0 = time.perf_counter()
        if name.endswith("_graph"):
            # one captured HIP-graph launch per level, every member on one workgroup
            os.environ["FIDS_BATCH_MODE"] = "graph"
        try:
            b = fids.Batch(params, *arrs)
        finally:
            os.environ.pop("FIDS_BATCH_MODE", None)
        t_init = time.perf_counter() - t0
        t0 = time.perf_counter()
        b.tune(levels=4)
        t_tune = time.perf_counter() - t0
        infos = (fids.StepInfo * (count * M))()
        best = None
        for _ in range(3):
            b.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = b.solve_all_raw(None, infos)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if st != 0:
                raise fids.FidsError(st, "fids_batch_solve_all")
            best = dt if best is None else min(best, dt)
        # the level kernel alone (symbols built first), for the roofline
        b.reset()
        b.prepare()
        torch.cuda.synchronize()
        k0 = torch.cuda.Event(enable_timing=True)
        k1 = torch.cuda.Event(enable_timing=True)
        k0.record(b.stream)
        st = b.solve_all_raw(None, infos)
        k1.record(b.stream)
        torch.cuda.synchronize()
        if st != 0:
            raise fids.FidsError(st, "fids_batch_solve_all")
        kern_ms = k0.elapsed_time(k1)
        its = np.array([infos[i].iters for i in range(count * M)])
        mvs = np.array([infos[i].matvecs for i in range(count * M)])
        fb = np.array([infos[i].pc_fp64_iters for i in range(count * M)])
        # algorithmic bytes of the launch: the per-level model of each member
        nbytes = 0.0
        for p_i, pb in enumerate(pbs):
            for m in range(M):
                k = p_i * M + m
                nbytes += level_bytes(None, pb.n, nexps[p_i], int(its[k]), int(mvs[k]), cfg=cfg)
        gbs = nbytes / (kern_ms * 1e-3) / 1e9
        out[name] = {"problem_levels_per_s": count * M / best, "solve_ms": best * 1e3, "init_s": t_init,
                     "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": gbs / HBM_PEAK_GBS, "bytes_per_launch": nbytes,
                                  "kernel_ms_per_launch": kern_ms, "kernel": "k_levels",
                                  "launch": f"all {M} levels of the {count} members, symbols prepared",
                                  "traffic": None},
                     "tune_s": t_tune,
                     "avg_iters": float(its.mean()), "levels_with_fp64_pc": int((fb > 0).sum()),
                     "launch_mode": ("one captured HIP-graph launch per level, one workgroup per member"
                                     if name.endswith("_graph") else "one persistent launch for all levels"),
                     "form": ("pcg-symmetrised-fp64-x0cubic-strang" if cfg["solver"] == 2 else
                              f"fgmres(20)-{'fp64' if cfg['precision'] == 0 else 'fp64/fp32pc'}-x0cubic-"
                              "kappa-scaled-strang")}
        tr = (measured_traffic(None, M, BATCH_TRAFFIC_FILE, "batch pcg-symmetrised-fp64-x0cubic", count)
              if name == "pcg" else None)
        if tr is not None:
            out[name]["roofline"]["traffic"] = tr["traffic_bytes_per_launch"]
            out[name]["roofline"]["traffic_source"] = os.path.relpath(BATCH_TRAFFIC_FILE,
                                                                      os.path.dirname(os.path.abspath(__file__)))
        print(f"[bench] batch {name}: {count * M / best:.0f} problem-levels/s ({best * 1e3:.1f} ms), "
              f"its {its.mean():.2f}, fp64-pc levels {(fb > 0).sum()}, kernel {kern_ms:.1f} ms, "
              f"{gbs:.0f} GB/s algorithmic",
              file=sys.stderr, flush=True)
        b.close()
    return out


# Table 11 rows (r, gamma, alpha, N_p, M) with the paper's printed Err_inf and
# FIDS+P iterations per level and CPU seconds (i5-8265U, MATLAB; context only)
TABLE11 = [
    (2, 0.5, 1.5, 64, 431, 6.362e-4, 7.7, 0.347), (2, 0.5, 1.5, 128, 1449, 1.542e-4, 7.9, 1.689),
    (2, 0.5, 1.5, 256, 4871, 4.469e-5, 8.0, 6.698), (2, 0.5, 1.5, 512, 16384, 1.333e-5, 8.2, 43.338),
    (3, 0.8, 1.5, 128, 431, 1.381e-4, 6.6, 0.439), (3, 0.8, 1.5, 256, 1184, 3.265e-5, 6.9, 1.545),
    (3, 0.8, 1.5, 512, 3251, 7.897e-6, 7.1, 8.143), (3, 0.8, 1.5, 1024, 8934, 2.319e-6, 7.0, 34.543),
    (2, 0.5, 1.9, 64, 862, 1.446e-3, 7.9, 0.748), (2, 0.5, 1.9, 128, 3327, 3.533e-4, 7.9, 3.838),
    (2, 0.5, 1.9, 256, 12855, 8.636e-5, 8.1, 18.073), (2, 0.5, 1.9, 512, 49668, 2.112e-5, 8.1, 132.04),
    (3, 0.8, 1.9, 128, 862, 3.521e-4, 7.3, 1.049), (3, 0.8, 1.9, 256, 2656, 8.596e-5, 7.3, 3.679),
    (3, 0.8, 1.9, 512, 8192, 2.100e-5, 7.4, 21.436), (3, 0.8, 1.9, 1024, 25268, 5.136e-6, 7.3, 86.540),
]


def table11_leg():
    """Example 2 at the Table 11 sizes with the paper's solver settings
    (BiCGSTAB, tol 1e-10, zero initial guess, SOE 1e-9): fast history with the
    Strang preconditioner (FIDS+P), without it (FIDS+I), the direct history
    with and without it (DIDS+P, DIDS+I), and FIDS+P with conjugate gradients
    on the symmetrised system instead of BiCGSTAB; Err_inf against the exact
    solution."""
    import torch

    from paper_2002_11978_amd import fids
    from paper_2002_11978_amd import workloads as W
    dev = torch.device("cuda:0")
    rows = []
    for (r, g, a, Np, M, err_p, its_p, cpu_s) in TABLE11:
        pb = W.example2(a, g, r, Np, M)
        k, f, phi = (torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (pb.kappa, pb.f, pb.phi))
        row = {"r": r, "gamma": g, "alpha": a, "N": Np, "M": M, "paper_err_inf": err_p, "paper_its": its_p,
               "paper_cpu_s": cpu_s}
        for name, extra in (("fids_p", dict(precond=0, history=0)), ("fids_i", dict(precond=1, history=0)),
                            ("dids_p", dict(precond=0, history=1)), ("dids_i", dict(precond=1, history=1)),
                            ("fids_p_pcg", dict(precond=0, history=0, solver=2))):
            # unpreconditioned runs take 100-300 iterations a level: the
            # largest rows are left out to keep the leg to a few minutes
            if extra["precond"] == 1 and M > 13000:
                continue
            kw = dict(solver=0, precision=0, x0_mode=0, store_states=int(extra["history"] == 0))
            kw.update(extra)
            prm = fids.default_params(alpha=a, gamma=g, n=pb.n, M=M, r=r, soe_tol=1e-9, krylov_tol=1e-10,
                                      krylov_maxit=2000, **kw)
            prob = fids.Problem(prm, k, f, phi)
            prob.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            uT, U, reps = prob.solve_all(return_all=True)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ei = float(np.max(np.abs(U.cpu().numpy() - pb.exact)))      # Err_inf = max_m ||u^m - u(t_m)||_inf
            # the paper's Its is matvecs / 2 for BiCGSTAB; CG iterations for PCG
            its = (np.mean([x.iters for x in reps]) if kw["solver"] == 2
                   else np.mean([x.matvecs for x in reps]) / 2)
            row[name] = {"s": dt, "levels_per_s": M / dt, "its": float(its), "err_inf": ei}
            prob.close()
        print(f"[bench] table11 {row}", file=sys.stderr, flush=True)
        rows.append(row)
    return rows


class Runner:
    def __init__(self, pb, form, tol, dev):
        import torch

        from paper_2002_11978_amd import fids
        self.fids, self.torch = fids, torch
        cfg = {k: v for k, v in FORMS[form].items() if k != "label"}
        self.params = fids.default_params(alpha=pb.alpha, gamma=pb.gamma, n=pb.n, M=pb.M, r=pb.r,
                                          soe_tol=1e-10, krylov_tol=tol, krylov_maxit=500,
                                          kappa_time_dependent=1, **cfg)
        self.prob = fids.Problem(self.params, pb.kappa_d, pb.f_d, pb.phi_d)
        self.M = pb.M
        self.level = 0
        self.infos = (fids.StepInfo * pb.M)()

    def levels(self, K):
        """Advance exactly K levels from the current one, one fids_solve_levels
        call per run up to level M (then back to level 0)."""
        done = 0
        while done < K:
            if self.level == self.M:
                self.prob.reset()
                self.level = 0
            c = min(K - done, self.M - self.level)
            st = self.prob.solve_levels_raw(c)
            if st != 0:
                raise self.fids.FidsError(st, "fids_solve_levels")
            self.level += c
            done += c

    def timed(self, K, W):
        """W untimed levels from level 0, then K timed levels (wall clock and
        HIP events on the problem's stream)."""
        torch = self.torch
        self.prob.reset()
        self.level = 0
        self.levels(W)
        first = self.level % self.M + 1
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(self.prob.stream)
        self.levels(K)
        e1.record(self.prob.stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, e0.elapsed_time(e1), first

    def solves(self, K, W):
        """W untimed full solves, then K timed full solves from level 0 (each
        a reset and one launch over all M levels, symbols built inside)."""
        torch = self.torch
        for _ in range(W):
            self.prob.reset()
            st = self.prob.solve_all_raw(None, None, self.infos)
            if st != 0:
                raise self.fids.FidsError(st, "fids_solve_all")
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(self.prob.stream)
        for _ in range(K):
            self.prob.reset()
            st = self.prob.solve_all_raw(None, None, self.infos)
            if st != 0:
                raise self.fids.FidsError(st, "fids_solve_all")
        e1.record(self.prob.stream)
        torch.cuda.synchronize()
        self.level = self.M
        return time.perf_counter() - t0, e0.elapsed_time(e1)

    def kernel_only(self):
        """One launch of the level kernel over all M levels (symbols prepared
        first), timed by HIP events on the problem's stream."""
        torch = self.torch
        self.prob.reset()
        self.prob.prepare()
        torch.cuda.synchronize()
        k0 = torch.cuda.Event(enable_timing=True)
        k1 = torch.cuda.Event(enable_timing=True)
        k0.record(self.prob.stream)
        st = self.prob.solve_all_raw(None, None, self.infos)
        k1.record(self.prob.stream)
        torch.cuda.synchronize()
        self.level = self.M
        if st != 0:
            raise self.fids.FidsError(st, "fids_solve_all")
        return k0.elapsed_time(k1)

    def full_solve(self):
        """A full solve from level 0 (symbols built inside): (u^M, seconds)."""
        torch = self.torch
        self.prob.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        uT, _, reps = self.prob.solve_all()
        torch.cuda.synchronize()
        self.level = self.M
        return uT.cpu().numpy(), time.perf_counter() - t0, reps

    def close(self):
        self.prob.close()


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "k_levels_n65535_M2048_traffic.json")
BATCH_TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                                  "k_levels_batch256_M256_traffic.json")
TRAFFIC_2D_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "k_levels_2d_n255_M256_traffic.json")
KERNEL_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2002_11978_amd", "csrc",
                          "fids_kernels.hip")


def measured_traffic(n, M, path=TRAFFIC_FILE, form=None, count=None):
    """HBM bytes per launch of the level kernel from a committed counter
    summary, or None if it is missing, for another workload, or was taken
    from a different kernel source."""
    import hashlib
    try:
        with open(path) as fh:
            t = json.load(fh)
        with open(KERNEL_SRC, "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
    except OSError:
        return None
    if t.get("kernel_sha256") != sha or t.get("M") != M:
        return None
    if count is not None:
        if t.get("count") != count:
            return None
    elif t.get("n") != n:
        return None
    if not str(t.get("form", "")).startswith(form or FORMS["headline"]["label"]):
        return None
    return t


def profile_pass(args):
    """Counter pass: one plain device copy of 256 MiB whose FETCH_SIZE /
    WRITE_SIZE calibrate the counters, then one launch of the level kernel
    over all levels with the symbols built before it (the headline form, or
    the 256-problem batch in its PCG form).  Every handle is closed before
    the interpreter shuts down."""
    import torch
    dev = torch.device("cuda:0")
    src = torch.ones(32 << 20, dtype=torch.float64, device=dev)      # 256 MiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    if args.profile_pass == "batch":
        profile_batch(args, dev)
        del src, dst
        torch.cuda.synchronize()
        return
    if args.profile_pass == "2d":
        ms = leg_2d(args.tol, forms=("headline",), kernel_only=True)
        del src, dst
        torch.cuda.synchronize()
        print(f"[profile-pass] copy 256 MiB, 2-D k_levels {ms:.1f} ms", file=sys.stderr, flush=True)
        return
    pb = workload(args.n, args.M)
    pb.kappa_d, pb.f_d, pb.phi_d = (torch.from_numpy(a).to(dev) for a in (pb.kappa, pb.f, pb.phi))
    run = Runner(pb, "headline", args.tol, dev)
    ms = run.kernel_only()
    run.close()                       # release the handle before the interpreter shuts down
    del src, dst
    torch.cuda.synchronize()
    print(f"[profile-pass] copy 256 MiB, k_levels {ms:.1f} ms", file=sys.stderr, flush=True)


def profile_batch(args, dev):
    """One persistent launch of the 256-problem batch (PCG form, tuned tiles,
    symbols built first): the launch the batch roofline is computed for."""
    import torch

    from paper_2002_11978_amd import fids
    from paper_2002_11978_amd import workloads as W
    M = 256
    pbs = [W.batch_member(p, M=M) for p in range(args.batch_count)]
    arrs = [[torch.from_numpy(getattr(pb, a)).to(dev) for pb in pbs] for a in ("kappa", "f", "phi")]
    params = [fids.default_params(alpha=pb.alpha, gamma=pb.gamma, n=pb.n, M=M, r=pb.r, soe_tol=1e-10,
                                  krylov_tol=args.tol, krylov_maxit=500, solver=2, precision=0, x0_mode=3, precond=2)
              for pb in pbs]
    b = fids.Batch(params, *arrs)
    b.tune(levels=4)
    b.reset()
    b.prepare()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    st = b.solve_all_raw(None, None)
    e1.record(b.stream)
    torch.cuda.synchronize()
    b.close()
    if st != 0:
        raise fids.FidsError(st, "fids_batch_solve_all")
    print(f"[profile-pass] copy 256 MiB, batch launch {e0.elapsed_time(e1):.1f} ms", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); independent problems shard "
              "across GPUs without communication", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2002_11978_amd import fids

    if args.profile_pass:
        profile_pass(args)
        return
    dev = torch.device("cuda:0")
    pb = workload(args.n, args.M)
    pb.kappa_d = torch.from_numpy(pb.kappa).to(dev)
    pb.f_d = torch.from_numpy(pb.f).to(dev)
    pb.phi_d = torch.from_numpy(pb.phi).to(dev)
    nexp = int(fids.soe_nodes(pb.gamma, (1.0 / pb.M) ** pb.r, 1.0, 1e-10)[0].size)
    forms = [f for f in args.forms.split(",") if f]
    res = {}
    finals = {}
    ref_uT = None
    for form in forms:
        run = Runner(pb, form, args.tol, dev)
        K = args.steps if form == forms[0] else max(1, min(args.steps, 2))
        Wu = args.warmup if form == forms[0] else 1
        print(f"[bench] {form}: n={pb.n} M={pb.M} ws={run.prob.ws_bytes / 2**20:.0f} MiB "
              f"warmup={Wu} timed={K} full solves", file=sys.stderr, flush=True)
        wall, ev_ms = run.solves(K, Wu)
        win = min(args.window, pb.M - 5)
        wwall, _, first = run.timed(win, 5)
        uT, full_s, reps = run.full_solve()
        kern_ms = run.kernel_only()
        mv = np.array([run.infos[i].matvecs for i in range(pb.M)])
        it = np.array([run.infos[i].iters for i in range(pb.M)])
        rr = np.array([run.infos[i].relres for i in range(pb.M)])
        fl = np.array([run.infos[i].flags for i in range(pb.M)])
        nbytes = float(sum(level_bytes(form, pb.n, nexp, int(it[i]), int(mv[i])) for i in range(pb.M)))
        finals[form] = uT
        if ref_uT is None:
            ref_uT = uT
        res[form] = dict(value=K * pb.M / wall, solves_timed=K, ms_per_solve=wall * 1e3 / K, event_ms=ev_ms,
                         window_levels_per_s=win / wwall, window_levels=[first, first + win - 1],
                         kernel_ms=kern_ms, kernel_levels_per_s=pb.M / (kern_ms * 1e-3), bytes=nbytes,
                         avg_iters=float(it.mean()), avg_matvecs=float(mv.mean()), relres_max=float(rr.max()),
                         levels_above_tol=int(((fl & fids.FIDS_LEVEL_ABOVE_TOL) != 0).sum()),
                         uT_rel_diff=float(np.max(np.abs(uT - ref_uT)) / np.max(np.abs(ref_uT))),
                         label=FORMS[form]["label"])
        print(f"[bench] {form}: {res[form]['value']:.1f} levels/s over {K} full solves, kernel {kern_ms:.1f} ms, "
              f"window {first}..{first + win - 1} {win / wwall:.1f} levels/s, its {it.mean():.2f}, "
              f"matvecs {mv.mean():.2f}, relres_max {rr.max():.2e}, above tol {res[form]['levels_above_tol']}, "
              f"uT diff {res[form]['uT_rel_diff']:.2e}", file=sys.stderr, flush=True)
        run.close()
    head = res[forms[0]]
    achieved = head["bytes"] / (head["kernel_ms"] * 1e-3) / 1e9
    out = {
        "metric": "solved time steps/s at N=65535,M=2048 vs plain FP64; % HBM peak; adj/fwd ratio",
        "value": head["value"],
        "unit": "time steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"1-D time-space fractional diffusion (IFL), n={pb.n} interior nodes, "
                               f"M={pb.M} graded levels, alpha=1.5, gamma=0.4, r=4, seeded kappa(x,t), f(x,t)",
                   "n": pb.n, "M": pb.M, "form": head["label"], "krylov_tol": args.tol, "soe_tol": 1e-10,
                   "nexp": nexp, "step": f"one full solve of all {pb.M} levels from level 0",
                   "levels_per_step": pb.M,
                   "avg_iterations": head["avg_iters"], "levels_above_tol": head["levels_above_tol"],
                   "parallelism": "single GPU"},
        "forms": {f: {k: v for k, v in r.items()} for f, r in res.items()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_levels",
                     "launch": f"all {pb.M} levels of the headline form, symbols prepared",
                     "kernel_ms_per_launch": head["kernel_ms"], "bytes_per_launch": head["bytes"]},
    }
    tr = measured_traffic(pb.n, pb.M) if forms[0] == "headline" else None
    if tr is not None:
        out["roofline"]["traffic"] = tr["traffic_bytes_per_launch"]
        out["roofline"]["traffic_source"] = os.path.relpath(TRAFFIC_FILE, os.path.dirname(os.path.abspath(__file__)))
    if "plain" in res:
        out["speedup_vs_plain_fp64"] = head["value"] / res["plain"]["value"]
        out["speedup_vs_plain_fp64_kernel"] = res["plain"]["kernel_ms"] / head["kernel_ms"]
        pl = finals["plain"]
        for f in res:
            res[f]["uT_rel_diff_vs_plain_fp64"] = float(np.max(np.abs(finals[f] - pl)) / np.max(np.abs(pl)))
        out["forms"] = {f: {k: v for k, v in r.items()} for f, r in res.items()}
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(args.tol)
        out["adj_fwd_ratio"] = out["adjoint"]["adj_over_fwd"]
    if not args.no_batch:
        out["batch"] = batch_leg(args.tol, args.batch_count)
    if not args.no_2d:
        out["two_d"] = leg_2d(args.tol)
    if args.table11:
        out["table11"] = table11_leg()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
