"""Pin the oracle's discrete adjoint (``dids_adjoint``) by central finite
differences of the oracle's own forward solve.

J = sum_i (u^M_i - u*_i)^2 is quadratic in (f, phi), so central differences
along f and phi are exact up to rounding; along kappa they carry O(eps^2).
"""
import numpy as np
import pytest

import oracle
from paper_2002_11978_amd import workloads as W


def _setup(time_dependent):
    pb = W.seeded(1.6, 0.5, 31, 12, kappa_seed=5, f_seed=7, time_dependent=time_dependent)
    target = W.seeded(1.6, 0.5, 31, 12, kappa_seed=6, f_seed=7, time_dependent=time_dependent)
    Ut = oracle.dids_solve(target.alpha, target.gamma, target.n, target.M, target.r,
                           target.kappa, target.f, target.phi)
    return pb, Ut[-1]


def _loss(pb, ustar, kappa, f, phi):
    U = oracle.dids_solve(pb.alpha, pb.gamma, pb.n, pb.M, pb.r, kappa, f, phi)
    return float(np.sum((U[-1] - ustar) ** 2)), U


@pytest.mark.parametrize("time_dependent", [False, True])
def test_dids_adjoint_matches_central_differences(time_dependent):
    pb, ustar = _setup(time_dependent)
    J0, U = _loss(pb, ustar, pb.kappa, pb.f, pb.phi)
    gk, gf, gp = oracle.dids_adjoint(pb.alpha, pb.gamma, pb.n, pb.M, pb.r, pb.kappa, pb.f,
                                     pb.phi, 2 * (U[-1] - ustar), U=U)
    rng = np.random.Generator(np.random.PCG64(8))
    for _ in range(4):
        dk = rng.normal(size=pb.kappa.shape)
        df = rng.normal(size=pb.f.shape)
        dp = rng.normal(size=pb.phi.shape)
        nrm = np.sqrt(np.sum(dk * dk) + np.sum(df * df) + np.sum(dp * dp))
        dk, df, dp = dk / nrm, df / nrm, dp / nrm
        eps = 1e-5
        Jp, _ = _loss(pb, ustar, pb.kappa + eps * dk, pb.f + eps * df, pb.phi + eps * dp)
        Jm, _ = _loss(pb, ustar, pb.kappa - eps * dk, pb.f - eps * df, pb.phi - eps * dp)
        fd = (Jp - Jm) / (2 * eps)
        ad = np.sum(gk * dk) + np.sum(gf * df) + np.sum(gp * dp)
        assert abs(fd - ad) <= 1e-7 * (abs(ad) + 1e-12 * J0), (fd, ad)
    # the f and phi parts alone are exact for a quadratic loss
    df = rng.normal(size=pb.f.shape)
    Jp, _ = _loss(pb, ustar, pb.kappa, pb.f + df, pb.phi)
    Jm, _ = _loss(pb, ustar, pb.kappa, pb.f - df, pb.phi)
    assert abs((Jp - Jm) / 2 - np.sum(gf * df)) <= 1e-9 * abs(np.sum(gf * df))
