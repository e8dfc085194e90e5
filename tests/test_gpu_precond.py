"""GPU check of the per-level Strang preconditioner itself (eq. 4.3), not
only through iteration counts: the device builds, for every level m, the
first column q of P_m^{-1}, P_m = b_m' I + kbar_m s(A), by a Bluestein DFT of
1 / (b_m' + kbar_m lam_k), and the real spectrum qhat of q's length-L
circulant embedding, through which the solver applies P_m^{-1}.  Reference:
P_m assembled as a dense n x n circulant from the oracle's Strang column
(c_S after eq. 4.3) and inverted by a dense solve; the embedding's spectrum
from a direct real FFT of that column.  Tolerance: 50 u cond(P_m) for q (both
sides solve the same system; u = 2^-53), plus 1e-13 of max |qhat| for the
spectrum.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_2002_11978_amd import fids
from paper_2002_11978_amd import workloads as W

from gpu_util import say, to_dev

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.mark.parametrize("n,alpha,gamma", [(1, 1.5, 0.5), (2, 1.5, 0.5), (257, 1.5, 0.5), (1000, 1.2, 0.3),
                                           (4095, 1.8, 0.7), (4095, 1.5, 0.4)])
@pytest.mark.parametrize("precond", [0, 2], ids=["strang", "strang-kappa-scaled"])
def test_strang_inverse_against_dense(n, alpha, gamma, precond):
    M = 64
    pb = W.seeded(alpha, gamma, n, M, kappa_seed=1, f_seed=2)
    params = fids.default_params(alpha=pb.alpha, gamma=pb.gamma, n=n, M=M, r=pb.r, precond=precond)
    prob = fids.Problem(params, to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi))
    cS = oracle.strang_column(oracle.ifl_column(n, alpha))
    g = 1.0 / math.gamma(1.0 - gamma)
    L = max(4, 1 << int(math.ceil(math.log2(2 * n))))
    e0 = np.zeros(n)
    e0[0] = 1.0
    for m in (1, 2, M // 2, M):
        bm = g * oracle.l1_weights(1.0, M, pb.r, gamma, m)[m - 1]
        kb = float(np.mean(pb.kappa[m - 1]))
        P = sla.circulant(bm * e0 + kb * cS)
        qref = np.linalg.solve(P, e0)
        lam = np.fft.fft(bm * e0 + kb * cS).real      # a circulant's eigenvalues (sizes the gate only)
        cond = float(np.abs(lam).max() / np.abs(lam).min())
        q, qhat = prob.precond_symbol(m)
        err = float(np.max(np.abs(q - qref)) / np.max(np.abs(qref)))
        emb = np.zeros(L)
        emb[:n] = qref
        if n > 1:
            emb[L - n + 1:] = qref[1:][::-1]
        ref_hat = np.fft.rfft(emb).real
        err_hat = float(np.max(np.abs(qhat - ref_hat)) / np.max(np.abs(ref_hat)))
        gate = 50.0 * U * cond
        say(f"  n={n} alpha={alpha} m={m}: q rel err {err:.2e} (gate {gate:.2e}, cond {cond:.2e}), "
            f"qhat rel err {err_hat:.2e}")
        assert err <= gate
        assert err_hat <= gate + 1e-13
    prob.close()


def test_identity_preconditioner_symbol():
    pb = W.seeded(1.5, 0.4, 300, 8)
    params = fids.default_params(alpha=pb.alpha, gamma=pb.gamma, n=pb.n, M=pb.M, r=pb.r, precond=1)
    prob = fids.Problem(params, to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi))
    q, qhat = prob.precond_symbol(3)
    assert q[0] == 1.0 and not np.any(q[1:])
    assert np.all(qhat == 1.0)
    with pytest.raises(fids.FidsError):
        prob.precond_symbol(0)
    with pytest.raises(fids.FidsError):
        prob.precond_symbol(pb.M + 1)
    prob.close()
