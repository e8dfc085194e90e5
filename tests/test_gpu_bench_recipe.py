"""GPU forms of the benchmark recipe against the oracle at n = 4095.

The benchmark workload (alpha 1.5, gamma 0.4, r 4, M = 2048, seeded kappa
and f) is solved at n = 4095, where the oracle's u^M is stored in
tests/golden/c2_recipe_n4095_M2048_uT.txt (written by
make_c2_recipe_reference.py, oracle only).  Every solver form must match it to
the FP64 gate (1e-8 relative max norm) or the mixed-precision gate (1e-7).
"""
import os

import numpy as np
import pytest

from paper_2002_11978_amd import fids
from paper_2002_11978_amd import workloads as W

from gpu_util import rel_maxnorm, say, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_recipe_n4095_M2048_uT.txt")

FORMS = [
    pytest.param(dict(solver=2, precision=0, x0_mode=3), 1e-8, id="headline-pcg-fp64-x0cubic"),
    pytest.param(dict(solver=1, precision=0, x0_mode=3), 1e-8, id="fgmres-fp64-x0cubic"),
    pytest.param(dict(solver=0, precision=0, x0_mode=0), 1e-8, id="plain-bicgstab-fp64"),
    pytest.param(dict(solver=1, precision=1, x0_mode=3), 1e-7, id="mixed-fgmres-fp32pc-x0cubic"),
    pytest.param(dict(solver=1, precision=0, x0_mode=3, precond=2), 1e-8, id="fgmres-fp64-kpc"),
]


@pytest.fixture(scope="module")
def recipe():
    if not os.path.exists(GOLDEN):
        pytest.skip("golden file missing: run tests/golden/make_c2_recipe_reference.py")
    ref = np.loadtxt(GOLDEN)
    pb = W.seeded(1.5, 0.4, 4095, 2048, r=4.0, kappa_seed=3, f_seed=4)
    return pb, ref


@pytest.mark.parametrize("kw,gate", FORMS)
def test_bench_recipe_form_matches_oracle(recipe, kw, gate):
    pb, ref = recipe
    p = fids.default_params(alpha=pb.alpha, gamma=pb.gamma, n=pb.n, M=pb.M, r=pb.r, soe_tol=1e-10,
                            krylov_tol=1e-10, krylov_maxit=500, **kw)
    prob = fids.Problem(p, to_dev(pb.kappa), to_dev(pb.f), to_dev(pb.phi))
    uT, _, reps = prob.solve_all()
    err = rel_maxnorm(uT.cpu().numpy(), ref)
    say(f"  {kw}: rel err vs oracle {err:.3e}, its {np.mean([r.iters for r in reps]):.2f}")
    prob.close()
    assert err <= gate
