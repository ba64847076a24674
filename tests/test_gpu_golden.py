"""Full-size parity: the GPU solution of the metric's seeded materials and source against the FP64
oracle's solution (oracle B: the fixed point of eqs. (iter1)-(iter2) with an exact inner solve by
sparse LU of M/tau + Khat and period sweeps), stored by tests/golden/make_oracle_solutions.py at
256^2 x 256 (config 2 sizes) and at 512^2 x 256 (the 2x-coarsened copy of config 3). Problem 1 has
a unique solution (Thm. thm:disc), so both sides, each stopped at a small residual, must agree:
relative L2 error at most 1e-8 on the stored slices (every node, or every second node in each
direction at 512^2) and on the norm of the whole field, in both precision modes."""
import json
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CASES = ["oracle_c2_seed0_n256_N256.npz", "oracle_c3half_seed0_n512_N256.npz"]


@pytest.fixture(scope="module")
def P():
    import paper_2502_21013_amd as P
    P.library()
    return P


@pytest.mark.parametrize("fname", CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_solution_matches_oracle(gpu, P, fname, precision):
    path = os.path.join(HERE, fname)
    if not os.path.exists(path):
        pytest.skip(f"{fname} has not been generated (tests/golden/make_oracle_solutions.py)")
    z = np.load(path)
    meta = json.loads(str(z["meta"]))
    pr = meta["problem"]
    say(f"golden {fname} {precision}")
    prob = W.with_size(W.config3(pr["seed"]), pr["n"], pr["N"])
    tol = min(1e-11, 10 * meta["tol"])
    U, st = P.Plan(prob, tol=tol, precision=precision, max_outer=4000).solve()
    assert st.rel_residual <= tol
    idx, s = [int(j) for j in z["slice_idx"]], int(z["stride"])
    ref = z["slices"]
    got = U[idx][:, ::s, ::s].cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    nrm = float(torch.sqrt((U * U).sum()))
    nref = float(np.sqrt(z["u_sq_sum"]))
    print(f"  outer {st.outer_iters}, rel_res {st.rel_residual:.2e}, rel L2 on slices {err:.2e}, "
          f"full-norm difference {abs(nrm - nref) / nref:.2e}", flush=True)
    assert err <= 1e-8
    assert abs(nrm - nref) <= 1e-8 * nref
