"""pt_solve_noalloc (the solve with the library's static device scratch as workspace) against
pt_solve with a caller-owned workspace: the same kernels on the same data, so the same iterates.
Two calls in a row on one GPU, the second on a smaller problem (the scratch keeps the first
call's contents, which the second must not depend on)."""
import numpy as np
import pytest

import workloads as W


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_solve_matches_workspace_solve(gpu, precision):
    import torch
    import paper_2502_21013_amd as P
    sizes = [(64, 64), (32, 32)]  # second call smaller than the first
    for n, N in sizes:
        prob = W.with_size(W.config2(1), n, N)
        print(f"noalloc case: {precision} n={n} N={N}", flush=True)
        plan = P.Plan(prob, tol=1e-10, precision=precision, max_outer=2000)
        U_ref, st_ref = plan.solve()
        U_na, st_na = plan.solve_noalloc()
        torch.cuda.synchronize()
        a, b = U_ref.cpu().numpy(), U_na.cpu().numpy()
        err = np.linalg.norm(a - b) / np.linalg.norm(a)
        print(f"  outer {st_ref.outer_iters}/{st_na.outer_iters} rel_res {st_na.rel_residual:.3e} "
              f"rel_L2 {err:.3e}", flush=True)
        assert st_na.status == 0 and st_na.rel_residual <= 1e-10
        assert st_na.outer_iters == st_ref.outer_iters
        assert err <= 1e-12
        # zero boundary, as every solve writes it
        assert np.all(b[:, 0, :] == 0) and np.all(b[:, -1, :] == 0)
        plan.close()


@pytest.mark.gpu
def test_noalloc_batch_solve_matches_batch_solve(gpu):
    import torch
    import paper_2502_21013_amd as P
    probs = [W.with_size(W.config2(s), 32, 32) for s in range(4)]
    print("noalloc batch case: 4 x 32^2 x 32 fp64", flush=True)
    plan = P.BatchPlan(probs, tol=1e-10, precision="fp64", max_outer=2000)
    U_ref, st_ref = plan.solve()
    U_na, st_na = plan.solve_noalloc()
    torch.cuda.synchronize()
    a, b = U_ref.cpu().numpy(), U_na.cpu().numpy()
    assert [s.outer_iters for s in st_na] == [s.outer_iters for s in st_ref]
    assert np.linalg.norm(a - b) / np.linalg.norm(a) <= 1e-12
    plan.close()
