"""COCG inner solve (remark rem:parallel: one complex-shifted system per frequency) with the
per-frequency stopping test ||r_k|| <= inner_rtol ||R_k||, masking of stopped frequencies, and
the breakdown error path, against the FP64 oracle on seeded inputs."""
import numpy as np
import pytest

import workloads as W
from oracle import fem, periodic as pp
from tests.gpu_helpers import rel_err, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2502_21013_amd as P
    P.library()
    return P


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_periodic_solve_stops_per_frequency(gpu, P, precision):
    """A tight per-frequency tolerance within a generous step budget gives the exact periodic
    solve (space-time LU of the oracle) without using the whole budget."""
    n, N = 32, 16
    say(f"cocg rtol periodic solve {precision}")
    p = W.with_size(W.config2(3), n, N)
    d = fem.discretise(p)
    R = W.random_field(N, n, 5, 1.0)
    ref = pp.to_full(d, pp.SpaceTimeLU(d).solve(pp.to_free(d, R)))
    eta = 1e-11 if precision == "fp64" else 1e-6
    plan = P.Plan(p, precision=precision, inner="cocg", inner_iters=64, inner_rtol=eta)
    X = plan.periodic_solve(dev(R)).cpu().numpy()
    assert rel_err(X, ref) <= (1e-9 if precision == "fp64" else 2e-5)


def test_solve_with_inner_tolerance_matches_oracle(gpu, P):
    """Outer solve with COCG to inner_rtol 1e-2 (at most 32 steps): the same solution as the
    oracle's exact inner solves, with fewer inner steps than the budget."""
    say("cocg rtol full solve config1")
    d = fem.discretise(W.config1())
    ref = pp.fixed_point(d, tol=1e-12, max_iter=2000)
    plan = P.Plan(W.config1(), tol=1e-12, inner="cocg", inner_iters=32, inner_rtol=1e-2, max_outer=2000)
    U, st = plan.solve()
    assert st.rel_residual <= 1e-12
    assert rel_err(U.cpu().numpy(), pp.to_full(d, ref.U)) <= 1e-8
    assert 1 < st.inner_iters_max < 32
    assert st.outer_iters <= st.inner_iters_sum <= st.outer_iters * st.inner_iters_max
    # a looser inner tolerance takes fewer inner steps per outer step, never more
    _, st2 = P.Plan(W.config1(), tol=1e-12, inner="cocg", inner_iters=32, inner_rtol=0.3, max_outer=4000).solve()
    assert st2.inner_iters_sum / st2.outer_iters < st.inner_iters_sum / st.outer_iters


def test_zero_right_hand_side_frequencies_are_masked(gpu, P):
    """A right-hand side constant in time: its DFT is exactly zero at every frequency but k = 0,
    so all of them (and the k = N/2 half of the packed slot 0) are masked from the start (no
    breakdown) and the solution is the static one, L X = R, on every slice."""
    n, N = 16, 16
    say("cocg zero-rhs frequencies")
    p = W.with_size(W.config2(2), n, N)
    d = fem.discretise(p)
    rng = np.random.default_rng(7)
    shape = np.zeros((n + 1, n + 1))
    shape[1:-1, 1:-1] = rng.standard_normal((n - 1, n - 1))
    R = np.repeat(shape[None], N, axis=0)
    plan = P.Plan(p, inner="cocg", inner_iters=40, inner_rtol=1e-12)
    X = plan.periodic_solve(dev(R)).cpu().numpy()
    ref = pp.to_full(d, pp.SpaceTimeLU(d).solve(pp.to_free(d, R)))
    assert rel_err(X, ref) <= 1e-9
    assert np.abs(X - X[:1]).max() <= 1e-12 * np.abs(X).max()


def test_breakdown_is_reported_without_fault(gpu, P):
    """The breakdown test forced from the host (breakdown_tol far above any |p^T A p| /
    Re(p^H A p)): the solve returns PT_ERR_BREAKDOWN after its first outer step, every kernel
    having finished normally, with a finite iterate and filled stats."""
    say("cocg forced breakdown")
    plan = P.Plan(W.with_size(W.config1(), 16, 16), inner="cocg", inner_iters=4, breakdown_tol=1e30)
    U, st = plan.solve(raise_on_error=False)
    assert st.status == -5
    assert st.outer_iters == 1
    assert "breakdown" in P.library().pt_last_error().decode().lower()
    assert torch.isfinite(U).all()
    # the same plan without the forced threshold converges
    ok = P.Plan(W.with_size(W.config1(), 16, 16), inner="cocg", inner_iters=4, tol=1e-10)
    _, st2 = ok.solve()
    assert st2.status == 0


def test_graph_replay_with_inner_tolerance_gives_identical_iterates(gpu, P):
    """Eager launches stop the inner loop once every frequency is masked; graph replay runs the
    whole step budget with the masked frequencies unchanged: the same iterates bit for bit."""
    say("cocg rtol graph replay")
    p = W.with_size(W.config2(5), 32, 16)
    mk = lambda **kw: P.Plan(p, tol=1e-10, check_every=3, inner="cocg", inner_iters=12, inner_rtol=1e-3, **kw)
    Ue, se = mk().solve()
    Ug, sg = mk(graph=True).solve()
    assert se.outer_iters == sg.outer_iters
    assert torch.equal(Ue, Ug)
    assert se.inner_iters_sum < sg.inner_iters_sum == 12 * sg.outer_iters
