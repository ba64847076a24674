"""GPU solver behaviour: error statuses, determinism, exact resume, and the full-size workloads.

Full-size checks use properties that hold at any size, evaluated by the oracle on the GPU
result: the oracle's residual F - A(U) of the GPU solution (everywhere for the 256^2 x 256
workload; on sampled time slices for the 1024^2 x 512 one, where each slice's residual is
bounded by the total), half-wave antisymmetry of the sin-driven solution, and the discrete
energy balance over a period.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fem, periodic as pp
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2502_21013_amd as P
    P.library()
    return P


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


# ---------------------------------------------------------------- error statuses

def test_nonfinite_load_is_reported(gpu, P):
    say("error: nonfinite load")
    p = W.with_size(W.config1(), 8, 8)
    F = W.random_field(8, 8, 1)
    F[3, 4, 4] = np.nan
    plan = P.Plan(p, load=dev(F))
    U, st = plan.solve(raise_on_error=False)
    assert st.status == -6  # PT_ERR_NONFINITE


def test_max_outer_returns_last_iterate(gpu, P):
    say("error: max_outer")
    p = W.with_size(W.config1(), 16, 16)
    plan = P.Plan(p, max_outer=3)
    U, st = plan.solve(raise_on_error=False)
    assert st.status == -4 and st.outer_iters == 3
    assert len(st.history) == 4 and st.history[-1] < st.history[0]
    assert float(U.abs().max()) > 0


def test_too_small_nu_max_diverges(gpu, P):
    # Khat = nu_max S with nu_max below half the largest differential reluctivity violates
    # the contraction condition (A3) in the saturated iron, and the iteration diverges.
    say("error: divergence")
    import dataclasses
    p = dataclasses.replace(W.with_size(W.config1(), 16, 16), nu_max=2.0, J0=200.0)
    plan = P.Plan(p, max_outer=300, diverge_factor=10.0)
    U, st = plan.solve(raise_on_error=False)
    assert st.status == -7  # PT_ERR_DIVERGED


def test_undersized_workspace_is_rejected_before_launch(gpu, P):
    say("error: workspace")
    from paper_2502_21013_amd import _lib as L
    import ctypes as C
    plan = P.Plan(W.with_size(W.config1(), 8, 8))
    U = plan.new_time_field()
    ws, nb = plan.workspace()
    st = P.library().pt_solve(plan._h, ws, C.c_size_t(nb.value - 256), C.c_void_p(U.data_ptr()), None, None)
    assert st == L.PT_ERR_WORKSPACE


# ---------------------------------------------------------------- determinism and resume

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bitwise_deterministic(gpu, P, precision):
    say(f"determinism {precision}")
    p = W.with_size(W.config2(1), 64, 32)
    plan = P.Plan(p, tol=1e-10, precision=precision)
    U1, s1 = plan.solve()
    U2, s2 = plan.solve()
    assert s1.outer_iters == s2.outer_iters
    assert torch.equal(U1, U2)


def test_resume_continues_exactly(gpu, P):
    # the fixed-point map is memoryless: k1 steps, then k2 more from the stored iterate,
    # equal k1 + k2 steps in one call
    say("resume")
    p = W.with_size(W.config2(2), 32, 16)
    a = P.Plan(p, max_outer=20)
    Ua, _ = a.solve(raise_on_error=False)
    b = P.Plan(p, max_outer=7)
    Ub, sb = b.solve(raise_on_error=False)
    c = P.Plan(p, max_outer=13, use_initial_guess=True)
    Uc, sc = c.solve(Ub.clone(), raise_on_error=False)
    assert sb.outer_iters == 7 and sc.outer_iters == 13
    assert torch.equal(Ua, Uc)


def test_checking_every_few_steps_gives_the_same_iterates(gpu, P):
    say("check_every")
    p = W.with_size(W.config2(3), 32, 16)
    U1, s1 = P.Plan(p, tol=1e-9).solve()
    U4, s4 = P.Plan(p, tol=1e-9, check_every=4).solve()
    assert s4.outer_iters >= s1.outer_iters and s4.outer_iters - s1.outer_iters < 4
    assert s4.rel_residual <= 1e-9


def test_per_kernel_timer_counts_and_mask(gpu, P):
    # The event timer sees every launch of the fixed-point step: one residual sweep per step plus
    # the final one, one inverse per step, one restriction and one up sweep per step on the finest
    # level. With a class mask only those classes are bracketed, with the same counts, and the
    # iterates are bitwise those of an untimed solve.
    say("per-kernel timer")
    p = W.with_size(W.config2(3), 64, 16)
    U0, s0 = P.Plan(p, tol=1e-9).solve()
    Ua, sa = P.Plan(p, tol=1e-9, timing=True).solve()
    k = sa.outer_iters
    assert k == s0.outer_iters and torch.equal(Ua, U0)
    n = sa.kernel_launches
    assert n["residual_sweep"] == k + 1 and n["inverse_rfft_update"] == k
    assert n["vcycle_down_fine"] == k and n["vcycle_up_fine"] == k and n["matvec_dot"] == k
    assert all(v > 0 for v in sa.kernel_ms.values())
    Ub, sb = P.Plan(p, tol=1e-9, timing=("inverse_rfft_update", "residual_sweep")).solve()
    assert torch.equal(Ub, U0)
    assert set(sb.kernel_ms) == {"inverse_rfft_update", "residual_sweep"}
    assert sb.kernel_launches["residual_sweep"] == k + 1 and sb.kernel_launches["inverse_rfft_update"] == k
    with pytest.raises(ValueError):
        P.Plan(p, timing=("no_such_kernel",))


# ---------------------------------------------------------------- full-size workloads

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config2_full_size_against_oracle_residual(gpu, P, precision):
    say(f"config2 full size {precision}")
    p = W.config2(0)
    plan = P.Plan(p, tol=1e-8, precision=precision)
    U, st = plan.solve()
    assert st.rel_residual <= 1e-8
    Uh = U.cpu().numpy()
    del U
    d = fem.discretise(p)
    Uf = pp.to_free(d, Uh)
    F = pp.load_series(d)
    R = pp.residual(d, Uf, F)
    rel = np.linalg.norm(R) / np.linalg.norm(F)
    assert rel <= 1e-8 * 1.001
    assert abs(rel - st.rel_residual) <= 1e-3 * st.rel_residual
    N = p.N
    # half-wave antisymmetry holds to the solver tolerance
    assert np.linalg.norm(Uf[N // 2:] + Uf[: N // 2]) <= 1e-6 * np.linalg.norm(Uf)
    # energy balance tau sum ||d u||_M^2 = 2 sum <f - K(u), u> up to the residual
    dU = (Uf - np.roll(Uf, 1, axis=0)) / p.tau
    lhs = p.tau * np.sum(dU * (d.M @ dU.T).T)
    rhs = 2 * np.sum((F - pp.K_free(d, Uf)) * Uf)
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_config3_full_size_sampled_slices(gpu, P, precision):
    say(f"config3 full size {precision}")
    p = W.config3(0)
    plan = P.Plan(p, tol=1e-8, precision=precision)
    U, st = plan.solve()
    assert st.rel_residual <= 1e-8
    d = fem.discretise(p)
    Fnorm = np.linalg.norm(d.b) * np.sqrt(np.sum(np.sin(2 * np.pi * np.arange(1, p.N + 1) / p.N) ** 2))
    assert abs(Fnorm - st.f_norm) <= 1e-10 * Fnorm
    Mt = (d.M / p.tau).tocsr()
    for n in (0, 137, 300, 511):
        un = pp.to_free(d, U[n:n + 1].cpu().numpy())[0]
        um = pp.to_free(d, U[(n - 1) % p.N:(n - 1) % p.N + 1].cpu().numpy())[0]
        fn = np.sin(2 * np.pi * (n + 1) / p.N) * d.b
        Rn = fn - Mt @ (un - um) - pp.K_free(d, un[None])[0]
        assert np.linalg.norm(Rn) <= 1e-8 * Fnorm
    del U
    plan.close()
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- the paper's initialisation

def test_static_start_reaches_the_same_solution(gpu, P):
    # the static start (sigma = 0 problems) then the periodic iteration converge to the
    # oracle's periodic solution; the start itself is the oracle's sigma = 0 solution
    import dataclasses
    say("static start")
    p = W.with_size(W.config2(7), 16, 16)
    d = fem.discretise(p)
    ref = pp.fixed_point(d, tol=1e-12, max_iter=3000)
    plan = P.Plan(p, tol=1e-12, max_outer=3000, init_static=True, init_tol=1e-12)
    U, st = plan.solve()
    assert st.init_iters > 10 and st.rel_residual <= 1e-12
    assert 0 < st.rel_initial < 1
    assert np.linalg.norm(U.cpu().numpy() - pp.to_full(d, ref.U)) <= 1e-8 * np.linalg.norm(pp.to_full(d, ref.U))
    # the start: static solution = periodic solution of the sigma = 0 problem
    p0 = dataclasses.replace(p, sigma_in=0.0)
    d0 = fem.discretise(p0)
    U0 = pp.fixed_point(d0, tol=1e-13, max_iter=3000).U
    Fs = pp.load_series(d)
    R0 = pp.residual(d, U0, Fs)
    assert abs(np.linalg.norm(R0) / np.linalg.norm(Fs) - st.rel_initial) <= 1e-6 * st.rel_initial


def test_static_start_is_exact_without_conductivity(gpu, P):
    import dataclasses
    say("static start sigma 0")
    p = dataclasses.replace(W.with_size(W.config2(8), 16, 16), sigma_in=0.0)
    U, st = P.Plan(p, tol=1e-10, init_static=True, init_tol=1e-11).solve()
    assert st.outer_iters == 0 and st.init_iters > 10 and st.rel_residual <= 1e-10


def test_relative_to_initial_residual_matches_from_zero(gpu, P):
    # from U^0 = 0 the paper's denominator ||F - A(U^0)|| is ||F||
    say("stop relative to the initial residual")
    p = W.with_size(W.config2(9), 16, 16)
    U1, s1 = P.Plan(p, tol=1e-9).solve()
    U2, s2 = P.Plan(p, tol=1e-9, stop_relative_initial=True).solve()
    assert s1.outer_iters == s2.outer_iters and torch.equal(U1, U2)
    assert s2.rel_initial == pytest.approx(1.0)
    # after a static start the rule divides by the start's residual: more steps to the same tol
    U3, s3 = P.Plan(p, tol=1e-9, init_static=True, stop_relative_initial=True).solve()
    assert s3.rel_residual <= 1e-9 and s3.rel_residual * s3.rel_initial <= 1e-9
