"""GPU adjoint: the adjoint state, the loss and its parameter gradients against the FP64
oracle (oracle/adjoint.py: sparse LU of the assembled transposed Jacobian), the autograd
function, and central finite differences of the GPU loss at the full 256^2 x 256 size.

Tolerances: with the forward and adjoint iterations both stopped at a relative residual of
1e-12, the adjoint state and the gradients carry an error of about cond(J) x 1e-12; the
bound used is a relative L2 error of 1e-8, as for the forward solution. Finite differences
at full size use a fixed number of outer steps (400: the residual sits at its FP64
rounding floor of about 3e-13) so that the perturbed solves are smooth functions of the
parameter, and a step of 1e-3 relative (truncation error about 1e-7); they are held to
1e-5 relative.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import adjoint as AD
from oracle import fem, periodic as pp
from tests.gpu_helpers import say, rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2502_21013_amd as P
    P.library()
    return P


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def small_problem(n, N, seed, J0=40.0):
    rng = np.random.default_rng(seed)
    theta = np.repeat(np.exp(rng.normal(0.0, 0.1, n * n)), 2)
    return dataclasses.replace(W.with_size(W.config1(), n, N), J0=J0, theta=theta)


@pytest.fixture(scope="module")
def small_case():
    p = small_problem(16, 16, 3)
    d = fem.discretise(p)
    U = pp.fixed_point(d, tol=1e-13, max_iter=3000).U
    G = AD.gradients(d, U)
    return p, d, U, G


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_adjoint_state_and_gradients_match_oracle(gpu, P, small_case, precision):
    say(f"adjoint parity {precision}")
    p, d, Uo, G = small_case
    plan = P.Plan(p, theta=dev(p.theta), tol=1e-12, max_outer=3000, precision=precision, adjoint=True)
    U, st = plan.solve()
    assert rel_err(U.cpu().numpy(), pp.to_full(d, Uo)) <= 1e-8
    Lam, ast = plan.adjoint_solve(U)
    assert ast.rel_residual <= 1e-12 and ast.outer_iters > 10
    assert rel_err(Lam.cpu().numpy(), pp.to_full(d, G.lam)) <= 1e-8
    loss, gt, gs = plan.loss_gradients(U, Lam)
    assert loss == pytest.approx(G.loss, rel=1e-9)
    assert rel_err(gt.cpu().numpy(), G.theta) <= 1e-8
    assert rel_err(gs.cpu().numpy(), G.sigma) <= 1e-8
    # per-cell sums
    _, gtc, gsc = plan.loss_gradients(U, Lam, per_cell=True)
    assert rel_err(gtc.cpu().numpy(), AD.per_cell(G.theta)) <= 1e-8
    assert rel_err(gsc.cpu().numpy(), AD.per_cell(G.sigma)) <= 1e-8
    plan.close()


def test_loss_without_adjoint_state(gpu, P, small_case):
    say("loss only")
    p, d, Uo, G = small_case
    plan = P.Plan(p, theta=dev(p.theta), adjoint=True)
    U = dev(pp.to_full(d, Uo))
    loss, gt, gs = plan.loss_gradients(U, None)
    assert loss == pytest.approx(G.loss, rel=1e-12)
    assert float(gt.abs().max()) == 0.0
    # without lambda the sigma entry is the direct part tau sum du^T M_T du = loss_T / sigma_T
    lam0 = AD.gradients(d, Uo, lam=np.zeros_like(Uo))
    assert rel_err(gs.cpu().numpy(), lam0.sigma) <= 1e-12


def test_adjoint_graph_replay_is_identical(gpu, P, small_case):
    say("adjoint graph")
    p, d, Uo, G = small_case
    U = dev(pp.to_full(d, Uo))
    L1, s1 = P.Plan(p, theta=dev(p.theta), tol=1e-11, adjoint=True, check_every=4).adjoint_solve(U)
    L2, s2 = P.Plan(p, theta=dev(p.theta), tol=1e-11, adjoint=True, check_every=4, graph=True).adjoint_solve(U)
    assert s1.outer_iters == s2.outer_iters and torch.equal(L1, L2)


def test_autograd_function_matches_oracle(gpu, P):
    say("autograd")
    from paper_2502_21013_amd.adjoint import eddy_loss
    n, N = 16, 16
    p = small_problem(n, N, 9)
    d = fem.discretise(p)
    # per-cell sigma: sigma_in on the conducting block (whose edges lie on grid lines)
    sig_tri = d.mat.sigma
    assert np.array_equal(sig_tri[0::2], sig_tri[1::2])
    theta_c = torch.tensor(p.theta[0::2], dtype=torch.float64, device="cuda:0", requires_grad=True)
    sigma_c = torch.tensor(sig_tri[0::2], dtype=torch.float64, device="cuda:0", requires_grad=True)
    loss = eddy_loss(p, theta_c, sigma_c, tol=1e-12, max_outer=3000)
    loss.backward()
    G = AD.gradients(d, pp.fixed_point(d, tol=1e-13, max_iter=3000).U)
    assert float(loss.detach()) == pytest.approx(G.loss, rel=1e-9)
    assert rel_err(theta_c.grad.cpu().numpy(), AD.per_cell(G.theta)) <= 1e-8
    assert rel_err(sigma_c.grad.cpu().numpy(), AD.per_cell(G.sigma)) <= 1e-8


def test_adjoint_requires_an_adjoint_plan(gpu, P):
    plan = P.Plan(W.with_size(W.config1(), 8, 8))
    with pytest.raises(P.PTError):
        plan.adjoint_solve(plan.new_time_field())


# ---------------------------------------------------------------- full size, finite differences

def test_config5_gradients_match_central_differences(gpu, P):
    say("config5 finite differences")
    p = W.config5(0)
    n = p.n
    theta_c = np.asarray(p.theta[0::2])
    d_sig = fem.materials(p, fem.build_mesh(n)).sigma   # sigma_in on the block, 0 elsewhere
    sigma_c = d_sig[0::2].copy()
    base = dataclasses.replace(p, theta=None)

    def plan_for(th_c, sg_c, **kw):
        return P.Plan(base, theta=dev(np.repeat(th_c, 2)), sigma=dev(np.repeat(sg_c, 2)), adjoint=True, **kw)

    # the adjoint source is a second difference in time of U, so its relative residual has a
    # higher FP64 floor than the forward one (about 1e-12 at this size)
    plan = plan_for(theta_c, sigma_c, tol=3e-12, max_outer=3000)
    U, st = plan.solve()
    Lam, ast = plan.adjoint_solve(U)
    assert ast.rel_residual <= 3e-12
    loss0, gt, gs = plan.loss_gradients(U, Lam, per_cell=True)
    gt, gs = gt.cpu().numpy(), gs.cpu().numpy()
    plan.close()
    del U, Lam
    rng = np.random.default_rng(2025)
    # 16 seeded cells for theta among those in the iron block, 8 on the conducting block for sigma
    iron_c = np.flatnonzero(fem.materials(p, fem.build_mesh(n)).iron[0::2])
    cond_c = np.flatnonzero(sigma_c > 0)
    cells_t = rng.choice(iron_c, 16, replace=False)
    cells_s = rng.choice(cond_c, 8, replace=False)

    def loss_of(th_c, sg_c):
        pl = plan_for(th_c, sg_c, tol=1e-300, max_outer=400)
        Ux, sx = pl.solve(raise_on_error=False)
        assert sx.outer_iters == 400 and sx.rel_residual < 1e-12   # at the FP64 rounding floor
        lx, _, _ = pl.loss_gradients(Ux, None)
        pl.close()
        return lx

    worst = 0.0
    for c in cells_t:
        h = 1e-3 * theta_c[c]
        tp, tm = theta_c.copy(), theta_c.copy()
        tp[c] += h
        tm[c] -= h
        fd = (loss_of(tp, sigma_c) - loss_of(tm, sigma_c)) / (2 * h)
        err = abs(fd - gt[c]) / abs(gt[c])
        worst = max(worst, err)
        say(f"theta cell {c}: adjoint {gt[c]:.9e} fd {fd:.9e} rel {err:.2e}")
        assert err <= 1e-5
    for c in cells_s:
        h = 1e-3 * sigma_c[c]
        sp_, sm = sigma_c.copy(), sigma_c.copy()
        sp_[c] += h
        sm[c] -= h
        fd = (loss_of(theta_c, sp_) - loss_of(theta_c, sm)) / (2 * h)
        err = abs(fd - gs[c]) / abs(gs[c])
        worst = max(worst, err)
        say(f"sigma cell {c}: adjoint {gs[c]:.9e} fd {fd:.9e} rel {err:.2e}")
        assert err <= 1e-5
    say(f"worst relative difference {worst:.2e}; loss {loss0:.9e}")
