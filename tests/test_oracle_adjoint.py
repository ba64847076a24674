"""Pins of the oracle's loss and adjoint gradient (oracle/adjoint.py).

Each pin is independent of the formula it checks:
* the loss against a different quadrature of int sigma |d_tau u|^2 (edge midpoints, exact
  for the quadratic integrand on each triangle);
* dl/dU and the Jacobian J = dA/dU against central differences of l and of A;
* the adjoint gradients dl/dtheta_T and dl/dsigma_T against central differences of the
  loss of re-solved problems (Newton to 1e-14 on the perturbed problem);
* special cases: no conductivity (no loss, no gradient), and the scaling law of a linear
  material (theta -> c theta, sigma -> c sigma, J0 -> c J0 leaves U unchanged and scales l
  by c, so Euler's relation sum theta dl/dtheta + sum sigma dl/dsigma + J0 dl/dJ0 = l
  holds, with the J0-derivative by differences).
"""
import dataclasses

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import adjoint as AD
from oracle import fem, periodic as pp


def discretise_with(p, sigma_tri=None):
    """Discretisation of p with an optional per-triangle conductivity replacing sigma_rect."""
    d = fem.discretise(p)
    if sigma_tri is None:
        return d
    mat = dataclasses.replace(d.mat, sigma=np.asarray(sigma_tri, dtype=np.float64))
    M = fem.restrict(fem.mass_full(d.mesh, mat.sigma), d.mesh.free)
    return dataclasses.replace(d, mat=mat, M=M)


def solve(d):
    U, hist = pp.newton(d, tol=1e-14)
    R = pp.residual(d, U, pp.load_series(d))
    assert np.linalg.norm(R) <= 1e-13 * np.linalg.norm(pp.load_series(d))
    return U


@pytest.fixture(scope="module")
def small():
    # 8 x 8 cells, N = 8, strong source so that the iron saturates; seeded theta
    rng = np.random.default_rng(5)
    theta = np.repeat(np.exp(rng.normal(0.0, 0.1, 64)), 2)
    p = dataclasses.replace(W.with_size(W.config1(), 8, 8), J0=60.0, theta=theta)
    d = discretise_with(p)
    U = solve(d)
    return p, d, U


def test_loss_equals_edge_midpoint_quadrature(small):
    p, d, U = small
    m = d.mesh
    Uf = pp.to_full(d, U).reshape(p.N, -1)
    dU = (Uf - np.roll(Uf, 1, axis=0)) / p.tau
    v = dU[:, m.tri]                                    # (N, ntri, 3)
    mids = 0.5 * (v + np.roll(v, -1, axis=2))           # values at the three edge midpoints
    quad = np.sum(m.area / 3.0 * d.mat.sigma * np.sum(mids ** 2, axis=2), axis=1)
    ref = p.tau * np.sum(quad)
    assert AD.loss(d, U) == pytest.approx(ref, rel=1e-13)
    assert ref > 0


def test_loss_gradient_in_U_by_differences(small):
    p, d, U = small
    g = AD.loss_grad_U(d, U)
    rng = np.random.default_rng(1)
    for _ in range(3):
        Wd = rng.standard_normal(U.shape)
        eps = 1e-4
        fd = (AD.loss(d, U + eps * Wd) - AD.loss(d, U - eps * Wd)) / (2 * eps)
        assert np.sum(g * Wd) == pytest.approx(fd, rel=1e-9)


def test_jacobian_by_differences(small):
    p, d, U = small
    J = AD.jacobian_A(d, U)
    rng = np.random.default_rng(2)
    Wd = rng.standard_normal(U.shape) * np.abs(U).max()
    eps = 1e-6
    fd = (pp.apply_A(d, U + eps * Wd) - pp.apply_A(d, U - eps * Wd)) / (2 * eps)
    Jw = (J @ Wd.reshape(-1)).reshape(U.shape)
    assert np.linalg.norm(Jw - fd) <= 1e-7 * np.linalg.norm(fd)
    # the diagonal blocks are symmetric; J itself is not (the time coupling is one-sided)
    N, nf = U.shape
    blk = J[:nf, :nf]
    assert abs(blk - blk.T).max() <= 1e-12 * abs(blk).max()
    Mt = d.M / p.tau
    assert abs(J - J.T).max() == pytest.approx(abs(Mt).max(), rel=1e-12)


def test_adjoint_state_solves_the_transposed_system(small):
    p, d, U = small
    lam = AD.adjoint_state(d, U)
    J = AD.jacobian_A(d, U)
    g = AD.loss_grad_U(d, U)
    rng = np.random.default_rng(3)
    Wd = rng.standard_normal(U.shape)
    lhs = np.dot((J @ Wd.reshape(-1)), lam.reshape(-1))
    assert lhs == pytest.approx(np.sum(Wd * g), rel=1e-10)


def _cells_to_probe(d, count, rng, where):
    cand = np.flatnonzero(where)
    return rng.choice(cand, size=min(count, cand.size), replace=False)


def test_theta_gradient_matches_central_differences(small):
    p, d, U = small
    G = AD.gradients(d, U)
    rng = np.random.default_rng(4)
    tris = list(_cells_to_probe(d, 4, rng, d.mat.iron)) + list(_cells_to_probe(d, 2, rng, ~d.mat.iron))
    for t in tris:
        h = 1e-5 * p.theta[t]
        vals = []
        for sgn in (1, -1):
            th = np.array(p.theta)
            th[t] += sgn * h
            dp = discretise_with(dataclasses.replace(p, theta=th))
            vals.append(AD.loss(dp, solve(dp)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert G.theta[t] == pytest.approx(fd, rel=1e-6, abs=1e-9 * abs(G.loss)), t


def test_sigma_gradient_matches_central_differences(small):
    p, d, U = small
    G = AD.gradients(d, U)
    rng = np.random.default_rng(6)
    cond = d.mat.sigma > 0
    tris = list(_cells_to_probe(d, 4, rng, cond)) + list(_cells_to_probe(d, 2, rng, ~cond))
    for t in tris:
        h = 1e-5
        vals = []
        for sgn in (1, -1):
            s = d.mat.sigma.copy()
            s[t] += sgn * h
            dp = discretise_with(p, s)
            vals.append(AD.loss(dp, solve(dp)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert G.sigma[t] == pytest.approx(fd, rel=1e-6, abs=1e-9 * abs(G.loss)), t


def test_no_conductivity_no_loss_no_gradient():
    p = dataclasses.replace(W.with_size(W.config1(), 8, 8), sigma_in=0.0)
    d = discretise_with(p)
    U = solve(d)
    G = AD.gradients(d, U)
    assert G.loss == 0.0
    assert np.abs(G.theta).max() == 0.0 and np.abs(G.lam).max() == 0.0


def test_linear_material_scaling_relation():
    # nu_b = 0: K(u) = theta nu S_theta u is linear. Scaling theta, sigma and J0 by c scales
    # U by 1 and the loss by c (l = tau sum du^T M du, M ~ sigma), so by Euler's relation
    #   sum_T theta_T dl/dtheta_T + sum_T sigma_T dl/dsigma_T + J0 dl/dJ0 = l.
    rng = np.random.default_rng(8)
    theta = np.repeat(np.exp(rng.normal(0.0, 0.2, 64)), 2)
    p = dataclasses.replace(W.with_size(W.config1(), 8, 8), nu_b=0.0, theta=theta, J0=3.0)
    d = discretise_with(p)
    U = solve(d)
    G = AD.gradients(d, U)
    h = 1e-5 * p.J0
    lp = AD.loss(discretise_with(dataclasses.replace(p, J0=p.J0 + h)),
                 solve(discretise_with(dataclasses.replace(p, J0=p.J0 + h))))
    lm = AD.loss(discretise_with(dataclasses.replace(p, J0=p.J0 - h)),
                 solve(discretise_with(dataclasses.replace(p, J0=p.J0 - h))))
    dJ = (lp - lm) / (2 * h)
    euler = np.sum(p.theta * G.theta) + np.sum(d.mat.sigma * G.sigma) + p.J0 * dJ
    assert euler == pytest.approx(G.loss, rel=1e-7)
    # and the loss is quadratic in J0 for a linear material: J0 dl/dJ0 = 2 l
    assert p.J0 * dJ == pytest.approx(2 * G.loss, rel=1e-7)


def test_per_cell_sums_pairs():
    g = np.arange(8.0)
    assert np.array_equal(AD.per_cell(g), np.array([1.0, 5.0, 9.0, 13.0]))
