"""Cycle-averaged eddy-current loss and its gradient by the adjoint method (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Loss. The Joule loss of one period, int_0^T int_Omega sigma |du/dt|^2, discretised with the
implicit-Euler difference quotient d u^n = (u^n - u^{n-1}) / tau (u^0 = u^N) and the
consistent sigma-mass:
    l(U) = tau sum_n (d u^n)^T M (d u^n).

Parameters. theta_T (the nu scale of triangle T; nu_T = theta_T nuhat_T) and sigma_T (the
conductivity of T, M = sum_T sigma_T M_T with the unit-conductivity element mass
M_T = |T|/12 [[2,1,1],[1,2,1],[1,1,2]]).

Gradient. U(theta, sigma) is defined by A(U) = F (Problem 1, eqs. (disc1)-(disc2)). With
J = dA/dU and the adjoint state lambda solving J^T lambda = dl/dU,
    dl/dp = (partial l / partial p) - lambda^T (partial A / partial p).
J has the diagonal blocks M/tau + K'(u^n) and the cyclic sub-diagonal blocks -M/tau;
K'(u) is symmetric (K is the gradient of an energy), so J^T has the same diagonal blocks
and the cyclic super-diagonal -M/tau: the adjoint equation
    (M/tau) (lambda^n - lambda^{n+1}) + K'(u^n) lambda^n = (dl/dU)^n,  lambda^{N+1} = lambda^1,
runs backward in time and is again periodic. Here it is solved directly by a sparse LU of
the assembled J^T.

Per-triangle partial derivatives (U, lambda fixed; sums over n = 1..N):
    dl/dU^n             = (2/tau) M (2 u^n - u^{n-1} - u^{n+1})
    lambda^T dA/dtheta_T = sum_n |T| nuhat_T(|grad u^n_T|^2) grad u^n_T . grad lambda^n_T
    partial l/dsigma_T   = tau sum_n (d u^n)^T M_T (d u^n)
    lambda^T dA/dsigma_T = sum_n (lambda^n)^T M_T (d u^n)
F does not depend on theta or sigma.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem
from .periodic import cyclic_shift


def loss(d: fem.Discretisation, Uf: np.ndarray) -> float:
    """l(U) = tau sum_n (d u^n)^T M (d u^n), U on the free nodes (N, nfree)."""
    dU = (Uf - np.roll(Uf, 1, axis=0)) / d.p.tau
    return float(d.p.tau * np.sum(dU * (d.M @ dU.T).T))


def loss_grad_U(d: fem.Discretisation, Uf: np.ndarray) -> np.ndarray:
    """dl/dU^n = (2/tau) M (2 u^n - u^{n-1} - u^{n+1}) (cyclic in n)."""
    D2 = 2.0 * Uf - np.roll(Uf, 1, axis=0) - np.roll(Uf, -1, axis=0)
    return (2.0 / d.p.tau) * (d.M @ D2.T).T


def _full(d: fem.Discretisation, v: np.ndarray) -> np.ndarray:
    out = np.zeros(v.shape[:-1] + (d.mesh.nodes,))
    out[..., d.free_idx] = v
    return out


def jacobian_A(d: fem.Discretisation, Uf: np.ndarray) -> sp.csc_matrix:
    """J = dA/dU: blocks M/tau + K'(u^n) on the diagonal, -M/tau at (n, n-1) cyclically."""
    p = d.p
    N = p.N
    Mt = (d.M / p.tau).tocsr()
    blocks = [fem.restrict(fem.jacobian_K(p, d.mesh, d.mat, _full(d, Uf[j])), d.mesh.free) for j in range(N)]
    J = sp.kron(sp.identity(N), Mt) - sp.kron(cyclic_shift(N), Mt) + sp.block_diag(blocks)
    return J.tocsc()


def adjoint_state(d: fem.Discretisation, Uf: np.ndarray) -> np.ndarray:
    """lambda with J^T lambda = dl/dU, by sparse LU of the assembled J^T."""
    J = jacobian_A(d, Uf)
    g = loss_grad_U(d, Uf)
    lam = spla.spsolve(J.T.tocsc(), g.reshape(-1))
    return lam.reshape(Uf.shape)


@dataclass
class Gradients:
    loss: float
    theta: np.ndarray   # (ntri,) dl/dtheta_T
    sigma: np.ndarray   # (ntri,) dl/dsigma_T
    lam: np.ndarray     # (N, nfree) adjoint state


def element_mass_form(m: fem.Mesh, V: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Per triangle and summed over the leading axis: V_T^T M_T W_T with the unit-conductivity
    element mass, i.e. |T|/12 (sum_a v_a w_a + (sum_a v_a)(sum_a w_a)). V, W: (..., nodes)."""
    v = V[..., m.tri]
    w = W[..., m.tri]
    s = np.einsum("...ta,...ta->...t", v, w) + v.sum(-1) * w.sum(-1)
    s = s.reshape(-1, m.tri.shape[0]).sum(0)
    return m.area / 12.0 * s


def gradients(d: fem.Discretisation, Uf: np.ndarray, lam: np.ndarray | None = None) -> Gradients:
    """dl/dtheta_T and dl/dsigma_T for every triangle, at the solution U of A(U) = F."""
    p, m, mat = d.p, d.mesh, d.mat
    if lam is None:
        lam = adjoint_state(d, Uf)
    Ufull = _full(d, Uf)
    Lfull = _full(d, lam)
    gu = fem.gradients(m, Ufull)             # (N, ntri, 2)
    gl = fem.gradients(m, Lfull)
    s2 = np.einsum("ntd,ntd->nt", gu, gu)
    nuhat = fem.nu_of_s2(s2, mat, p) / mat.theta
    g_theta = -np.sum(m.area * nuhat * np.einsum("ntd,ntd->nt", gu, gl), axis=0)
    dU = (Ufull - np.roll(Ufull, 1, axis=0)) / p.tau
    g_sigma = p.tau * element_mass_form(m, dU, dU) - element_mass_form(m, Lfull, dU)
    return Gradients(loss=loss(d, Uf), theta=g_theta, sigma=g_sigma, lam=lam)


def per_cell(g_tri: np.ndarray) -> np.ndarray:
    """Sum of the two triangles of each cell (triangle ids 2c and 2c+1)."""
    return g_tri.reshape(-1, 2).sum(axis=1)
