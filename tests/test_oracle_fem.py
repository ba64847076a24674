"""Pins of the oracle's finite-element pieces against closed forms and invariants.

Each check is independent of the oracle's own assembly code: closed-form stencils
built directly with Kronecker products, hand-derived mass/load totals, the energy
whose gradient K must be, the monotonicity/Lipschitz bounds of assumption (A1),
and special cases that reduce K to a linear operator.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import fem


def five_point(n: int) -> sp.csr_matrix:
    """5-point stencil (4, -1, -1, -1, -1) on the (n-1)^2 interior nodes, x fastest."""
    m = n - 1
    T = sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
    I = sp.identity(m)
    return (sp.kron(I, T) + sp.kron(T, I)).tocsr()


@pytest.mark.parametrize("n", [4, 8, 17, 32])
def test_stiffness_is_five_point_stencil(n):
    # On the SW-NE split grid the P1 stiffness is the h-independent 5-point stencil:
    # the coupling across the diagonal vanishes because the opposite angles are right angles.
    d = fem.discretise(W.Problem(n=n, N=4))
    diff = (d.S - five_point(n)).toarray()
    assert np.max(np.abs(diff)) < 1e-13


@pytest.mark.parametrize("n", [4, 8, 32])
def test_mass_total_and_structure(n):
    p = W.Problem(n=n, N=4, sigma_in=2.5)
    d = fem.discretise(p)
    M = d.M
    # 1^T M 1 = int sigma = sigma * area of the block (block strictly inside, aligned for n % 4 == 0)
    assert abs(M.sum() - 2.5 * 0.25) < 1e-14
    assert abs(M - M.T).max() < 1e-16
    ev = np.linalg.eigvalsh(M.toarray())
    assert ev.min() > -1e-15
    # rows of nodes with no conducting neighbour triangle vanish (degenerate mass, (A2))
    xy = d.mesh.xy[d.free_idx]
    outside = (xy[:, 0] < 0.25 - 1e-12) | (xy[:, 0] > 0.75 + 1e-12) | \
              (xy[:, 1] < 0.25 - 1e-12) | (xy[:, 1] > 0.75 + 1e-12)
    assert np.all(np.asarray(abs(M).sum(axis=1)).ravel()[outside] == 0.0)


def test_mass_interior_row_closed_form():
    # Interior node of the conducting block: 6 triangles of area h^2/2, consistent mass
    # |T|/12 (2 on the diagonal, 1 off it): diagonal h^2/2, and h^2/12 to each of the
    # six neighbours E, W, N, S, NE, SW (two triangles share each of those edges).
    n = 16
    h = 1.0 / n
    d = fem.discretise(W.Problem(n=n, N=4))
    i, j = 8, 8
    def fid(a, b):  # free-node index of node (a, b)
        return (b - 1) * (n - 1) + (a - 1)
    row = d.M.getrow(fid(i, j)).toarray().ravel()
    expect = np.zeros_like(row)
    expect[fid(i, j)] = h * h / 2
    for (a, b) in [(i + 1, j), (i - 1, j), (i, j + 1), (i, j - 1), (i + 1, j + 1), (i - 1, j - 1)]:
        expect[fid(a, b)] = h * h / 12
    assert np.max(np.abs(row - expect)) < 1e-17


def test_load_total_aligned_coil():
    # n = 20: the coil [0.1,0.2]x[0.3,0.7] is a union of cells, so sum b = J0 * area = 0.04 J0.
    p = W.Problem(n=20, N=4, J0=7.0)
    d = fem.discretise(p)
    assert abs(d.b.sum() - 7.0 * 0.04) < 1e-13


def test_load_total_brute_force_count():
    # Non-aligned grid: count coil triangles by their centroids with plain loops.
    n = 32
    p = W.Problem(n=n, N=4, J0=3.0)
    d = fem.discretise(p)
    h = 1.0 / n
    count = 0
    for j in range(n):
        for i in range(n):
            for (cx, cy) in [((i + 2 / 3) * h, (j + 1 / 3) * h), ((i + 1 / 3) * h, (j + 2 / 3) * h)]:
                if 0.1 <= cx <= 0.2 and 0.3 <= cy <= 0.7:
                    count += 1
    # every coil triangle has all its vertices free (the coil is away from the boundary)
    assert abs(d.b.sum() - 3.0 * count * h * h / 2) < 1e-13


def _rand_u(d, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    u = np.zeros(d.mesh.nodes)
    u[d.free_idx] = rng.standard_normal(d.nfree) * scale
    return u


def test_K_linear_law_is_scaled_stiffness():
    p = W.Problem(n=12, N=4, nu_a=3.5, nu_b=0.0, nu_out=3.5)
    d = fem.discretise(p)
    u = _rand_u(d, 1)
    Ku = fem.apply_K(p, d.mesh, d.mat, u)[d.free_idx]
    assert np.allclose(Ku, 3.5 * (d.S @ u[d.free_idx]), rtol=0, atol=1e-12)


@pytest.mark.parametrize("scale", [0.05, 1.0, 20.0])
def test_K_is_gradient_of_energy(scale):
    # K = grad E with E(u) = sum_T |T| W(|grad u_T|^2), W' = nu/2 (central differences).
    p = W.Problem(n=6, N=4, nu_rect=W.Rect(0.0, 0.0, 1.0, 0.6))
    d = fem.discretise(p)
    u = _rand_u(d, 2, scale=scale / 6)
    Ku = fem.apply_K(p, d.mesh, d.mat, u)
    eps = 1e-6 * max(1.0, np.abs(u).max())
    for idx in d.free_idx[::3]:
        e = np.zeros_like(u)
        e[idx] = eps
        fd = (fem.energy(p, d.mesh, d.mat, u + e) - fem.energy(p, d.mesh, d.mat, u - e)) / (2 * eps)
        assert abs(fd - Ku[idx]) <= 1e-6 * max(1.0, np.abs(Ku).max())


def test_nu_law_values():
    # nu(s) = 1 + 9 s^2/(1+s^2): nu(0) = 1, nu(1) = 5.5, nu(3) = 9.1, -> 10 as s -> infinity.
    p = W.config1()
    m = fem.build_mesh(2)
    mat = fem.materials(p, m)
    s2 = np.array([0.0, 1.0, 9.0, 1e12])
    iron = fem.Materials(sigma=np.zeros(4), iron=np.ones(4, bool), theta=np.ones(4), J=np.zeros(4))
    nu = fem.nu_of_s2(s2, iron, p)
    assert np.allclose(nu, [1.0, 5.5, 9.1, 10.0], rtol=1e-12)
    air = fem.Materials(sigma=np.zeros(4), iron=np.zeros(4, bool), theta=np.ones(4), J=np.zeros(4))
    assert np.all(fem.nu_of_s2(s2, air, p) == 1.0)
    assert mat.iron.dtype == bool


def test_K_monotone_and_lipschitz():
    # (A1) for this law: the Jacobian tensor nu I + 2 nu' g g^T has eigenvalues in [1, 11.125],
    # so 1 ||v||_S^2 <= <K(u+v) - K(u), v> <= 11.125 ||v||_S^2 (mean-value theorem).
    p = W.Problem(n=10, N=4, nu_rect=W.Rect(0.0, 0.0, 1.0, 1.0))
    d = fem.discretise(p)
    for seed, scale in [(0, 0.01), (1, 0.3), (2, 3.0), (3, 30.0)]:
        u = _rand_u(d, seed, scale)
        v = _rand_u(d, seed + 100, scale)
        dK = fem.apply_K(p, d.mesh, d.mat, u + v) - fem.apply_K(p, d.mesh, d.mat, u)
        num = dK[d.free_idx] @ v[d.free_idx]
        vs = v[d.free_idx] @ (d.S @ v[d.free_idx])
        assert vs * (1 - 1e-12) <= num <= 11.125 * vs * (1 + 1e-12)


def test_K_is_odd_and_vanishes_on_affine_fields():
    p = W.config1()
    d = fem.discretise(W.with_size(p, 16, 4))
    u = _rand_u(d, 5, 0.3)
    assert np.allclose(fem.apply_K(d.p, d.mesh, d.mat, -u), -fem.apply_K(d.p, d.mesh, d.mat, u), atol=1e-14)
    # affine u with constant nu: the flux is constant, so K(u) = 0 at interior nodes
    p2 = W.Problem(n=16, N=4, nu_b=0.0)
    d2 = fem.discretise(p2)
    u2 = 0.7 * d2.mesh.xy[:, 0] - 1.3 * d2.mesh.xy[:, 1]
    assert np.max(np.abs(fem.apply_K(p2, d2.mesh, d2.mat, u2)[d2.free_idx])) < 1e-13


def test_jacobian_matches_directional_difference():
    p = W.Problem(n=8, N=4, nu_rect=W.Rect(0.0, 0.0, 1.0, 1.0))
    d = fem.discretise(p)
    u = _rand_u(d, 7, 0.5)
    v = _rand_u(d, 8, 1.0)
    J = fem.jacobian_K(p, d.mesh, d.mat, u)
    eps = 1e-6
    fd = (fem.apply_K(p, d.mesh, d.mat, u + eps * v) - fem.apply_K(p, d.mesh, d.mat, u - eps * v)) / (2 * eps)
    assert np.allclose((J @ v)[d.free_idx], fd[d.free_idx], rtol=1e-7, atol=1e-8)


def test_region_membership_has_no_centroid_ties():
    # the centroid coordinates (k + 1/3) h and (k + 2/3) h never equal a rectangle edge
    for n in (32, 256, 1024):
        for v in (0.05, 0.1, 0.2, 0.25, 0.3, 0.7, 0.75, 0.95):
            frac = (v * n) % 1.0
            assert min(abs(frac - 1 / 3), abs(frac - 2 / 3)) > 1e-6
