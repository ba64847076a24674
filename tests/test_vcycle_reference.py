"""Pins of the test-side V-cycle reference (tests/gpu_helpers.vcycle_reference, V(1,1) and
V(0,1)) against facts that do not depend on it: P1 interpolation is exact on linear functions,
the Galerkin coarse mass equals the mass assembled on the coarse mesh when the conductivity is
constant on coarse triangles, V(1,1) is symmetric in the bilinear form and V(0,1) is the
transpose of V(1,0), both are the exact solve on the 2 x 2-cell grid, and as stationary
iterations they contract at a mesh-independent rate."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import dft, fem
from tests.gpu_helpers import _prolongation, vcycle_reference


def test_prolongation_is_exact_on_linear_functions():
    for nc in (1, 2, 8):
        P = _prolongation(nc)
        c = np.arange(nc + 1)
        X, Y = np.meshgrid(c, c)
        f = np.arange(2 * nc + 1) / 2
        FX, FY = np.meshgrid(f, f)
        assert np.abs(P @ (3 * X - 2 * Y + 1).ravel() - (3 * FX - 2 * FY + 1).ravel()).max() == 0.0


def test_galerkin_coarse_mass_is_the_coarse_assembly():
    # the conductivity block [0.25, 0.75]^2 is a union of coarse triangles on both grids
    p = W.with_size(W.config2(0), 16, 8)
    pc = W.with_size(W.config2(0), 8, 8)
    Mf = fem.mass_full(fem.build_mesh(16), fem.discretise(p).mat.sigma)
    Mc = fem.mass_full(fem.build_mesh(8), fem.discretise(pc).mat.sigma)
    P = _prolongation(8)
    assert abs(P.T @ Mf @ P - Mc).max() <= 1e-15 * abs(Mc).max()


def _regions_problem(n, N):
    # two regions with their own Khat coefficient, the inner one a union of triangles of every grid
    # down to 8 x 8 cells (its edges on multiples of 1/8)
    R = W.Region
    regs = (R("outer", a=1.0, nu_hat=3.0), R("inner", sigma=2.0, a=2.0, b=1.0, nu_hat=7.0))
    layout = ((W.Rect(0.0, 0.0, 1.0, 1.0), 0), (W.Rect(0.25, 0.25, 0.75, 0.625), 1))
    return W.Problem(n=n, N=N, law="rational", regions=regs, layout=layout, nu_max=10.0)


def test_region_khat_galerkin_coarse_is_the_coarse_assembly():
    # P^T Khat_f P equals the per-region stiffness assembled on the coarse mesh when the regions
    # are unions of coarse triangles; a constant coefficient gives nu_hat S
    pf, pc = _regions_problem(16, 8), _regions_problem(8, 8)
    df, dc = fem.discretise(pf), fem.discretise(pc)
    Kf = fem.stiffness_full(df.mesh, df.khat_coef)
    Kc = fem.stiffness_full(dc.mesh, dc.khat_coef)
    P = _prolongation(8)
    assert abs(P.T @ Kf @ P - Kc).max() <= 1e-13 * abs(Kc).max()
    assert set(np.unique(df.khat_coef)) == {3.0, 7.0}
    m = df.mesh
    assert abs(fem.stiffness_full(m, np.full(m.area.shape, 3.0)) - 3.0 * fem.stiffness_full(m)).max() <= 1e-13


def test_reference_cycle_with_region_khat():
    # with a per-region Khat the V(0,1) and V(1,0) cycles are still transposes of each other, and
    # the cycle is the exact solve on the 2 x 2-cell grid
    d = fem.discretise(_regions_problem(16, 8))
    rng = np.random.default_rng(9)
    R1, R2 = (rng.standard_normal((d.mesh.nodes, 4)) + 1j * rng.standard_normal((d.mesh.nodes, 4)) for _ in range(2))
    R1[~d.mesh.free] = 0
    R2[~d.mesh.free] = 0
    B01 = vcycle_reference(d, 0.8, R1, pre=0, post=1)
    B10 = vcycle_reference(d, 0.8, R2, pre=1, post=0)
    for s in range(1, 4):
        a, b = np.sum(B01[:, s] * R2[:, s]), np.sum(R1[:, s] * B10[:, s])
        assert abs(a - b) <= 1e-13 * abs(a)
    d2 = fem.discretise(_regions_problem(2, 8))
    R = rng.standard_normal((9, 4)) + 1j * rng.standard_normal((9, 4))
    R[~d2.mesh.free] = 0
    B = vcycle_reference(d2, 0.8, R, pre=0)
    z = dft.shifts(8, d2.p.tau)
    fi = d2.free_idx
    for s in range(1, 4):
        A = (d2.Khat + z[s] * d2.M).toarray()
        assert np.allclose(A @ B[fi, s], R[fi, s], rtol=1e-13, atol=0)


def _setup(n, N, seed):
    p = W.with_size(W.config2(seed), n, N)
    d = fem.discretise(p)
    rng = np.random.default_rng(seed)
    R = rng.standard_normal(((n + 1) ** 2, N // 2)) + 1j * rng.standard_normal(((n + 1) ** 2, N // 2))
    R[~d.mesh.free] = 0
    return d, R


def test_reference_cycle_is_symmetric():
    d, R1 = _setup(16, 8, 1)
    _, R2 = _setup(16, 8, 2)
    B1, B2 = vcycle_reference(d, 0.8, R1), vcycle_reference(d, 0.8, R2)
    for s in range(1, 4):
        a, b = np.sum(B1[:, s] * R2[:, s]), np.sum(R1[:, s] * B2[:, s])
        assert abs(a - b) <= 1e-13 * abs(a)


def test_reference_v01_is_the_transpose_of_v10():
    # The V(0,1) cycle smooths after the coarse correction only; its transpose in the bilinear
    # form is the V(1,0) cycle that smooths before it only (A, D and P^T M P are symmetric), so
    # r2^T B01 r1 = r1^T B10 r2. The two cycles run different code (no pre- / no post-smoothing).
    d, R1 = _setup(16, 8, 1)
    _, R2 = _setup(16, 8, 2)
    B01 = vcycle_reference(d, 0.8, R1, pre=0, post=1)
    B10 = vcycle_reference(d, 0.8, R2, pre=1, post=0)
    for s in range(1, 4):
        a, b = np.sum(B01[:, s] * R2[:, s]), np.sum(R1[:, s] * B10[:, s])
        assert abs(a - b) <= 1e-13 * abs(a)
    # and V(0,1) is not symmetric itself (the pins above and below would not see a cycle that
    # ignored the pre flag)
    B01b = vcycle_reference(d, 0.8, R2, pre=0, post=1)
    a, b = np.sum(B01[:, 1] * R2[:, 1]), np.sum(R1[:, 1] * B01b[:, 1])
    assert abs(a - b) > 1e-6 * abs(a)


@pytest.mark.parametrize("pre", [1, 0])
def test_reference_cycle_is_exact_on_the_coarsest_grid(pre):
    d, R = _setup(2, 8, 3)
    B = vcycle_reference(d, 0.8, R, pre=pre)
    z = dft.shifts(8, d.p.tau)
    A = lambda zz: (d.Khat + zz * d.M).toarray()
    fi = d.free_idx
    for s in range(1, 4):
        assert np.allclose(A(z[s]) @ B[fi, s], R[fi, s], rtol=1e-13, atol=0)


@pytest.mark.parametrize("n,pre", [(16, 1), (32, 1), (32, 0)])
def test_reference_cycle_contracts(n, pre):
    d, R = _setup(n, 8, 4)
    z = dft.shifts(8, d.p.tau)
    fi = d.free_idx
    for s in (1, 3):
        A = (d.Khat + z[s] * d.M).tocsr()
        x = np.zeros(fi.size, complex)
        r0 = np.linalg.norm(R[fi, s])
        for _ in range(6):
            res = np.zeros_like(R[:, :1].ravel())
            res[fi] = R[fi, s] - A @ x
            Rs = np.zeros_like(R)
            Rs[:, s] = res
            x = x + vcycle_reference(d, 0.8, Rs, pre=pre)[fi, s]
        rate = (np.linalg.norm(R[fi, s] - A @ x) / r0) ** (1 / 6)
        assert rate < 0.5
        # and the iterate approaches the direct solution
        xs = spla.spsolve(A.tocsc(), R[fi, s])
        assert np.linalg.norm(x - xs) <= 0.05 * np.linalg.norm(xs)
