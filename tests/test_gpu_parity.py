"""GPU parity: every entry point of the C ABI against the FP64 oracle on seeded inputs.

Tolerances (FP64 path): pointwise operators agree to rounding (relative 1e-12 in the
max norm); transforms to 1e-12 relative; full periodic solutions to a relative L2 error
of 1e-8 when both sides stop at a relative residual of 1e-12 (the error is at most the
condition number of the linearised space-time operator times the residual, and the
condition number at these sizes is below 1e3). FP32+refinement reaches the same FP64
residual, so it meets the same solution bound; its FP32-only kernels (transforms,
operator, preconditioner) are held to 2e-6 relative (a few float ulps times log N).
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import dft, fem, periodic as pp
from tests.gpu_helpers import say, oracle_K_full, oracle_shifted, rel_err, vcycle_reference

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2502_21013_amd as P
    P.library()
    return P


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


# ---------------------------------------------------------------- nonlinear operator

@pytest.mark.parametrize("n,N,seed,scale", [(4, 4, 0, 1.0), (32, 8, 1, 0.05), (32, 8, 2, 3.0), (64, 4, 3, 0.3)])
def test_apply_K_matches_oracle(gpu, P, n, N, seed, scale):
    say(f"apply_K n={n} N={N} seed={seed}")
    p = W.with_size(W.config2(seed), n, N)
    d = fem.discretise(p)
    U = W.random_field(N, n, seed, scale)
    plan = P.Plan(p)
    KU = plan.apply_K(dev(U)).cpu().numpy()
    ref = oracle_K_full(d, U)
    assert np.max(np.abs(KU - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_apply_K_partial_slices_and_theta(gpu, P):
    n, N = 16, 8
    say(f"apply_K theta n={n} N={N}")
    p0 = W.config5(seed=3, n=n, N=N)
    d = fem.discretise(p0)
    U = W.random_field(N, n, 7, 0.5)
    theta = dev(p0.theta)
    plan = P.Plan(p0, theta=theta)
    KU = plan.apply_K(dev(U), nslices=3).cpu().numpy()
    ref = oracle_K_full(d, U)
    assert np.max(np.abs(KU[:3] - ref[:3])) <= 1e-12 * np.max(np.abs(ref[:3]))


# ---------------------------------------------------------------- residual

@pytest.mark.parametrize("n,N,seed", [(32, 32, 0), (16, 64, 1), (8, 4, 2)])
def test_residual_matches_oracle(gpu, P, n, N, seed):
    say(f"residual n={n} N={N} seed={seed}")
    p = W.with_size(W.config2(seed), n, N)
    d = fem.discretise(p)
    U = W.random_field(N, n, seed + 10, 0.1)
    plan = P.Plan(p)
    R, rel, fn = plan.residual(dev(U))
    R = R.cpu().numpy()
    F = pp.load_series(d)
    Rref = pp.to_full(d, pp.residual(d, pp.to_free(d, U), F))
    assert np.max(np.abs(R - Rref)) <= 1e-12 * np.max(np.abs(Rref))
    assert abs(fn - np.linalg.norm(F)) <= 1e-12 * np.linalg.norm(F)
    assert abs(rel - np.linalg.norm(Rref) / np.linalg.norm(F)) <= 1e-12 * rel


def test_residual_with_explicit_load_and_sigma_table(gpu, P):
    n, N = 16, 16
    say(f"residual explicit load n={n} N={N}")
    p = W.with_size(W.config1(), n, N)
    rng = np.random.default_rng(5)
    sigma = rng.uniform(0.0, 2.0, 2 * n * n) * (rng.uniform(size=2 * n * n) < 0.5)
    d = fem.discretise(p)
    # the oracle with the same per-triangle conductivity
    d.mat.sigma = sigma.copy()
    d.M = fem.restrict(fem.mass_full(d.mesh, sigma), d.mesh.free)
    F = W.random_field(N, n, 11, 1.0)
    U = W.random_field(N, n, 12, 0.3)
    plan = P.Plan(p, sigma=dev(sigma), load=dev(F))
    R, rel, fn = plan.residual(dev(U))
    Ff = pp.to_free(d, F)
    Rref = pp.to_full(d, pp.residual(d, pp.to_free(d, U), Ff))
    assert np.max(np.abs(R.cpu().numpy() - Rref)) <= 1e-12 * np.max(np.abs(Rref))


# ---------------------------------------------------------------- time DFT

@pytest.mark.parametrize("N", [4, 8, 32, 64, 128, 256, 512, 1024])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_time_dft_matches_definition(gpu, P, N, precision):
    n = 8
    say(f"rfft/irfft N={N} {precision}")
    p = W.with_size(W.config1(), n, N)
    X = W.random_field(N, n, N, 1.0)
    plan = P.Plan(p, precision=precision)
    Xh = plan.rfft(dev(X)).cpu().numpy()
    ref = dft.rfft_packed(X.reshape(N, -1)).T            # (nodes, S)
    tol = 1e-12 if precision == "fp64" else 2e-6
    assert rel_err(Xh, ref) <= tol
    cd = np.complex128 if precision == "fp64" else np.complex64
    back = plan.irfft(dev(ref.astype(cd)))
    assert rel_err(back.cpu().numpy(), X) <= tol


# ---------------------------------------------------------------- residual spectrum (fused step)

@pytest.mark.parametrize("n,N,seed", [(8, 8, 0), (16, 64, 1), (32, 128, 2), (8, 512, 3), (8, 1024, 4), (8, 4, 5)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_residual_spectrum_is_the_dft_of_the_residual(gpu, P, n, N, seed, precision):
    # 4 <= N/2 <= 256 runs the fused sweep (residual and its DFT in one pass), N = 4 and 1024 the
    # two-kernel path. Either way: the DFT entry point applied to the residual entry point to a
    # few units in the last place (same twiddles and butterflies; the compiler may fuse a
    # multiply-add differently in the two kernels), the same FP64 norms up to the order of
    # their partial sums (the fused sweep adds each node's terms on the lanes that transform
    # it), and the oracle's DFT of the oracle residual to the transform tolerance
    say(f"residual spectrum n={n} N={N} {precision}")
    p = W.with_size(W.config2(seed), n, N)
    d = fem.discretise(p)
    U = W.random_field(N, n, seed + 20, 0.1)
    plan = P.Plan(p, precision=precision)
    Rh, rel, fn = plan.residual_spectrum(dev(U))
    R, rel2, fn2 = plan.residual(dev(U))
    two = plan.rfft(R)
    ulp = 8 * (2.0 ** -52 if precision == "fp64" else 2.0 ** -23)
    assert float((Rh - two).abs().max()) <= ulp * float(two.abs().max())
    assert abs(rel - rel2) <= 1e-13 * rel2 and fn == fn2
    F = pp.load_series(d)
    Rref = pp.to_full(d, pp.residual(d, pp.to_free(d, U), F))
    ref = dft.rfft_packed(Rref.reshape(N, -1)).T            # (nodes, S)
    tol = 1e-12 if precision == "fp64" else 2e-6
    assert rel_err(Rh.cpu().numpy(), ref) <= tol
    plan.close()


# ---------------------------------------------------------------- frequency-domain operator

@pytest.mark.parametrize("n,N", [(8, 8), (32, 32), (16, 128)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shifted_operator_matches_oracle(gpu, P, n, N, precision):
    say(f"shifted_apply n={n} N={N} {precision}")
    p = W.with_size(W.config2(1), n, N)
    d = fem.discretise(p)
    rng = np.random.default_rng(n + N)
    nodes = (n + 1) ** 2
    Xh = rng.standard_normal((nodes, N // 2)) + 1j * rng.standard_normal((nodes, N // 2))
    Xh[~d.mesh.free] = 0
    plan = P.Plan(p, precision=precision)
    cd = np.complex128 if precision == "fp64" else np.complex64
    Y = plan.shifted_apply(dev(Xh.astype(cd))).cpu().numpy()
    ref = oracle_shifted(d, Xh)
    tol = 1e-12 if precision == "fp64" else 2e-6
    assert rel_err(Y, ref) <= tol


# grid targets 110 / 66 / 22 give chunks of 3 rows at these sizes, so chunks start on odd rows
@pytest.mark.parametrize("n,N,grid,precision", [(16, 16, 0, "fp64"), (64, 32, 0, "fp64"), (64, 32, 8, "fp64"),
                                                (64, 32, 110, "fp64"), (64, 32, 66, "fp32"), (32, 16, 22, "fp64")])
def test_vcycle_is_symmetric_and_contracts(gpu, P, n, N, grid, precision):
    # B_s^T = B_s for the bilinear form (needed by COCG), and x <- x + B (r - A x)
    # converges at a mesh-independent rate. Small grid targets give long row chunks that
    # start at even and odd rows (the sweeping kernels' rolling windows).
    say(f"vcycle n={n} N={N} grid={grid} {precision}")
    p = W.with_size(W.config2(2), n, N)
    d = fem.discretise(p)
    plan = P.Plan(p, grid_slot=grid, precision=precision, cycle="v11")
    rng = np.random.default_rng(3)
    nodes = (n + 1) ** 2
    r1 = rng.standard_normal((nodes, N // 2)) + 1j * rng.standard_normal((nodes, N // 2))
    r2 = rng.standard_normal((nodes, N // 2)) + 1j * rng.standard_normal((nodes, N // 2))
    r1[~d.mesh.free] = 0
    r2[~d.mesh.free] = 0
    cd = np.complex128 if precision == "fp64" else np.complex64
    tol = 1e-12 if precision == "fp64" else 2e-5
    r1, r2 = r1.astype(cd), r2.astype(cd)
    B1 = plan.precond_apply(dev(r1)).cpu().numpy().astype(np.complex128)
    B2 = plan.precond_apply(dev(r2)).cpu().numpy().astype(np.complex128)
    for s in range(1, N // 2):
        a = np.sum(B1[:, s] * r2[:, s])
        b = np.sum(r1[:, s] * B2[:, s])
        assert abs(a - b) <= tol * max(abs(a), 1e-30)
    for part in (np.real, np.imag):  # slot 0: two real symmetric operators
        a = np.sum(part(B1[:, 0]) * part(r2[:, 0]))
        b = np.sum(part(r1[:, 0]) * part(B2[:, 0]))
        assert abs(a - b) <= tol * abs(a)
    # stationary iteration with the V-cycle: error reduction per cycle
    x = np.zeros_like(r1)
    rn = [np.linalg.norm(r1, axis=0)]
    for _ in range(6):
        Ax = plan.shifted_apply(dev(x)).cpu().numpy()
        x = x + plan.precond_apply(dev((r1 - Ax).astype(cd))).cpu().numpy()
        rn.append(np.linalg.norm(r1 - plan.shifted_apply(dev(x)).cpu().numpy(), axis=0))
    rate = (rn[-1] / rn[0]) ** (1 / 6)
    assert np.all(rate < 0.5), rate.max()


# n = 16: the finest level in the per-level sweeps, the rest (9, 5, 3 points per side) in the
# small-level kernel; n = 64 and 128: two and three levels in the per-level sweeps; (64, 8, 66):
# row chunks that start on odd rows. Both cycle shapes, V(1,1) and V(0,1).
@pytest.mark.parametrize("n,N,grid", [(16, 8, 0), (64, 8, 0), (128, 4, 0), (64, 8, 66)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("cycle", ["v11", "v01"])
def test_vcycle_matches_its_definition(gpu, P, n, N, grid, precision, cycle):
    say(f"vcycle definition n={n} N={N} grid={grid} {precision} {cycle}")
    p = W.with_size(W.config2(2), n, N)
    d = fem.discretise(p)
    plan = P.Plan(p, precision=precision, vc_omega=0.8, cycle=cycle, grid_slot=grid)
    rng = np.random.default_rng(n + N)
    nodes = (n + 1) ** 2
    R = rng.standard_normal((nodes, N // 2)) + 1j * rng.standard_normal((nodes, N // 2))
    R[~d.mesh.free] = 0
    cd = np.complex128 if precision == "fp64" else np.complex64
    R = R.astype(cd)
    B = plan.precond_apply(dev(R)).cpu().numpy().astype(np.complex128)
    ref = vcycle_reference(d, 0.8, R.astype(np.complex128), pre=1 if cycle == "v11" else 0)
    tol = 1e-12 if precision == "fp64" else 5e-5
    assert rel_err(B, ref) <= tol
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_v01_cycle_contracts(gpu, P, precision):
    # the default cycle of the Galerkin step: x <- x + B (r - A x) converges at a
    # mesh-independent rate (checked at two sizes)
    for n in (32, 64):
        say(f"v01 contraction n={n} {precision}")
        p = W.with_size(W.config2(2), n, 16)
        d = fem.discretise(p)
        plan = P.Plan(p, precision=precision, cycle="v01")
        rng = np.random.default_rng(5)
        nodes = (n + 1) ** 2
        r1 = rng.standard_normal((nodes, 8)) + 1j * rng.standard_normal((nodes, 8))
        r1[~d.mesh.free] = 0
        cd = np.complex128 if precision == "fp64" else np.complex64
        r1 = r1.astype(cd)
        x = np.zeros_like(r1)
        rn0 = np.linalg.norm(r1, axis=0)
        for _ in range(6):
            Ax = plan.shifted_apply(dev(x)).cpu().numpy()
            x = x + plan.precond_apply(dev((r1 - Ax).astype(cd))).cpu().numpy()
        rn = np.linalg.norm(r1 - plan.shifted_apply(dev(x)).cpu().numpy(), axis=0)
        rate = (rn / rn0) ** (1 / 6)
        assert np.all(rate < 0.5), rate.max()
        plan.close()


# ---------------------------------------------------------------- periodic linear solve

@pytest.mark.parametrize("n,N", [(16, 16), (32, 8)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_periodic_solve_matches_spacetime_lu(gpu, P, n, N, precision):
    say(f"periodic_solve n={n} N={N} {precision}")
    p = W.with_size(W.config2(3), n, N)
    d = fem.discretise(p)
    R = W.random_field(N, n, 21, 1.0)
    plan = P.Plan(p, precision=precision, inner="cocg", inner_iters=30)
    X = plan.periodic_solve(dev(R)).cpu().numpy()
    ref = pp.to_full(d, pp.SpaceTimeLU(d).solve(pp.to_free(d, R)))
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert rel_err(X, ref) <= tol


# ---------------------------------------------------------------- full solve

@pytest.fixture(scope="module")
def c1_oracle():
    d = fem.discretise(W.config1())
    r = pp.fixed_point(d, tol=1e-12, max_iter=2000)
    return d, r


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("inner,iters", [("galerkin1", 1), ("cocg", 2)])
def test_config1_solution_matches_oracle(gpu, P, c1_oracle, precision, inner, iters):
    say(f"solve config1 {precision} {inner}")
    d, ref = c1_oracle
    plan = P.Plan(W.config1(), tol=1e-12, precision=precision, inner=inner, inner_iters=iters, max_outer=2000)
    U, st = plan.solve()
    U = U.cpu().numpy()
    assert st.rel_residual <= 1e-12
    Uref = pp.to_full(d, ref.U)
    assert rel_err(U, Uref) <= 1e-8
    # the GPU residual of the returned iterate agrees with the oracle's residual of it
    Rref = pp.residual(d, pp.to_free(d, U), ref.F)
    assert abs(np.linalg.norm(Rref) / np.linalg.norm(ref.F) - st.rel_residual) <= 1e-3 * st.rel_residual + 1e-15


def test_config1_tolerance_and_iteration_count(gpu, P, c1_oracle):
    say("solve config1 tol 1e-10")
    d, ref = c1_oracle
    plan = P.Plan(W.config1(), tol=1e-10)
    U, st = plan.solve()
    oracle_iters = next(k for k, r in enumerate(ref.rel) if r <= 1e-10)
    assert st.rel_residual <= 1e-10
    # inexact inner solves cost only a few extra outer steps over the exact oracle
    assert oracle_iters <= st.outer_iters <= oracle_iters + 30
    h = np.array(st.history)
    assert np.all(h[1:] < h[:-1])  # monotone decrease of the residual


def test_manufactured_solution_explicit_load(gpu, P):
    n, N = 32, 16
    say(f"manufactured n={n} N={N}")
    p = W.with_size(W.config2(4), n, N)
    d = fem.discretise(p)
    a, b, c = W.manufactured_coeffs(1)
    t = p.tau * np.arange(1, N + 1)
    prof = a + b * np.cos(2 * np.pi * t) + c * np.sin(4 * np.pi * t)
    xy = d.mesh.xy[d.free_idx]
    Ustar = prof[:, None] * (np.sin(np.pi * xy[:, 0]) * np.sin(np.pi * xy[:, 1]))[None, :] * 3.0
    F = pp.to_full(d, pp.apply_A(d, Ustar))
    plan = P.Plan(p, tol=1e-12, load=dev(F), max_outer=2000)
    U, st = plan.solve()
    assert rel_err(U.cpu().numpy(), pp.to_full(d, Ustar)) <= 1e-9


def test_half_wave_symmetry_and_energy_balance(gpu, P):
    n, N = 64, 32
    say(f"symmetry/energy n={n} N={N}")
    p = W.with_size(W.config2(0), n, N)
    d = fem.discretise(p)
    plan = P.Plan(p, tol=1e-12, max_outer=2000)
    U, st = plan.solve()
    U = U.cpu().numpy()
    assert np.linalg.norm(U[N // 2:] + U[:N // 2]) <= 1e-10 * np.linalg.norm(U)
    Uf = pp.to_free(d, U)
    F = pp.load_series(d)
    dU = (Uf - np.roll(Uf, 1, axis=0)) / p.tau
    lhs = p.tau * np.sum(dU * (d.M @ dU.T).T)
    rhs = 2 * np.sum((F - pp.K_free(d, Uf)) * Uf)
    assert abs(lhs - rhs) <= 1e-8 * abs(lhs)


# ---------------------------------------------------------------- extreme sizes

@pytest.mark.parametrize("law", ["rational", "expcap"])
def test_apply_K_reads_boundary_entries_as_zero(gpu, P, law):
    # the time-field convention: boundary entries of an input are read as 0, so K of a field
    # with a nonzero boundary ring is K of the same field with the ring zeroed
    say(f"apply_K boundary ring {law}")
    n, N = 16, 4
    p = W.transformer(n, N) if law == "expcap" else W.with_size(W.config2(4), n, N)
    U = W.random_field(N, n, 13, 0.05)
    V = U.copy()
    rng = np.random.default_rng(14)
    for sl in (np.s_[:, 0, :], np.s_[:, -1, :], np.s_[:, :, 0], np.s_[:, :, -1]):
        V[sl] = rng.standard_normal(V[sl].shape)
    kw = dict(region=dev(W.region_ids(p))) if law == "expcap" else {}
    plan = P.Plan(p, **kw)
    a, b = plan.apply_K(dev(U)), plan.apply_K(dev(V))
    assert torch.equal(a, b)
    r, _, _ = plan.residual(dev(U))
    s, _, _ = plan.residual(dev(V))
    assert torch.equal(r, s)
    plan.close()


def test_largest_grid_operator_and_solve(gpu, P):
    # n = 4096, the ABI's largest grid (13 multigrid levels), N = 8.
    # (a) With uniform nu (no iron) and no current, K annihilates an affine field at every node
    # whose neighbours are all interior (P1 is exact on linear functions, and |grad u| is the same
    # on every triangle, so the law gives one nu everywhere); boundary entries are read as 0, so
    # the nodes next to the boundary see the jump. A time-constant field has no mass term: the
    # operator, the residual sweep and its fused DFT all return zero there, up to rounding.
    # (b) The seeded problem at this size converges in both precision modes to the same iterate.
    n, N = 4096, 8
    say(f"largest grid n={n} N={N}")
    base = W.with_size(W.config2(5), n, N)
    p = dataclasses.replace(base, nu_rect=W.Rect(0.0, 0.0, 0.0, 0.0), J0=0.0)
    x = np.linspace(0.0, 1.0, n + 1)
    u = 0.3 * x[None, :] - 0.7 * x[:, None] + 0.1          # u(x_i, y_j) = 0.3 x - 0.7 y + 0.1
    u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = 0.0
    U = dev(np.broadcast_to(u, (N, n + 1, n + 1)).copy())
    scale = 4 * p.nu_out * float(np.abs(u).max())
    plan = P.Plan(p, precision="fp64")
    KU = plan.apply_K(U)
    assert float(KU[:, 2:-2, 2:-2].abs().max()) <= 1e-12 * scale
    assert float(KU[:, 1, 1:-1].abs().min()) >= 0.05 * p.nu_out     # the jump next to y = 0
    R, _, fn = plan.residual(U)
    assert fn == 0.0
    assert float(R[:, 2:-2, 2:-2].abs().max()) <= 1e-12 * scale
    assert torch.allclose(R[:, 1:-1, 1:-1], -KU[:, 1:-1, 1:-1], rtol=0, atol=1e-12 * scale)
    Rh, _, _ = plan.residual_spectrum(U)
    Rh = Rh.reshape(n + 1, n + 1, -1)
    assert float(Rh[2:-2, 2:-2].abs().max()) <= 1e-11 * scale
    plan.close()
    del KU, R, Rh, U
    sol = {}
    for precision in ("fp64", "fp32"):
        pl = P.Plan(base, tol=1e-8, precision=precision, max_outer=2000)
        V, st = pl.solve()
        assert st.rel_residual <= 1e-8
        sol[precision] = (V, st.outer_iters)
        pl.close()
    (a, ka), (b, kb) = sol["fp32"], sol["fp64"]
    assert abs(ka - kb) <= 8
    assert float((a - b).norm() / b.norm()) <= 1e-6

_extreme_ref = {}

@pytest.mark.parametrize("n,N", [(4, 4), (8, 1024), (16, 64), (64, 8)])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_solution_at_extreme_sizes_matches_oracle(gpu, P, n, N, precision):
    # smallest grid and period, the longest period (two time pairs per lane in the residual
    # sweep), a period with fewer slots than a wavefront, and a short period on a larger grid
    say(f"extreme n={n} N={N} {precision}")
    p = W.with_size(W.config2(11), n, N)
    if (n, N) not in _extreme_ref:
        d = fem.discretise(p)
        _extreme_ref[(n, N)] = (d, pp.fixed_point(d, tol=1e-13, max_iter=3000))
    d, ref = _extreme_ref[(n, N)]
    U, st = P.Plan(p, tol=1e-12, max_outer=3000, precision=precision).solve()
    assert st.rel_residual <= 1e-12
    assert rel_err(U.cpu().numpy(), pp.to_full(d, ref.U)) <= 1e-8
