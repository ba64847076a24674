"""Pins of the oracle's region mode and of the law of Sec. 4, nu(s) = a min(exp(b s^2), c) + d, on
the transformer cross-section (figure fig:domain, table tab:coef), checked against facts fixed
by the paper's table and by the mathematics rather than against the oracle itself."""
import numpy as np
import pytest

import workloads as W
from oracle import fem, periodic as pp

MU0_INV = 1e7 / (4 * np.pi)   # vacuum reluctivity, the table's d of air and windings


def _rand_u(d, seed, scale):
    rng = np.random.default_rng(seed)
    u = np.zeros(d.mesh.nodes)
    u[d.free_idx] = rng.standard_normal(d.nfree) * scale
    return u


def _mat_one(law, a, b, c, dd, n=1):
    one = np.ones(n)
    return fem.Materials(sigma=0 * one, iron=one > 0, theta=one.copy(), J=0 * one, law=law,
                         a=a * one, b=b * one, c=c * one, d=dd * one)


def test_table_saturates_at_vacuum_reluctivity():
    # The exp-capped law of iron and steel ends at a c + d, which the table's values put at the
    # vacuum reluctivity 1/mu0 = 10^7/(4 pi) (the d of air): a mistyped a, c or d breaks this.
    regs = {r.name: r for r in W.TRANSFORMER_REGIONS}
    for name in ("iron", "steel"):
        r = regs[name]
        assert abs(r.a * r.c + r.d - MU0_INV) <= 1e-5 * MU0_INV
        mat = _mat_one("expcap", r.a, r.b, r.c, r.d, 3)
        s2 = np.array([2 * np.log(r.c) / r.b, 10 * np.log(r.c) / r.b, 1e6])
        assert np.allclose(fem.nu_of_s2(s2, mat, None), r.a * r.c + r.d, rtol=1e-15)
    for name in ("air", "winding+", "winding-"):
        assert regs[name].a == 0.0 and regs[name].d == pytest.approx(MU0_INV, rel=1e-15)


def test_expcap_law_values_and_continuity():
    # nu(0) = a + d; nu(s) = a exp(b s^2) + d below saturation; continuous at s^2 = ln(c)/b,
    # where the derivative drops from a b c to 0 (right derivative).
    r = {x.name: x for x in W.TRANSFORMER_REGIONS}["iron"]
    mat = _mat_one("expcap", r.a, r.b, r.c, r.d, 1)
    zs = np.log(r.c) / r.b
    assert fem.nu_of_s2(np.array([0.0]), mat, None)[0] == pytest.approx(r.a + r.d, rel=1e-15)
    lo, hi = fem.nu_of_s2(np.array([zs * (1 - 1e-12)]), mat, None)[0], fem.nu_of_s2(np.array([zs]), mat, None)[0]
    assert abs(lo - hi) <= 1e-9 * hi
    dlo = fem.dnu_ds2(np.array([zs * (1 - 1e-9)]), mat, None)[0]
    assert dlo == pytest.approx(r.a * r.b * r.c, rel=1e-6)
    assert fem.dnu_ds2(np.array([zs * (1 + 1e-9)]), mat, None)[0] == 0.0
    # the derivative is the difference quotient of the law away from the kink
    for z in (0.3, 2.0, 5.0):
        e = 1e-6
        fd = (fem.nu_of_s2(np.array([z + e]), mat, None)[0] - fem.nu_of_s2(np.array([z - e]), mat, None)[0]) / (2 * e)
        assert fd == pytest.approx(fem.dnu_ds2(np.array([z]), mat, None)[0], rel=1e-7)


def _transformer(n=8, N=4):
    return W.transformer(n, N)


def test_transformer_layout():
    # every region present; the windings are interior and come in +/- pairs of equal area
    p = _transformer(64)
    rid = W.region_ids(p)
    counts = np.bincount(rid, minlength=len(p.regions))
    assert np.all(counts > 0)
    assert counts[3] == counts[4]
    d = fem.discretise(p)
    # the steel wall (sigma = 1e7) is the only conductor: M is nonzero only near it
    sig = d.mat.sigma
    assert set(np.unique(sig)) == {0.0, 1e7}
    assert np.all(rid[sig > 0] == 2)
    # the windings carry +-1.9e4 A/m^2: equal and opposite total currents
    area = d.mesh.area
    assert np.sum(d.mat.J * area) == pytest.approx(0.0, abs=1e-9 * np.sum(np.abs(d.mat.J) * area))


@pytest.mark.parametrize("scale", [0.02, 0.3, 3.0])
def test_expcap_K_is_gradient_of_energy(scale):
    # K = grad E with E(u) = sum_T |T| W(|grad u_T|^2), W' = nu/2 (central differences), with
    # fields below, around and beyond saturation of the iron and steel laws
    p = _transformer(8)
    d = fem.discretise(p)
    u = _rand_u(d, 4, scale)
    Ku = fem.apply_K(p, d.mesh, d.mat, u)
    eps = 1e-7 * max(1.0, np.abs(u).max())
    for idx in d.free_idx[::2]:
        e = np.zeros_like(u)
        e[idx] = eps
        fd = (fem.energy(p, d.mesh, d.mat, u + e) - fem.energy(p, d.mesh, d.mat, u - e)) / (2 * eps)
        assert abs(fd - Ku[idx]) <= 1e-6 * np.abs(Ku).max()


@pytest.mark.parametrize("scale", [0.02, 0.3, 3.0])
def test_expcap_jacobian_is_derivative_of_K(scale):
    p = _transformer(8)
    d = fem.discretise(p)
    u = _rand_u(d, 6, scale)
    v = _rand_u(d, 7, scale)
    J = fem.jacobian_K(p, d.mesh, d.mat, u)
    eps = 1e-7
    fd = (fem.apply_K(p, d.mesh, d.mat, u + eps * v) - fem.apply_K(p, d.mesh, d.mat, u - eps * v)) / (2 * eps)
    ref = (J @ v)[d.free_idx]
    assert np.linalg.norm(fd[d.free_idx] - ref) <= 1e-6 * np.linalg.norm(ref)


def test_expcap_K_monotone_and_lipschitz_per_region_bounds():
    # (A1): the Jacobian tensor nu I + 2 nu'(s^2) g g^T has eigenvalues nu and (nu s)', which for
    # nu = a min(exp(b s^2), c) + d lie in [a + d, a c (1 + 2 ln c) + d]; so with
    # gamma = min_i (a_i + d_i) and L = max_i (a_i c_i (1 + 2 ln c_i) + d_i) over the regions,
    # gamma ||v||_S^2 <= <K(u+v) - K(u), v> <= L ||v||_S^2.
    p = _transformer(10)
    d = fem.discretise(p)
    gam = min(r.a + r.d for r in p.regions)
    L = max(r.a * r.c * (1 + 2 * np.log(r.c)) + r.d for r in p.regions)
    for seed, scale in [(0, 0.01), (1, 0.3), (2, 1.0), (3, 10.0)]:
        u = _rand_u(d, seed, scale)
        v = _rand_u(d, seed + 100, scale)
        dK = fem.apply_K(p, d.mesh, d.mat, u + v) - fem.apply_K(p, d.mesh, d.mat, u)
        num = dK[d.free_idx] @ v[d.free_idx]
        vs = v[d.free_idx] @ (d.S @ v[d.free_idx])
        assert gam * vs * (1 - 1e-12) <= num <= L * vs * (1 + 1e-12)


def test_region_mode_reproduces_rectangle_problem():
    # config 1 written as regions (air, iron, conductor, iron and conductor, coil) with the
    # rational law: the same mass, load and K(u) as the rectangle problem
    p = W.config1()
    R = W.Region
    regs = (R("air", a=p.nu_out), R("iron", a=p.nu_a, b=p.nu_b), R("cond", sigma=p.sigma_in, a=p.nu_out),
            R("iron+cond", sigma=p.sigma_in, a=p.nu_a, b=p.nu_b), R("coil", a=p.nu_out, j=p.J0))
    ir, sg, cl = p.nu_rect, p.sigma_rect, p.coil_rect
    both = W.Rect(max(ir.x0, sg.x0), max(ir.y0, sg.y0), min(ir.x1, sg.x1), min(ir.y1, sg.y1))
    layout = ((W.Rect(0, 0, 1, 1), 0), (sg, 2), (ir, 1), (both, 3), (cl, 4))
    q = W.Problem(n=p.n, N=p.N, law="rational", regions=regs, layout=layout)
    d1, d2 = fem.discretise(p), fem.discretise(q)
    assert abs(d1.M - d2.M).max() == 0.0
    assert np.array_equal(d1.b, d2.b)
    u = _rand_u(d1, 9, 0.3)
    assert np.allclose(fem.apply_K(p, d1.mesh, d1.mat, u), fem.apply_K(q, d2.mesh, d2.mat, u), rtol=1e-14, atol=1e-13)


def test_transformer_fixed_point_with_region_khat_contracts():
    # Thm. thm:iter with a per-region Khat (coefficient nu_hat_i per region, here the midpoint of
    # the region's (A1) range [a_i + d_i, a_i c_i (1 + 2 ln c_i) + d_i] clipped to the law's range
    # of values at the fields reached): the iteration reaches the solution and each step contracts
    # the error in the Khat norm. Fields small enough (j scaled down) to stay below saturation.
    p = W.transformer(8, 4, j_scale=1e-3)
    d = fem.discretise(p)
    rid = W.region_ids(p)
    nu_hat = np.array([r.a + r.d for r in p.regions])[rid] * 1.2
    d.khat_coef = nu_hat
    ref = pp.fixed_point(d, tol=1e-13, max_iter=400)
    assert ref.converged
    steps = np.array(ref.khat_step)
    assert np.all(steps[1:] <= steps[:-1] * (1 + 1e-9))
