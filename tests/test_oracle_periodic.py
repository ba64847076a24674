"""Pins of the oracle's periodic solvers against theory and independent computations.

* DFT block diagonalisation (remark rem:parallel): P U == idft((Khat + z_k M) dft(U)).
* Single-mode closed form for a linear law.
* Fixed-point iteration (Theorem thm:iter): one-step convergence when K = Khat,
  the exact rate 1 - c/nu_max when sigma = 0 and nu = c, contraction <= q in the
  Khat-norm at every step, and h/tau-independent rates.
* Final solution: manufactured discrete solution, all-at-once Newton, sequential
  time stepping to the limit cycle, the discrete energy balance (from the identity
  d_tau |a|^2 = 2 (d_tau a, a) - tau |d_tau a|^2 summed over a period), half-wave
  symmetry, zero source, independence of the initial iterate.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dft, fem, periodic as pp


def small(n=8, N=8, **kw):
    return fem.discretise(W.with_size(W.Problem(**kw), n, N))


# ---------------------------------------------------------------- DFT

def test_dft_by_definition_matches_library_fft():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((16, 5))
    assert np.allclose(dft.dft(X), np.fft.fft(X, axis=0), atol=1e-12)
    P = dft.rfft_packed(X)
    R = np.fft.rfft(X, axis=0)
    assert np.allclose(P[1:], R[1:8], atol=1e-12)
    assert np.allclose(P[0].real, R[0].real) and np.allclose(P[0].imag, R[8].real)
    assert np.allclose(dft.irfft_packed(P, 16), X, atol=1e-13)


def test_shift_symbols():
    z = dft.shifts(8, 0.125)
    assert z[0] == 0
    assert abs(z[4] - 16.0) < 1e-12           # z_{N/2} = 2 / tau
    assert np.all(z.real >= 0)
    assert np.all(z[1:4].imag > 0)


def test_periodic_operator_is_dft_diagonal():
    d = small(8, 16)
    rng = np.random.default_rng(1)
    U = rng.standard_normal((16, d.nfree))
    PU = pp.apply_P(d, U)
    # assembled matrix agrees with the matrix-free product
    assert np.allclose((pp.spacetime_matrix(d) @ U.reshape(-1)).reshape(U.shape), PU, atol=1e-12)
    Uh = np.fft.fft(U, axis=0)
    N, tau = d.p.N, d.p.tau
    z = (1 - np.exp(-2j * np.pi * np.arange(N) / N)) / tau
    Yh = np.stack([d.Khat @ Uh[k] + z[k] * (d.M @ Uh[k]) for k in range(N)])
    assert np.allclose(np.fft.ifft(Yh, axis=0).real, PU, atol=1e-11)
    # k = 0 block is the static problem with Khat only
    assert np.allclose(Yh[0], d.Khat @ Uh[0])


def test_single_mode_closed_form():
    # nu = nu_max everywhere: K = Khat, the fixed point converges in one step and the
    # periodic solution of the sin source has DFT support on k = 1 and N-1 only.
    p = W.Problem(n=8, N=16, nu_a=10.0, nu_b=0.0, nu_out=10.0)
    d = fem.discretise(p)
    r = pp.fixed_point(d, tol=1e-13, max_iter=3)
    assert r.iters == 1 and r.converged
    Uh = np.fft.fft(r.U, axis=0)
    mag = np.linalg.norm(Uh, axis=1)
    assert np.all(mag[[0] + list(range(2, 15))] < 1e-12 * mag[1])
    N, tau = p.N, p.tau
    z1 = (1 - np.exp(-2j * np.pi / N)) / tau
    bh1 = np.fft.fft(pp.load_series(d), axis=0)[1]
    A = (d.Khat + z1 * d.M).toarray()
    assert np.allclose(Uh[1], np.linalg.solve(A, bh1), rtol=1e-11, atol=1e-14)


def test_load_series_samples_the_new_time_level():
    # Problem 1 evaluates f^n at t_n = n tau, n = 1..N, and row j of the series holds f^{j+1}.
    # With N divisible by 4 the sin source takes closed values at quarter periods:
    # f^{N/4} = b (t = T/4), f^{N/2} = 0 (t = T/2), f^{3N/4} = -b, f^N = 0 (t = T); the cos
    # source has f^N = b and f^{N/2} = -b. Sampling at t_{n-1} instead would give
    # sin(2 pi (N/4 - 1)/N) b in row N/4 - 1 and b in row 0 of the cos series.
    for T in (1.0, 0.02):
        d = small(8, 16, T=T)
        b = d.b
        N = d.p.N
        assert np.linalg.norm(b) > 0
        F = pp.load_series(d)
        assert F.shape == (N, d.nfree)
        tol = 1e-15 * np.max(np.abs(b))
        assert np.max(np.abs(F[N // 4 - 1] - b)) <= tol
        assert np.max(np.abs(F[N // 2 - 1])) <= 1e-14 * np.max(np.abs(b))
        assert np.max(np.abs(F[3 * N // 4 - 1] + b)) <= tol
        assert np.max(np.abs(F[N - 1])) <= 1e-14 * np.max(np.abs(b))
        # the first row is the source one step into the period
        assert np.allclose(F[0], np.sin(2 * np.pi / N) * b, rtol=0, atol=tol)
        C = pp.load_series(d, "cos")
        assert np.max(np.abs(C[N - 1] - b)) <= tol
        assert np.max(np.abs(C[N // 2 - 1] + b)) <= tol
        assert np.max(np.abs(C[N // 4 - 1])) <= 1e-14 * np.max(np.abs(b))
        assert np.allclose(C[0], np.cos(2 * np.pi / N) * b, rtol=0, atol=tol)


def test_period_sweep_solver_matches_spacetime_lu():
    d = small(8, 8)
    rng = np.random.default_rng(3)
    R = rng.standard_normal((8, d.nfree))
    a = pp.SpaceTimeLU(d).solve(R)
    b = pp.PeriodSweepLU(d).solve(R)
    assert np.allclose(a, b, atol=1e-12)
    assert np.allclose(pp.apply_P(d, a), R, atol=1e-11)


# ---------------------------------------------------------------- fixed point

def test_closed_form_rate_without_conductivity():
    # sigma = 0, nu = c: each slice is Khat-preconditioned Richardson on c S, error x (1 - c/nu_max).
    c = 2.5
    p = W.Problem(n=8, N=8, sigma_in=0.0, nu_a=c, nu_b=0.0, nu_out=c)
    d = fem.discretise(p)
    r = pp.fixed_point(d, tol=1e-9, max_iter=400)
    ratios = np.array(r.rel[1:]) / np.array(r.rel[:-1])
    assert len(ratios) > 50
    assert np.allclose(ratios, 1 - c / p.nu_max, rtol=1e-7)


def test_contraction_in_khat_norm_every_step():
    # Theorem thm:iter, eq. (q): ||U^{k+1} - U||_Khat <= q ||U^k - U||_Khat with q = 0.9.
    p = W.with_size(W.config1(), 16, 16)
    d = fem.discretise(p)
    ref = pp.fixed_point(d, tol=1e-14, max_iter=600)
    lin = pp.SpaceTimeLU(d)
    U = np.zeros_like(ref.U)
    F = pp.load_series(d)
    errs = [pp.khat_norm(d, U - ref.U)]
    for _ in range(60):
        U = U + lin.solve(pp.residual(d, U, F))
        errs.append(pp.khat_norm(d, U - ref.U))
    ratios = np.array(errs[1:]) / np.array(errs[:-1])
    assert np.all(ratios <= 0.9 + 1e-9)


@pytest.mark.slow
def test_rate_independent_of_h_and_tau():
    # Phi is a q-contraction in the Khat-norm, so successive steps shrink by <= q = 0.9
    # at every iteration; the observed residual rate is the same on every grid.
    rates = []
    for n, N in [(8, 8), (16, 16), (32, 8), (8, 32), (32, 32)]:
        d = fem.discretise(W.with_size(W.config1(), n, N))
        r = pp.fixed_point(d, tol=1e-9, max_iter=500)
        steps = np.array(r.khat_step)
        assert np.all(steps[1:] / steps[:-1] <= 0.9 + 1e-9)
        rel = np.array(r.rel)
        rates.append((rel[-1] / rel[-21]) ** (1 / 20))
    rates = np.array(rates)
    assert np.all(np.abs(rates - 0.9) <= 0.01)
    assert rates.max() - rates.min() <= 0.02


# ---------------------------------------------------------------- final solution

def manufactured(d, seed=0):
    a, b, c = W.manufactured_coeffs(seed)
    p = d.p
    t = p.tau * np.arange(1, p.N + 1)
    prof = a + b * np.cos(2 * np.pi * t / p.T) + c * np.sin(4 * np.pi * t / p.T)
    xy = d.mesh.xy[d.free_idx]
    space = np.sin(np.pi * xy[:, 0]) * np.sin(np.pi * xy[:, 1])
    return prof[:, None] * space[None, :] * 5.0


def test_manufactured_discrete_solution():
    d = fem.discretise(W.with_size(W.config1(), 16, 16))
    Ustar = manufactured(d)
    F = pp.apply_A(d, Ustar)
    r = pp.fixed_point(d, tol=1e-13, max_iter=800, F=F)
    assert r.converged
    assert np.linalg.norm(r.U - Ustar) <= 1e-10 * np.linalg.norm(Ustar)


def test_newton_agrees_with_fixed_point():
    d = fem.discretise(W.with_size(W.Problem(J0=60.0), 8, 8))
    fp = pp.fixed_point(d, tol=1e-14, max_iter=800)
    Un, hist = pp.newton(d, tol=1e-14)
    assert hist[-1] <= 1e-14 * 10
    assert np.linalg.norm(Un - fp.U) <= 1e-12 * np.linalg.norm(fp.U)
    # Newton converges quadratically near the solution
    h = np.array(hist)
    tail = h[h > 1e-13]
    if len(tail) >= 3:
        assert tail[-1] <= 10 * tail[-2] ** 1.5


def test_time_stepping_reaches_the_periodic_solution():
    d = fem.discretise(W.with_size(W.config1(), 8, 16))
    fp = pp.fixed_point(d, tol=1e-13, max_iter=800)
    last = pp.time_stepping(d, periods=4)
    assert np.linalg.norm(last - fp.U) <= 1e-9 * np.linalg.norm(fp.U)
    # wrap-around: one implicit-Euler step from u^N reproduces u^1
    first = pp.time_stepping(d, periods=1, u_start=fp.U[-1])
    assert np.linalg.norm(first[0] - fp.U[0]) <= 1e-10 * np.linalg.norm(fp.U[0])


def test_energy_balance_over_a_period():
    # tau sum_n ||d_tau u^n||_M^2 = 2 sum_n <f^n - K(u^n), u^n>
    d = fem.discretise(W.with_size(W.config1(), 16, 16))
    r = pp.fixed_point(d, tol=1e-13, max_iter=800)
    U, F = r.U, r.F
    tau = d.p.tau
    dU = (U - np.roll(U, 1, axis=0)) / tau
    lhs = tau * np.sum(dU * (d.M @ dU.T).T)
    rhs = 2 * np.sum((F - pp.K_free(d, U)) * U)
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)
    assert lhs > 0


def test_half_wave_symmetry():
    # sin source: f^{n+N/2} = -f^n and K is odd, so uniqueness gives u^{n+N/2} = -u^n.
    d = fem.discretise(W.with_size(W.config1(), 16, 16))
    r = pp.fixed_point(d, tol=1e-13, max_iter=800)
    U = r.U
    assert np.linalg.norm(U[8:] + U[:8]) <= 1e-11 * np.linalg.norm(U)


def test_zero_source_gives_zero_and_initial_guess_does_not_matter():
    d = fem.discretise(W.with_size(W.config1(), 8, 8))
    F0 = np.zeros((8, d.nfree))
    rng = np.random.default_rng(4)
    r0 = pp.fixed_point(d, tol=1e-12, F=F0, U0=rng.standard_normal((8, d.nfree)), max_iter=600)
    assert np.linalg.norm(r0.U) < 1e-8
    a = pp.fixed_point(d, tol=1e-13, max_iter=800)
    b = pp.fixed_point(d, tol=1e-13, max_iter=800, U0=rng.standard_normal((8, d.nfree)))
    assert np.linalg.norm(a.U - b.U) <= 1e-11 * np.linalg.norm(a.U)
