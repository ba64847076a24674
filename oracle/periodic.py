"""Time-periodic implicit-Euler system and its solvers (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Problem 1 (eqs. (disc1)-(disc2)): find U = (u^1, ..., u^N) with
    M (u^n - u^{n-1}) / tau + K(u^n) = f^n,  n = 1..N,   u^0 = u^N.
Array convention: U[j] holds u^{j+1}, so U[N-1] = u^N = u^0. Vectors live on the
free (interior) nodes unless a function says otherwise.

Fixed-point iteration (eqs. (iter1)-(iter2)) with the linear operator Khat:
    M d_tau u^{n,k+1} + Khat u^{n,k+1} = f^n + Khat u^{n,k} - K(u^{n,k}),  u^{0,k+1} = u^{N,k+1}.
Written with P = I_N (x) (M/tau + Khat) - C_N (x) (M/tau), C_N the cyclic shift
(C_N)[n, n-1] = 1, the iteration reads P U^{k+1} = F + P U^k - A(U^k), because
P U^k - A(U^k) = Khat U^k - K(U^k) (the mass terms cancel). That is the
correction form U^{k+1} = U^k + P^{-1} (F - A(U^k)) used here.

Stopping rule (Sec. 4, "Initialization"): ||F - A(U^k)||_2 <= tol ||F - A(U^0)||_2;
with U^0 = 0 the denominator is ||F||_2 because K(0) = 0.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads import Problem
from . import fem


# ------------------------------------------------------------------ data

def load_series(d: fem.Discretisation, waveform: Optional[str] = None) -> np.ndarray:
    """F[j] = w(2 pi t_{j+1} / T) b with t_n = n tau (source sampled at the new time level)."""
    p = d.p
    w = waveform or p.waveform
    t = p.tau * np.arange(1, p.N + 1)
    phase = 2.0 * np.pi * t / p.T
    s = np.sin(phase) if w == "sin" else np.cos(phase)
    return s[:, None] * d.b[None, :]


def to_full(d: fem.Discretisation, Uf: np.ndarray) -> np.ndarray:
    """Free-node series (N, nfree) -> full grid (N, n+1, n+1) with zero boundary."""
    n = d.p.n
    out = np.zeros((Uf.shape[0], (n + 1) ** 2))
    out[:, d.free_idx] = Uf
    return out.reshape(Uf.shape[0], n + 1, n + 1)


def to_free(d: fem.Discretisation, Ufull: np.ndarray) -> np.ndarray:
    N = Ufull.shape[0]
    return Ufull.reshape(N, -1)[:, d.free_idx]


def K_free(d: fem.Discretisation, Uf: np.ndarray) -> np.ndarray:
    """K applied slice by slice to free-node vectors (boundary values are zero)."""
    full = np.zeros(Uf.shape[:-1] + (d.mesh.nodes,))
    full[..., d.free_idx] = Uf
    return fem.apply_K(d.p, d.mesh, d.mat, full)[..., d.free_idx]


def apply_A(d: fem.Discretisation, Uf: np.ndarray) -> np.ndarray:
    """A(U)^n = M (u^n - u^{n-1}) / tau + K(u^n), u^0 = u^N."""
    dU = Uf - np.roll(Uf, 1, axis=0)
    return (d.M @ dU.T).T / d.p.tau + K_free(d, Uf)


def residual(d: fem.Discretisation, Uf: np.ndarray, F: np.ndarray) -> np.ndarray:
    return F - apply_A(d, Uf)


# ------------------------------------------------------------------ linear periodic operator

def cyclic_shift(N: int) -> sp.csr_matrix:
    """C_N with (C_N)[n, n-1] = 1 and (C_N)[0, N-1] = 1 (u^0 = u^N)."""
    rows = np.arange(N)
    cols = (rows - 1) % N
    return sp.csr_matrix((np.ones(N), (rows, cols)), shape=(N, N))


def spacetime_matrix(d: fem.Discretisation) -> sp.csc_matrix:
    """P = I_N (x) (M/tau + Khat) - C_N (x) (M/tau), the matrix of eq. (iter1)-(iter2)."""
    N, tau = d.p.N, d.p.tau
    Mt = d.M / tau
    D = (Mt + d.Khat).tocsr()
    P = sp.kron(sp.identity(N, format="csr"), D) - sp.kron(cyclic_shift(N), Mt)
    return P.tocsc()


def apply_P(d: fem.Discretisation, Uf: np.ndarray) -> np.ndarray:
    """P U without assembling P: (M/tau + Khat) u^n - (M/tau) u^{n-1}."""
    tau = d.p.tau
    prev = np.roll(Uf, 1, axis=0)
    return (d.M @ (Uf - prev).T).T / tau + (d.Khat @ Uf.T).T


class SpaceTimeLU:
    """Exact periodic solve by sparse LU of the assembled space-time matrix (oracle A)."""

    def __init__(self, d: fem.Discretisation):
        t0 = time.perf_counter()
        self.d = d
        self.lu = spla.splu(spacetime_matrix(d), permc_spec="COLAMD")
        self.factor_s = time.perf_counter() - t0

    def solve(self, R: np.ndarray) -> np.ndarray:
        N, nf = R.shape
        return self.lu.solve(R.reshape(-1)).reshape(N, nf)


class PeriodSweepLU:
    """Exact periodic solve by one sparse LU of D = M/tau + Khat and period sweeps (oracle B).

    Solves D v^n = r^n + (M/tau) v^{n-1} for n = 1..N, restarting with v^0 := v^N
    until the end-of-period value stops changing. The sweep map is affine with
    linear part B^N, B = D^{-1} M / tau, so it converges for any start."""

    def __init__(self, d: fem.Discretisation, sweep_tol: float = 1e-15, max_sweeps: int = 200):
        t0 = time.perf_counter()
        self.d = d
        self.Mt = (d.M / d.p.tau).tocsr()
        self.lu = spla.splu((self.Mt + d.Khat).tocsc(), permc_spec="COLAMD")
        self.factor_s = time.perf_counter() - t0
        self.sweep_tol = sweep_tol
        self.max_sweeps = max_sweeps
        self.last_sweeps = 0

    def solve(self, R: np.ndarray) -> np.ndarray:
        N, nf = R.shape
        V = np.zeros_like(R)
        vN = np.zeros(nf)
        for s in range(self.max_sweeps):
            prev = vN
            for j in range(N):
                V[j] = self.lu.solve(R[j] + self.Mt @ prev)
                prev = V[j]
            change = np.linalg.norm(V[N - 1] - vN)
            vN = V[N - 1].copy()
            self.last_sweeps = s + 1
            if change <= self.sweep_tol * max(np.linalg.norm(vN), 1e-300):
                break
        return V


# ------------------------------------------------------------------ fixed-point iteration

@dataclass
class FixedPointResult:
    U: np.ndarray                 # (N, nfree)
    rel: List[float]              # ||F - A(U^k)|| / ||F|| for k = 0..iters
    khat_step: List[float]        # ||U^{k+1} - U^k||_Khat
    iters: int
    converged: bool
    factor_s: float
    loop_s: float
    F: np.ndarray = field(repr=False, default=None)


def fixed_point(d: fem.Discretisation, tol: float = 1e-10, max_iter: int = 2000,
                solver: str = "spacetime", U0: Optional[np.ndarray] = None,
                F: Optional[np.ndarray] = None, lin=None, callback=None) -> FixedPointResult:
    """Fixed-point iteration (eqs. (iter1)-(iter2)) with Khat = nu_max S and an exact inner solve.
    callback(k, rel, U), if given, is called after the residual of every iterate U^k (progress
    reports and checkpoints of long runs; it does not change the iteration)."""
    if F is None:
        F = load_series(d)
    if lin is None:
        lin = SpaceTimeLU(d) if solver == "spacetime" else PeriodSweepLU(d)
    U = np.zeros_like(F) if U0 is None else U0.copy()
    fnorm = np.linalg.norm(F)
    Kh = d.Khat
    rels, steps = [], []
    t0 = time.perf_counter()
    converged = False
    k = 0
    while True:
        R = residual(d, U, F)
        rel = np.linalg.norm(R) / fnorm if fnorm > 0 else np.linalg.norm(R)
        rels.append(float(rel))
        if callback is not None:
            callback(k, float(rel), U)
        if not np.isfinite(rel):
            break
        if rel <= tol:
            converged = True
            break
        if k >= max_iter:
            break
        dU = lin.solve(R)
        steps.append(float(np.sqrt(np.sum(dU * (Kh @ dU.T).T))))
        U = U + dU
        k += 1
    return FixedPointResult(U=U, rel=rels, khat_step=steps, iters=k, converged=converged,
                            factor_s=lin.factor_s, loop_s=time.perf_counter() - t0, F=F)


def khat_norm(d: fem.Discretisation, E: np.ndarray) -> float:
    """||E||_Khat = sqrt(sum_n <Khat e^n, e^n>) (norm of Theorem 2, eq. (q))."""
    return float(np.sqrt(np.sum(E * (d.Khat @ E.T).T)))


# ------------------------------------------------------------------ all-at-once Newton (tiny meshes)

def newton(d: fem.Discretisation, tol: float = 1e-14, max_iter: int = 50,
           F: Optional[np.ndarray] = None, U0: Optional[np.ndarray] = None):
    """Newton's method on A(U) = F with the exact space-time Jacobian and Armijo back-tracking
    (the outer loop of method (M2), with a sparse direct solve in place of multigrid in time)."""
    p = d.p
    if F is None:
        F = load_series(d)
    N = p.N
    U = np.zeros_like(F) if U0 is None else U0.copy()
    fnorm = np.linalg.norm(F)
    Mt = (d.M / p.tau).tocsr()
    shift = sp.kron(sp.identity(N), Mt) - sp.kron(cyclic_shift(N), Mt)
    hist = []
    for _ in range(max_iter):
        R = residual(d, U, F)
        r = np.linalg.norm(R)
        hist.append(r / fnorm)
        if r <= tol * fnorm:
            break
        blocks = []
        for j in range(N):
            full = np.zeros(d.mesh.nodes)
            full[d.free_idx] = U[j]
            blocks.append(fem.restrict(fem.jacobian_K(p, d.mesh, d.mat, full), d.mesh.free))
        J = (shift + sp.block_diag(blocks)).tocsc()
        dU = spla.spsolve(J, R.reshape(-1)).reshape(U.shape)
        lam = 1.0
        while lam > 1e-6:
            Un = U + lam * dU
            if np.linalg.norm(residual(d, Un, F)) <= (1 - 1e-4 * lam) * r:
                break
            lam *= 0.5
        U = Un
    return U, hist


# ------------------------------------------------------------------ sequential time stepping (M3)

def time_stepping(d: fem.Discretisation, periods: int, F: Optional[np.ndarray] = None,
                  u_start: Optional[np.ndarray] = None, newton_tol: float = 1e-14):
    """Implicit Euler M (u^n - u^{n-1})/tau + K(u^n) = f^n marched from u^0 over several periods,
    each step solved by Newton with Armijo back-tracking (method (M3)). Returns the last period."""
    p = d.p
    if F is None:
        F = load_series(d)
    N, tau = p.N, p.tau
    Mt = (d.M / tau).tocsr()
    u = np.zeros(d.nfree) if u_start is None else u_start.copy()
    last = np.zeros_like(F)
    for _ in range(periods):
        for j in range(N):
            uprev = u.copy()
            rhs = F[j] + Mt @ uprev

            def res(v):
                return rhs - Mt @ v - K_free(d, v[None])[0]
            r = res(u)
            scale = max(np.linalg.norm(rhs), 1e-300)
            for _ in range(50):
                rn = np.linalg.norm(r)
                if rn <= newton_tol * scale:
                    break
                full = np.zeros(d.mesh.nodes)
                full[d.free_idx] = u
                J = (Mt + fem.restrict(fem.jacobian_K(p, d.mesh, d.mat, full), d.mesh.free)).tocsc()
                du = spla.spsolve(J, r)
                lam = 1.0
                while lam > 1e-6:
                    rt = res(u + lam * du)
                    if np.linalg.norm(rt) <= (1 - 1e-4 * lam) * rn:
                        break
                    lam *= 0.5
                u = u + lam * du
                r = rt
            last[j] = u
    return last
