"""Seeded, synthetic problem descriptions for the time-periodic eddy-current problem.

This module is the only code shared by the CPU oracle and the GPU path. It holds
problem *descriptions* (geometry rectangles, material-law parameters, source
amplitude, grid and time sizes) and seeded random draws. It contains none of the
method's arithmetic: no mesh, no assembly, no operator, no solver.

The problem (Sec. 4 of the paper, "Test problem"): find the z-component u of the
magnetic vector potential on the unit square with u = 0 on the boundary and

    sigma * du/dt - div(nu(|grad u|) grad u) = j,   T-periodic in time,

discretised by P1 finite elements on a uniform grid (each square split along the
SW-NE diagonal) and by implicit Euler with N steps per period (Problem 1,
eqs. (disc1)-(disc2)). The synthetic stand-in for the paper's transformer
cross-section keeps its structure: a nonlinear iron region, a current-driven coil
strip and a conducting block where sigma > 0 (sigma = 0 elsewhere, so the mass
operator is degenerate, assumption (A2)).

Material law inside the iron rectangle:  nu(s) = theta * (nu_a + nu_b s^2/(1+s^2)),
outside:                                   nu(s) = theta * nu_out,
where theta is an optional per-triangle scale (1 by default).
Source: f(x, t) = J0 * w(2 pi t / T) on the coil rectangle, w = sin (or cos).
Linear part of the fixed-point iteration: Khat = nu_max * (P1 stiffness).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Rect", "Region", "Problem", "config1", "config2", "config3", "config4", "config5", "transformer",
    "region_ids", "with_size", "random_field", "manufactured_coeffs", "CONFIG1_TOL",
]


@dataclass(frozen=True)
class Rect:
    """Closed axis-aligned rectangle [x0, x1] x [y0, y1]."""
    x0: float
    y0: float
    x1: float
    y1: float

    def as_tuple(self) -> Tuple[float, float, float, float]:
        return (self.x0, self.y0, self.x1, self.y1)


@dataclass(frozen=True)
class Region:
    """Material of one region of a cross-section (Sec. 4, table tab:coef): conductivity sigma,
    parameters a, b, c, d of the reluctivity law and current-density amplitude j, and the
    region's coefficient nu_hat of the iteration's linear operator Khat (0: the problem's
    nu_max)."""
    name: str
    sigma: float = 0.0
    a: float = 0.0
    b: float = 0.0
    c: float = 1.0
    d: float = 1.0
    j: float = 0.0
    nu_hat: float = 0.0


@dataclass(frozen=True)
class Problem:
    """Description of one time-periodic problem instance.

    Grid: n x n square cells of side h = 1/n on the unit square, (n+1)^2 nodes.
    Time: N implicit-Euler steps per period T, tau = T/N, t_n = n tau, n = 1..N.
    """
    n: int = 32
    N: int = 32
    T: float = 1.0
    sigma_in: float = 1.0
    sigma_rect: Rect = Rect(0.25, 0.25, 0.75, 0.75)
    nu_a: float = 1.0
    nu_b: float = 9.0
    nu_out: float = 1.0
    nu_rect: Rect = Rect(0.3, 0.05, 0.7, 0.95)
    J0: float = 10.0
    coil_rect: Rect = Rect(0.1, 0.3, 0.2, 0.7)
    waveform: str = "sin"        # "sin" or "cos"
    nu_max: float = 10.0
    # Optional per-triangle nu scale theta (length 2 n^2, ordering tri = 2 (j n + i) + {0, 1}).
    theta: Optional[np.ndarray] = field(default=None, compare=False, repr=False)
    # Region mode (when `regions` is set): the rectangles above are not used; each triangle
    # belongs to the region of the last rectangle of `layout` containing its centroid, and takes
    # that region's conductivity, current amplitude and law parameters. `law` selects the
    # reluctivity law of every region: "rational" nu = a + b s^2/(1+s^2), "expcap"
    # nu = a min(exp(b s^2), c) + d (the law of Sec. 4).
    law: str = "rational"
    regions: Optional[Tuple[Region, ...]] = None
    layout: Optional[Tuple[Tuple[Rect, int], ...]] = None

    @property
    def tau(self) -> float:
        return self.T / self.N

    @property
    def nodes(self) -> int:
        return (self.n + 1) ** 2

    @property
    def free_nodes(self) -> int:
        return (self.n - 1) ** 2

    @property
    def st_dofs(self) -> int:
        """Space-time degrees of freedom: free nodes times time slices."""
        return self.free_nodes * self.N


CONFIG1_TOL = 1e-10


def config1() -> Problem:
    """Plain method, FP64, small: 32 x 32 cells, N = 32, J0 = 10, unjittered iron block."""
    return Problem(n=32, N=32)


def _seeded_materials(seed: int) -> Tuple[float, Rect]:
    """Draw order: J0 = 10**U(0, 2), then a U(-0.05, 0.05) jitter of the four iron
    rectangle coordinates (x0, y0, x1, y1)."""
    rng = np.random.default_rng(seed)
    J0 = float(10.0 ** rng.uniform(0.0, 2.0))
    jit = rng.uniform(-0.05, 0.05, 4)
    base = Rect(0.3, 0.05, 0.7, 0.95)
    iron = Rect(base.x0 + jit[0], base.y0 + jit[1], base.x1 + jit[2], base.y1 + jit[3])
    return J0, iron


def config2(seed: int = 0) -> Problem:
    """256 x 256 cells (66,049 nodes), N = 256, seeded J0 and iron jitter."""
    J0, iron = _seeded_materials(seed)
    return Problem(n=256, N=256, J0=J0, nu_rect=iron)


def config3(seed: Optional[int] = 0) -> Problem:
    """1024 x 1024 cells (1,050,625 nodes), N = 512. seed=None gives the unjittered J0 = 10 case."""
    if seed is None:
        return Problem(n=1024, N=512)
    J0, iron = _seeded_materials(seed)
    return Problem(n=1024, N=512, J0=J0, nu_rect=iron)


def config4(seed: int = 0, count: int = 64) -> List[Problem]:
    """Batch of independent instances: n from {64,128,256,512}, N from {64,128,256},
    J0 log-uniform in [1, 100], iron rectangle with random corners inside [0.2, 0.8]^2."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice([64, 128, 256, 512]))
        N = int(rng.choice([64, 128, 256]))
        J0 = float(10.0 ** rng.uniform(0.0, 2.0))
        xs = np.sort(rng.uniform(0.2, 0.8, 2))
        ys = np.sort(rng.uniform(0.2, 0.8, 2))
        out.append(Problem(n=n, N=N, J0=J0, nu_rect=Rect(xs[0], ys[0], xs[1], ys[1])))
    return out


def config5(seed: int = 0, n: int = 256, N: int = 256) -> Problem:
    """Differentiation-mode instance: per-triangle log-normal nu scale with sd 0.1
    (constant on each square cell, so one value per cell, repeated for its two triangles)."""
    rng = np.random.default_rng(seed)
    cell = np.exp(rng.normal(0.0, 0.1, n * n))
    theta = np.repeat(cell, 2)
    return Problem(n=n, N=N, theta=theta)


def region_ids(p: Problem) -> np.ndarray:
    """Region of every triangle (uint8, ordering tri = 2 (j n + i) + {0, 1}) of a region-mode
    problem: the last rectangle of p.layout that contains the triangle's centroid (closed
    rectangles; centroids ((3i+2)/(3n), (3j+1)/(3n)) for T_a and ((3i+1)/(3n), (3j+2)/(3n)) for
    T_b). The first layout entry must cover the whole square."""
    if p.regions is None or p.layout is None:
        raise ValueError("not a region-mode problem")
    n = p.n
    cj, ci = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ci, cj = ci.ravel(), cj.ravel()
    cx = np.empty(2 * n * n)
    cy = np.empty(2 * n * n)
    cx[0::2] = (3 * ci + 2) / (3.0 * n)
    cy[0::2] = (3 * cj + 1) / (3.0 * n)
    cx[1::2] = (3 * ci + 1) / (3.0 * n)
    cy[1::2] = (3 * cj + 2) / (3.0 * n)
    rid = np.full(2 * n * n, 255, dtype=np.uint8)
    for r, k in p.layout:
        inside = (cx >= r.x0) & (cx <= r.x1) & (cy >= r.y0) & (cy <= r.y1)
        rid[inside] = k
    if np.any(rid == 255):
        raise ValueError("the layout does not cover every triangle")
    return rid


# Transformer cross-section of Sec. 4 (figure fig:domain, table tab:coef): a 355 mm x 466 mm
# tank whose 10 mm steel wall encloses air, an iron core [60, 295] x [28, 438] mm with the window
# [140, 215] x [108, 358] mm, and four windings 13 mm x 220 mm starting at y = 123 mm, at
# x = 28 and 183 mm (winding-) and x = 159 and 314 mm (winding+).
TRANSFORMER_MM = (355.0, 466.0)
TRANSFORMER_REGIONS = (
    Region("air", sigma=0.0, a=0.0, b=0.0, c=1.0, d=1e7 / (4.0 * np.pi), j=0.0),
    Region("iron", sigma=0.0, a=5.85, b=2.196, c=136026.0, d=23.15, j=0.0),
    Region("steel", sigma=1e7, a=130.171, b=1.102, c=6112.97, d=43.742, j=0.0),
    Region("winding+", sigma=0.0, a=0.0, b=0.0, c=1.0, d=1e7 / (4.0 * np.pi), j=1.9e4),
    Region("winding-", sigma=0.0, a=0.0, b=0.0, c=1.0, d=1e7 / (4.0 * np.pi), j=-1.9e4),
)


def _mm_rect(x0, y0, x1, y1) -> Rect:
    """A rectangle of the cross-section in mm, its axes scaled independently onto [0, 1]."""
    lx, ly = TRANSFORMER_MM
    return Rect(x0 / lx, y0 / ly, x1 / lx, y1 / ly)


def transformer(n: int = 128, N: int = 64, law: str = "expcap", nu_max: Optional[float] = None,
                j_scale: float = 1.0, khat_factor: Optional[float] = None) -> Problem:
    """The transformer cross-section of Sec. 4 drawn on the unit square (each axis scaled onto
    [0, 1], so the grid stays uniform and square: a transformer-like geometry with the paper's
    layout and materials, not its exact aspect ratio), with the law nu = a min(exp(b s^2), c) + d
    of table tab:coef, T = 0.02 s, the cos source j_i cos(2 pi t / T) (j_i scaled by j_scale) and
    Khat = nu_max S, nu_max = max_i (a_i c_i + d_i) by default (the largest reluctivity the law
    takes). khat_factor: Khat = S_nuhat with nu_hat_i = khat_factor (a_i + d_i) per region
    instead (the law's value at zero field, scaled)."""
    regs = tuple(replace(r, j=r.j * j_scale) for r in TRANSFORMER_REGIONS)
    if khat_factor is not None:
        regs = tuple(replace(r, nu_hat=float(khat_factor) * (r.a + r.d)) for r in regs)
    layout = (
        (Rect(0.0, 0.0, 1.0, 1.0), 2),                 # steel tank wall ...
        (_mm_rect(10, 10, 345, 456), 0),               # ... around the air inside it
        (_mm_rect(60, 28, 295, 438), 1),               # iron core
        (_mm_rect(140, 108, 215, 358), 0),             # core window (air)
        (_mm_rect(28, 123, 41, 343), 4),               # winding-
        (_mm_rect(183, 123, 196, 343), 4),             # winding-
        (_mm_rect(159, 123, 172, 343), 3),             # winding+
        (_mm_rect(314, 123, 327, 343), 3),             # winding+
    )
    if nu_max is None:
        nu_max = max(r.a * r.c + r.d for r in regs)
    return Problem(n=n, N=N, T=0.02, waveform="cos", nu_max=float(nu_max), law=law, regions=regs, layout=layout)


def with_size(p: Problem, n: int, N: int) -> Problem:
    """Same materials and source on another grid / number of time steps."""
    theta = None
    if p.theta is not None:
        if p.n != n:
            raise ValueError("cannot resize a problem with a per-triangle theta field")
        theta = p.theta
    return replace(p, n=n, N=N, theta=theta)


def random_field(N: int, n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded random space-time field U[N, n+1, n+1] (float64) with zero boundary ring."""
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((N, n + 1, n + 1)) * scale
    U[:, 0, :] = 0.0
    U[:, -1, :] = 0.0
    U[:, :, 0] = 0.0
    U[:, :, -1] = 0.0
    return U


def manufactured_coeffs(seed: int = 0) -> Tuple[float, float, float]:
    """Coefficients (a, b, c) of a manufactured discrete solution
    u*(x, y, t) = sin(pi x) sin(pi y) (a + b cos(2 pi t / T) + c sin(4 pi t / T))."""
    rng = np.random.default_rng(seed)
    a, b, c = rng.uniform(0.05, 0.5, 3)
    return float(a), float(b), float(c)
