"""P1 finite elements on a uniform triangulation of the unit square (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Discretisation of the magneto-quasistatic model of Sec. 4 ("Test problem"):
    sigma du/dt - div(nu(|grad u|) grad u) = j  in Omega,  u = 0 on the boundary,
with piecewise linear finite elements in space ("Simulation setup", Sec. 4).

Mesh convention: nodes (i h, j h), i, j = 0..n, id = j (n+1) + i. Cell (i, j) is
split along its SW-NE diagonal into T_a = {(i,j), (i+1,j), (i+1,j+1)} and
T_b = {(i,j), (i+1,j+1), (i,j+1)}; triangle id = 2 (j n + i) + {0 for T_a, 1 for T_b}.
A triangle belongs to a region rectangle iff its centroid lies in the closed
rectangle; the centroid coordinates are computed as (3 i + 2) / (3 n) etc. in
float64 so that membership is reproducible bit for bit.

Everything below is written for general triangles (gradients from vertex
coordinates), not for the structured stencil; the structured closed forms are
test pins.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from workloads import Problem


@dataclass
class Mesh:
    n: int
    h: float
    xy: np.ndarray        # (nodes, 2) coordinates
    tri: np.ndarray       # (ntri, 3) node ids
    area: np.ndarray      # (ntri,)
    grad: np.ndarray      # (ntri, 3, 2) gradients of the three barycentric functions
    centroid: np.ndarray  # (ntri, 2)
    free: np.ndarray      # (nodes,) bool, interior nodes

    @property
    def nodes(self) -> int:
        return self.xy.shape[0]


def build_mesh(n: int) -> Mesh:
    h = 1.0 / n
    jj, ii = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    xy = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1)

    def nid(i, j):
        return j * (n + 1) + i

    cj, ci = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ci = ci.ravel()
    cj = cj.ravel()
    ta = np.stack([nid(ci, cj), nid(ci + 1, cj), nid(ci + 1, cj + 1)], axis=1)
    tb = np.stack([nid(ci, cj), nid(ci + 1, cj + 1), nid(ci, cj + 1)], axis=1)
    tri = np.empty((2 * n * n, 3), dtype=np.int64)
    tri[0::2] = ta
    tri[1::2] = tb

    # Exact centroids: T_a ((i+2/3)h, (j+1/3)h), T_b ((i+1/3)h, (j+2/3)h).
    cen = np.empty((2 * n * n, 2))
    cen[0::2, 0] = (3 * ci + 2) / (3.0 * n)
    cen[0::2, 1] = (3 * cj + 1) / (3.0 * n)
    cen[1::2, 0] = (3 * ci + 1) / (3.0 * n)
    cen[1::2, 1] = (3 * cj + 2) / (3.0 * n)

    p = xy[tri]                               # (ntri, 3, 2)
    e1 = p[:, 1] - p[:, 0]
    e2 = p[:, 2] - p[:, 0]
    det = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
    area = 0.5 * np.abs(det)
    # grad(phi_a) = rot(p_c - p_b) / det for the cyclic order (a, b, c)
    grad = np.empty((tri.shape[0], 3, 2))
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        d = p[:, c] - p[:, b]
        grad[:, a, 0] = -d[:, 1] / det
        grad[:, a, 1] = d[:, 0] / det

    free = np.zeros((n + 1, n + 1), dtype=bool)
    free[1:-1, 1:-1] = True
    return Mesh(n=n, h=h, xy=xy, tri=tri, area=area, grad=grad, centroid=cen, free=free.ravel())


def in_rect(cen: np.ndarray, r) -> np.ndarray:
    x0, y0, x1, y1 = r.as_tuple()
    return (cen[:, 0] >= x0) & (cen[:, 0] <= x1) & (cen[:, 1] >= y0) & (cen[:, 1] <= y1)


@dataclass
class Materials:
    sigma: np.ndarray     # (ntri,)
    iron: np.ndarray      # (ntri,) bool: nonlinear law applies
    theta: np.ndarray     # (ntri,) nu scale
    J: np.ndarray         # (ntri,) current density amplitude
    # Region mode: the law and its per-triangle parameters (None: the rectangle problem's law,
    # nu_a + nu_b s^2/(1+s^2) in iron and nu_out elsewhere, from the Problem)
    law: str = "rational"
    a: np.ndarray = None
    b: np.ndarray = None
    c: np.ndarray = None
    d: np.ndarray = None


def materials(p: Problem, m: Mesh) -> Materials:
    ntri = m.tri.shape[0]
    theta = np.ones(ntri) if p.theta is None else np.asarray(p.theta, dtype=np.float64)
    if theta.shape != (ntri,):
        raise ValueError("theta must have one entry per triangle")
    if p.regions is not None:
        # region mode (Sec. 4, "Test problem": sigma, the law and j piecewise constant per region)
        from workloads import region_ids
        rid = region_ids(p).astype(np.int64)
        tab = lambda f: np.array([getattr(r, f) for r in p.regions], dtype=np.float64)[rid]
        a = tab("a")
        return Materials(sigma=tab("sigma"), iron=a != 0.0, theta=theta, J=tab("j"), law=p.law,
                         a=a, b=tab("b"), c=tab("c"), d=tab("d"))
    sigma = np.where(in_rect(m.centroid, p.sigma_rect), p.sigma_in, 0.0)
    iron = in_rect(m.centroid, p.nu_rect)
    J = np.where(in_rect(m.centroid, p.coil_rect), p.J0, 0.0)
    return Materials(sigma=sigma, iron=iron, theta=theta, J=J)


def _assemble(m: Mesh, local: np.ndarray) -> sp.csr_matrix:
    """Sum element matrices local[t, a, b] into a global sparse matrix (all nodes)."""
    rows = np.repeat(m.tri, 3, axis=1).ravel()
    cols = np.tile(m.tri, (1, 3)).ravel()
    A = sp.coo_matrix((local.ravel(), (rows, cols)), shape=(m.nodes, m.nodes))
    return A.tocsr()


def stiffness_full(m: Mesh, coef: np.ndarray | float = 1.0) -> sp.csr_matrix:
    """P1 stiffness int coef grad(phi_b) . grad(phi_a), all nodes."""
    coef = np.broadcast_to(np.asarray(coef, dtype=np.float64), m.area.shape)
    local = np.einsum("t,tad,tbd->tab", coef * m.area, m.grad, m.grad)
    return _assemble(m, local)


def mass_full(m: Mesh, sigma: np.ndarray) -> sp.csr_matrix:
    """Consistent P1 mass int sigma phi_b phi_a: |T|/12 [[2,1,1],[1,2,1],[1,1,2]] per triangle."""
    ref = (np.ones((3, 3)) + np.eye(3)) / 12.0
    local = (sigma * m.area)[:, None, None] * ref[None]
    return _assemble(m, local)


def load_full(m: Mesh, J: np.ndarray) -> np.ndarray:
    """Exact integral of the piecewise-constant J against each hat function: |T|/3 per vertex."""
    b = np.zeros(m.nodes)
    np.add.at(b, m.tri.ravel(), np.repeat(J * m.area / 3.0, 3))
    return b


def restrict(A: sp.spmatrix, free: np.ndarray) -> sp.csr_matrix:
    idx = np.flatnonzero(free)
    return A.tocsr()[idx][:, idx].tocsr()


# ---------------------------------------------------------------- nonlinear law

def _saturation(mat: Materials) -> np.ndarray:
    """s^2 at which exp(b s^2) reaches c (the exp-capped law saturates beyond it): ln(c)/b,
    +inf where b = 0 (the law is the constant a + d there)."""
    with np.errstate(divide="ignore"):
        return np.where(mat.b > 0, np.log(mat.c) / np.where(mat.b > 0, mat.b, 1.0), np.inf)


def nu_of_s2(s2: np.ndarray, mat: Materials, p: Problem) -> np.ndarray:
    """Reluctivity per triangle, theta times
    rectangle problems:  nu_a + nu_b s^2/(1+s^2) in iron, nu_out elsewhere;
    region "rational":   a + b s^2/(1+s^2);
    region "expcap":     a min(exp(b s^2), c) + d (the law of Sec. 4)."""
    if mat.a is None:
        inside = p.nu_a + p.nu_b * s2 / (1.0 + s2)
        return mat.theta * np.where(mat.iron, inside, p.nu_out)
    if mat.law == "rational":
        return mat.theta * (mat.a + mat.b * s2 / (1.0 + s2))
    z = np.minimum(s2, _saturation(mat))
    return mat.theta * (mat.a * np.minimum(np.exp(mat.b * z), mat.c) + mat.d)


def dnu_ds2(s2: np.ndarray, mat: Materials, p: Problem) -> np.ndarray:
    """d nu / d(s^2): theta nu_b / (1+s^2)^2 in iron (rectangle problems), theta b / (1+s^2)^2
    (region "rational"), theta a b exp(b s^2) below saturation and 0 from it on (region "expcap",
    the right derivative at the kink)."""
    if mat.a is None:
        return mat.theta * np.where(mat.iron, p.nu_b / (1.0 + s2) ** 2, 0.0)
    if mat.law == "rational":
        return mat.theta * mat.b / (1.0 + s2) ** 2
    below = s2 < _saturation(mat)
    z = np.where(below, s2, 0.0)
    return mat.theta * np.where(below, mat.a * mat.b * np.exp(mat.b * z), 0.0)


def energy_density(s2: np.ndarray, mat: Materials, p: Problem) -> np.ndarray:
    """W(s^2) with dW/d(s^2) = nu/2, W(0) = 0:
    rectangle problems:  theta ((a+b) s^2/2 - (b/2) ln(1+s^2)) in iron, theta nu_out s^2/2 elsewhere;
    region "rational":   theta ((a+b) s^2/2 - (b/2) ln(1+s^2));
    region "expcap":     theta (d s^2 + a (exp(b z) - 1)/b + a c (s^2 - z)) / 2, z = min(s^2, ln(c)/b)
                         (a s^2/2 in place of the exp term where b = 0)."""
    if mat.a is None:
        inside = 0.5 * (p.nu_a + p.nu_b) * s2 - 0.5 * p.nu_b * np.log1p(s2)
        return mat.theta * np.where(mat.iron, inside, 0.5 * p.nu_out * s2)
    if mat.law == "rational":
        return mat.theta * (0.5 * (mat.a + mat.b) * s2 - 0.5 * mat.b * np.log1p(s2))
    zs = _saturation(mat)
    z = np.minimum(s2, zs)
    bpos = mat.b > 0
    bb = np.where(bpos, mat.b, 1.0)
    expint = np.where(bpos, np.expm1(bb * np.where(bpos, z, 0.0)) / bb, z)   # int_0^z exp(b t) dt
    cap = np.where(np.isfinite(zs), mat.c * (s2 - z), 0.0)     # int_z^s2 c dt
    return mat.theta * 0.5 * (mat.d * s2 + mat.a * (expint + cap))


def gradients(m: Mesh, U: np.ndarray) -> np.ndarray:
    """Elementwise constant gradient of u: U (..., nodes) -> (..., ntri, 2)."""
    uv = U[..., m.tri]                                   # (..., ntri, 3)
    return np.einsum("...ta,tad->...td", uv, m.grad)


def apply_K(p: Problem, m: Mesh, mat: Materials, U: np.ndarray) -> np.ndarray:
    """K(u)_i = sum over T containing i of |T| nu_T(|grad u_T|^2) grad u_T . grad phi_i.

    U has shape (..., nodes); the result is over all nodes (boundary rows included,
    the caller restricts to free nodes)."""
    g = gradients(m, U)
    s2 = np.einsum("...td,...td->...t", g, g)
    nu = nu_of_s2(s2, mat, p)
    flux = (nu * m.area)[..., None] * g                  # (..., ntri, 2)
    loc = np.einsum("...td,tad->...ta", flux, m.grad)    # (..., ntri, 3)
    out = np.zeros(U.shape)
    lead = U.shape[:-1]
    flat_out = out.reshape(-1, m.nodes)
    flat_loc = loc.reshape(-1, m.tri.shape[0] * 3)
    idx = m.tri.ravel()
    for r in range(flat_out.shape[0]):
        flat_out[r] = np.bincount(idx, weights=flat_loc[r], minlength=m.nodes)
    return flat_out.reshape(lead + (m.nodes,))


def energy(p: Problem, m: Mesh, mat: Materials, u: np.ndarray) -> float:
    """E(u) = sum_T |T| W(|grad u_T|^2); its gradient is K(u)."""
    g = gradients(m, u)
    s2 = np.einsum("td,td->t", g, g)
    return float(np.sum(m.area * energy_density(s2, mat, p)))


def jacobian_K(p: Problem, m: Mesh, mat: Materials, u: np.ndarray) -> sp.csr_matrix:
    """K'(u): per triangle |T| grad phi_a . (nu I + 2 nu'(s^2) g g^T) grad phi_b, all nodes."""
    g = gradients(m, u)
    s2 = np.einsum("td,td->t", g, g)
    nu = nu_of_s2(s2, mat, p)
    dnu = dnu_ds2(s2, mat, p)
    ten = nu[:, None, None] * np.eye(2)[None] + 2.0 * dnu[:, None, None] * g[:, :, None] * g[:, None, :]
    local = np.einsum("t,tad,tde,tbe->tab", m.area, m.grad, ten, m.grad)
    return _assemble(m, local)


@dataclass
class Discretisation:
    """All time-invariant pieces of the discrete problem, restricted to free nodes where noted."""
    p: Problem
    mesh: Mesh
    mat: Materials
    S: sp.csr_matrix      # free x free, unit-coefficient stiffness
    M: sp.csr_matrix      # free x free, sigma mass
    b: np.ndarray         # free, load amplitude
    free_idx: np.ndarray
    # per-triangle coefficient of Khat (None: Khat = nu_max S, the constant coefficient)
    khat_coef: np.ndarray = None

    @property
    def Khat(self) -> sp.csr_matrix:
        """The linear operator of eqs. (iter1)-(iter2): nu_max S, or the stiffness with the
        per-triangle coefficient khat_coef (a per-region choice in the family of Thm. thm:iter)."""
        if self.khat_coef is not None:
            return restrict(stiffness_full(self.mesh, self.khat_coef), self.mesh.free)
        return (self.p.nu_max * self.S).tocsr()

    @property
    def nfree(self) -> int:
        return self.free_idx.size


def discretise(p: Problem) -> Discretisation:
    m = build_mesh(p.n)
    mat = materials(p, m)
    S = restrict(stiffness_full(m), m.free)
    M = restrict(mass_full(m, mat.sigma), m.free)
    b = load_full(m, mat.J)[m.free]
    d = Discretisation(p=p, mesh=m, mat=mat, S=S, M=M, b=b, free_idx=np.flatnonzero(m.free))
    if p.regions is not None and any(r.nu_hat > 0 for r in p.regions):
        # Khat with a coefficient per region (Thm. thm:iter: any such Khat whose coefficient
        # bounds the law suitably); a region without one takes nu_max
        from workloads import region_ids
        coef = np.array([r.nu_hat if r.nu_hat > 0 else p.nu_max for r in p.regions], dtype=np.float64)
        d.khat_coef = coef[region_ids(p).astype(np.int64)]
    return d
