"""Shared helpers of the GPU parity tests: oracle-side expectations on the time-field layout."""
import sys

import numpy as np

from oracle import dft, fem, periodic as pp


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def full_nodes(d, Uf):
    """(N, nfree) -> (N, n+1, n+1)."""
    return pp.to_full(d, Uf)


def oracle_K_full(d, U):
    """K applied slice by slice to a time field (N, n+1, n+1), zero boundary rows."""
    N = U.shape[0]
    flat = U.reshape(N, -1)
    K = fem.apply_K(d.p, d.mesh, d.mat, flat)
    K[:, ~d.mesh.free] = 0.0
    return K.reshape(U.shape)


def oracle_shifted(d, Xh):
    """y_s = (Khat + z_s M) x_s on the frequency-field layout (nodes, S); slot 0 carries the
    k = 0 system on the real part and the k = N/2 system on the imaginary part."""
    N, tau = d.p.N, d.p.tau
    S = N // 2
    z = dft.shifts(N, tau)
    Y = np.zeros_like(Xh)
    fi = d.free_idx
    Kh, M = d.Khat, d.M
    for s in range(S):
        x = Xh[fi, s]
        if s == 0:
            yr = Kh @ x.real
            yi = Kh @ x.imag + z[N // 2].real * (M @ x.imag)
            Y[fi, 0] = yr + 1j * yi
        else:
            Y[fi, s] = Kh @ x + z[s] * (M @ x)
    return Y


def rel_err(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _prolongation(nc):
    """P1 interpolation from the (nc+1)^2 grid to the (2 nc + 1)^2 grid on the SW-NE split
    (full grids, node id = j * side + i): coarse nodes are copied, edge midpoints (horizontal,
    vertical and the SW-NE diagonal) take the mean of their two coarse ends."""
    import scipy.sparse as sp
    sc, nf = nc + 1, 2 * nc
    sf = nf + 1
    rows, cols, vals = [], [], []
    for j in range(sf):
        for i in range(sf):
            a = j * sf + i
            hi, hj = i // 2, j // 2
            if i % 2 == 0 and j % 2 == 0:
                rows.append(a), cols.append(hj * sc + hi), vals.append(1.0)
            else:
                for (ci, cj) in ((hi, hj), (hi + i % 2, hj + j % 2)):
                    rows.append(a), cols.append(cj * sc + ci), vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(sf * sf, sc * sc))


def vcycle_reference(d, omega, R, pre=1, post=1):
    """One V(pre,post) cycle B_s r_s per frequency slot (pre, post in {0, 1}; default V(1,1)),
    written out from its definition on the interior nodes of each level: x1 = omega D^{-1} r
    (x1 = 0 without pre-smoothing), r_c = P^T (r - A x1), x_c = the cycle on the next level
    (exact on the 2 x 2-cell grid), x2 = x1 + P x_c, x3 = x2 + omega D^{-1} (r - A x2)
    (x3 = x2 without post-smoothing), with A = Khat + z M, D = diag(Khat) + z diag(M), P the P1
    interpolation, and the coarse Khat and M the Galerkin products P^T Khat P, P^T M P (Khat =
    nu_max * (5-point stencil) or the per-region stiffness of d.Khat).
    R: (nodes, S) complex; slot 0 holds the k = 0 system on the real part and k = N/2 on the
    imaginary part."""
    p = d.p
    N, S, nu = p.N, p.N // 2, p.nu_max
    z = dft.shifts(N, p.tau)
    levels = []
    n = p.n
    Mf = fem.mass_full(d.mesh, d.mat.sigma).tocsr()
    Kf = (fem.stiffness_full(d.mesh, d.khat_coef) if d.khat_coef is not None
          else nu * fem.stiffness_full(d.mesh)).tocsr()
    while True:
        m = fem.build_mesh(n)
        free = np.flatnonzero(m.free)
        Kh = Kf[free][:, free].tocsr()
        M = Mf[free][:, free].tocsr()
        lev = {"n": n, "free": free, "Kh": Kh, "dK": Kh.diagonal(), "M": M, "dM": M.diagonal(),
               "nodes": (n + 1) ** 2}
        levels.append(lev)
        if n == 2:
            break
        Pf = _prolongation(n // 2)               # coarse (n/2) -> this level
        lev["P"] = Pf[free][:, np.flatnonzero(fem.build_mesh(n // 2).free)].tocsr()
        Mf = (Pf.T @ Mf @ Pf).tocsr()
        Kf = (Pf.T @ Kf @ Pf).tocsr()
        n //= 2

    def cycle(l, zz, r):
        L = levels[l]
        A = L["Kh"] + zz * L["M"]
        D = L["dK"] + zz * L["dM"]
        if L["n"] == 2:
            return r / D
        x1 = omega * r / D if pre else np.zeros_like(r)
        rc = L["P"].T @ (r - A @ x1)
        x2 = x1 + L["P"] @ cycle(l + 1, zz, rc)
        return x2 + omega * (r - A @ x2) / D if post else x2

    fi = levels[0]["free"]
    out = np.zeros_like(R, dtype=np.complex128)
    for s in range(S):
        r = R[fi, s].astype(np.complex128)
        if s == 0:
            out[fi, 0] = cycle(0, 0.0, r.real) + 1j * cycle(0, z[N // 2].real, r.imag)
        else:
            out[fi, s] = cycle(0, z[s], r)
    return out
