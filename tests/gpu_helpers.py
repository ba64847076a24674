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
