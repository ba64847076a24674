"""Discrete Fourier transform along time, by its definition (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Remark "rem:parallel" of the paper: a time-periodic, time-invariant linear system
becomes block diagonal under the DFT in time. For the implicit-Euler system
    (M/tau + Khat) v^n - (M/tau) v^{n-1} = r^n,  v^0 = v^N,
the DFT  V_k = sum_{j=0}^{N-1} v^{j+1} exp(-2 pi i j k / N)  turns the cyclic
shift into multiplication by exp(-2 pi i k / N), so each frequency solves
    (Khat + z_k M) V_k = R_k,   z_k = (1 - exp(-2 pi i k / N)) / tau.

Packed half-spectrum format of real sequences (N even), S = N/2 complex slots:
    slot 0      = (Re V_0) + i (Re V_{N/2})      (both are real for real input)
    slot k >= 1 = V_k,  k = 1 .. N/2 - 1.
"""
from __future__ import annotations

import numpy as np


def dft_matrix(N: int) -> np.ndarray:
    j = np.arange(N)
    return np.exp(-2j * np.pi * np.outer(j, j) / N)


def dft(X: np.ndarray) -> np.ndarray:
    """Full complex DFT along axis 0: out[k] = sum_j X[j] exp(-2 pi i j k / N)."""
    N = X.shape[0]
    W = dft_matrix(N)
    return np.tensordot(W, X, axes=(1, 0))


def idft(Y: np.ndarray) -> np.ndarray:
    """Inverse of dft(): out[j] = (1/N) sum_k Y[k] exp(+2 pi i j k / N)."""
    N = Y.shape[0]
    W = np.conj(dft_matrix(N))
    return np.tensordot(W, Y, axes=(1, 0)) / N


def pack(Vfull: np.ndarray) -> np.ndarray:
    """Full spectrum of a real sequence (N, ...) -> packed half spectrum (N/2, ...)."""
    N = Vfull.shape[0]
    out = Vfull[: N // 2].astype(np.complex128).copy()
    out[0] = Vfull[0].real + 1j * Vfull[N // 2].real
    return out


def unpack(P: np.ndarray, N: int) -> np.ndarray:
    """Packed half spectrum (N/2, ...) -> full Hermitian spectrum (N, ...)."""
    full = np.zeros((N,) + P.shape[1:], dtype=np.complex128)
    full[0] = P[0].real
    full[N // 2] = P[0].imag
    for k in range(1, N // 2):
        full[k] = P[k]
        full[N - k] = np.conj(P[k])
    return full


def rfft_packed(X: np.ndarray) -> np.ndarray:
    """Real series (N, ...) -> packed half spectrum (N/2, ...)."""
    return pack(dft(X))


def irfft_packed(P: np.ndarray, N: int) -> np.ndarray:
    """Packed half spectrum (N/2, ...) -> real series (N, ...), including the 1/N factor."""
    return idft(unpack(P, N)).real


def shifts(N: int, tau: float) -> np.ndarray:
    """z_k = (1 - exp(-2 pi i k / N)) / tau for k = 0..N/2 (the exact implicit-Euler symbol)."""
    k = np.arange(N // 2 + 1)
    return (1.0 - np.exp(-2j * np.pi * k / N)) / tau
