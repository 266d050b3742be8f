"""Time-axis operators of the harmonic-balance method.

Section 2.1: the unknowns are written as truncated Fourier series
(eq. upgh_def) and transformed to N = 2M-1 equally spaced time samples with
the DFT matrix E(j,k) = exp(-2 pi i j k / N) / N (eq. upghdft).  The
time-coupling matrix is H = E^{-1} Omega E (eq. NS-harm) where Omega is the
diagonal of i m omega.  Row j of E corresponds to the harmonic m with
m = j (mod N), |m| <= K, K = M - 1.

The real modal ordering used at the library interface is
[a_0, a_1, b_1, ..., a_K, b_K] with q(t) = a_0 + sum a_m cos(m w t) + b_m sin(m w t),
and samples t_n = n T / N.
"""
from __future__ import annotations

import numpy as np


def n_samples(K: int) -> int:
    return 2 * K + 1


def sample_times(K: int, period: float) -> np.ndarray:
    N = n_samples(K)
    return np.arange(N) * period / N


def harmonic_of_row(K: int) -> np.ndarray:
    """m_j for row j of E: j for j <= K, j - N above."""
    N = n_samples(K)
    j = np.arange(N)
    return np.where(j <= K, j, j - N)


def dft_matrix(K: int) -> np.ndarray:
    """E(j,k) = exp(-2 pi i j k/N)/N."""
    N = n_samples(K)
    j = np.arange(N)
    return np.exp(-2j * np.pi * np.outer(j, j) / N) / N


def omega_matrix(K: int, omega: float) -> np.ndarray:
    """Diagonal frequency-source matrix with entries i m_j omega."""
    return np.diag(1j * harmonic_of_row(K) * omega)


def hb_matrix(K: int, omega: float) -> np.ndarray:
    """H = E^{-1} Omega E; real up to rounding for odd N."""
    E = dft_matrix(K)
    H = np.linalg.inv(E) @ omega_matrix(K, omega) @ E
    return H.real.copy()


def modal_to_complex(a: np.ndarray, K: int) -> np.ndarray:
    """Real modal coefficients (axis 0, length 2K+1) -> complex u*_m for
    m = 0..K using u*_m = (a_m - i b_m)/2 and u*_0 = a_0."""
    out = np.zeros((K + 1,) + a.shape[1:], dtype=complex)
    out[0] = a[0]
    for m in range(1, K + 1):
        out[m] = 0.5 * (a[2 * m - 1] - 1j * a[2 * m])
    return out


def inverse_real_dft(K: int) -> np.ndarray:
    """B with samples = B @ modal (evaluate the real Fourier series at t_n)."""
    N = n_samples(K)
    n = np.arange(N)
    B = np.zeros((N, N))
    B[:, 0] = 1.0
    for m in range(1, K + 1):
        B[:, 2 * m - 1] = np.cos(2 * np.pi * m * n / N)
        B[:, 2 * m] = np.sin(2 * np.pi * m * n / N)
    return B


def real_dft(K: int) -> np.ndarray:
    """F with modal = F @ samples: a_0 = mean, a_m = (2/N) sum x cos,
    b_m = (2/N) sum x sin.  Obtained from E: u*_m = sum_k E(m,k) x_k and
    a_m = 2 Re u*_m, b_m = -2 Im u*_m."""
    E = dft_matrix(K)
    N = n_samples(K)
    F = np.zeros((N, N))
    F[0] = E[0].real
    for m in range(1, K + 1):
        F[2 * m - 1] = 2.0 * E[m].real
        F[2 * m] = -2.0 * E[m].imag
    return F


def to_samples(Y: np.ndarray, K: int) -> np.ndarray:
    """Modal (axis -2 of length N) -> samples, for arrays shaped (..., N, n)."""
    return np.einsum("nm,...ma->...na", inverse_real_dft(K), Y)


def to_modal(y: np.ndarray, K: int) -> np.ndarray:
    return np.einsum("mn,...na->...ma", real_dft(K), y)


def apply_time(Hm: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Apply an N x N time-axis matrix to arrays shaped (..., N, n)."""
    return np.einsum("nk,...ka->...na", Hm, y)
