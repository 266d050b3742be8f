"""Pins of the oracle's time-axis operators (Section 2.1, eqs. upghdft and
NS-harm) against closed forms."""
import numpy as np
import pytest

from oracle import spectral


@pytest.mark.parametrize("K", [0, 1, 2, 5, 10, 12])
def test_dft_round_trips(K):
    N = 2 * K + 1
    E = spectral.dft_matrix(K)
    assert np.allclose(np.linalg.inv(E) @ E, np.eye(N), atol=1e-13)
    # E^{-1} = N E^H (unitary up to scale): closed form of the inverse DFT
    assert np.allclose(np.linalg.inv(E), N * E.conj().T, atol=1e-12)
    F, B = spectral.real_dft(K), spectral.inverse_real_dft(K)
    assert np.allclose(F @ B, np.eye(N), atol=1e-13)
    assert np.allclose(B @ F, np.eye(N), atol=1e-13)


@pytest.mark.parametrize("K", [1, 3, 10])
def test_parseval(K):
    rng = np.random.default_rng(K)
    N = 2 * K + 1
    a = rng.normal(size=N)
    x = spectral.inverse_real_dft(K) @ a
    lhs = np.sum(x ** 2)
    rhs = N * (a[0] ** 2 + 0.5 * np.sum(a[1:] ** 2))
    assert abs(lhs - rhs) <= 1e-12 * rhs


def test_series_evaluation_matches_cos_sin():
    K, T = 3, 2.5
    t = spectral.sample_times(K, T)
    a = np.array([0.3, 1.0, -2.0, 0.5, 0.25, -0.1, 0.7])
    w = 2 * np.pi / T
    direct = (a[0] + sum(a[2 * m - 1] * np.cos(m * w * t) + a[2 * m] * np.sin(m * w * t)
                         for m in range(1, K + 1)))
    assert np.allclose(spectral.inverse_real_dft(K) @ a, direct, atol=1e-14)


@pytest.mark.parametrize("K", [1, 2, 5, 10, 12])
def test_H_closed_form(K):
    """Odd-N Fourier spectral differentiation matrix (Trefethen, Spectral
    Methods in MATLAB, ch. 3): H_nk = (w/2) (-1)^(n-k) csc(pi (n-k)/N), 0 on
    the diagonal."""
    N = 2 * K + 1
    w = 2 * np.pi / 0.8
    H = spectral.hb_matrix(K, w)
    n = np.arange(N)
    d = n[:, None] - n[None, :]
    with np.errstate(divide="ignore"):
        ref = np.where(d == 0, 0.0, 0.5 * w * (-1.0) ** d / np.sin(np.pi * d / N))
    assert np.allclose(H, ref, rtol=1e-12, atol=1e-12 * w)
    assert np.allclose(H, -H.T, atol=1e-12 * w)           # skew-symmetric
    assert np.allclose(np.diag(H), 0.0, atol=1e-12 * w)   # zero diagonal
    for j in range(N):                                    # circulant
        assert np.allclose(np.roll(H[0], j), H[j], atol=1e-12 * w)


@pytest.mark.parametrize("K", [1, 4, 10])
def test_H_differentiates_trig_polynomials(K):
    rng = np.random.default_rng(7)
    T = 1.3
    w = 2 * np.pi / T
    t = spectral.sample_times(K, T)
    a = rng.normal(size=2 * K + 1)
    x = a[0] + sum(a[2 * m - 1] * np.cos(m * w * t) + a[2 * m] * np.sin(m * w * t)
                   for m in range(1, K + 1))
    dx = sum(m * w * (-a[2 * m - 1] * np.sin(m * w * t) + a[2 * m] * np.cos(m * w * t))
             for m in range(1, K + 1))
    assert np.allclose(spectral.hb_matrix(K, w) @ x, dx, atol=1e-11 * w * np.abs(a).sum())


def test_H_eigenvalues():
    K, w = 4, 3.0
    ev = np.sort(np.linalg.eigvals(spectral.hb_matrix(K, w)).imag)
    assert np.allclose(ev, np.sort(w * np.arange(-K, K + 1)), atol=1e-10)
