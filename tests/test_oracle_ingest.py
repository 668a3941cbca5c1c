"""Pins of the ingest oracle (oracle/ingest.py, Sec. 2.1: X, Y, Z -> A, E, T
and the Fourier transform of the data) on the CPU.

pin                                             what a mistake it would catch
----------------------------------------------  ---------------------------------------------
noise with equal X, Y, Z auto-spectra and       a wrong sign or index in the A, E, T
   equal cross-spectra comes out uncorrelated,     combination (the paper: A, E, T are the
   with A and E of equal power                     uncorrelated observables, A and E alike)
common-mode X = Y = Z lands in T alone          the normalisations sqrt2, sqrt6, sqrt3
tdi_xyz inverts tdi_aet                         the inverse used to build ingest inputs
Tukey window = scipy.signal.windows.tukey        the taper length or phase
a cosine at a grid frequency, sampled from t0:  the dt scaling, the sign of the exponent
   d~(f_k) = (N dt / 2) e^{i phase}, 0 elsewhere   and of the t0 phase factor
Parseval: sum |x|^2 dt = sum over the full      a missing factor in the transform
   spectrum |d~|^2 df
band -> X, Y, Z series -> band, exactly         the inverse transform and the band offset
"""
import numpy as np
import pytest
from scipy.signal import windows

from oracle import ingest as G


def test_aet_uncorrelated_for_symmetric_xyz_noise():
    rng = np.random.default_rng(0)
    for a, b in ((2.0, -0.7), (1.0, 0.45), (3.0, 1.2)):
        C = a * np.eye(3) + b * (np.ones((3, 3)) - np.eye(3))   # X, Y, Z covariance
        # rows of the transform from unit inputs
        M = np.stack([np.array(G.tdi_aet(*np.eye(3)[:, j])) for j in range(3)], axis=1)
        D = M @ C @ M.T
        assert np.allclose(D - np.diag(np.diag(D)), 0.0, atol=1e-14)
        assert np.isclose(D[0, 0], D[1, 1]) and np.isclose(D[0, 0], a - b) and np.isclose(D[2, 2], a + 2 * b)
        # and on samples
        L = np.linalg.cholesky(C)
        xyz = L @ rng.normal(size=(3, 400000))
        aet = np.stack(G.tdi_aet(*xyz))
        S = aet @ aet.T / xyz.shape[1]
        assert np.abs(S - D).max() < 0.02 * a


def test_common_mode_is_t_only_and_inverse():
    s = np.linspace(-1.0, 2.0, 7)
    A, E, T = G.tdi_aet(s, s, s)
    assert np.allclose(A, 0) and np.allclose(E, 0) and np.allclose(T, np.sqrt(3.0) * s)
    A, E, T = G.tdi_aet(-s, 0 * s, s)
    assert np.allclose(A, np.sqrt(2.0) * s) and np.allclose(E, 0) and np.allclose(T, 0)
    rng = np.random.default_rng(1)
    x, y, z = rng.normal(size=(3, 50))
    back = G.tdi_xyz(*G.tdi_aet(x, y, z))
    assert np.allclose(np.stack(back), np.stack([x, y, z]), atol=1e-14)


@pytest.mark.parametrize("n,alpha", [(16, 0.5), (101, 0.1), (1000, 0.25), (64, 1.0), (33, 0.0)])
def test_tukey_matches_scipy(n, alpha):
    assert np.allclose(G.tukey(n, alpha), windows.tukey(n, alpha), atol=1e-15)


@pytest.mark.parametrize("t0", [0.0, 12345.6, -3.25])
def test_cosine_at_a_grid_frequency(t0):
    N, dt, k0, amp, ph = 4096, 5.0, 137, 1.7, 0.6
    f0 = k0 / (N * dt)
    t = t0 + dt * np.arange(N)
    x = amp * np.cos(2 * np.pi * f0 * t + ph)
    d = G.fd_series(x, dt, t0, 1, N // 2 - 1)
    want = np.zeros(N // 2 - 1, dtype=complex)
    want[k0 - 1] = amp * N * dt / 2 * np.exp(1j * ph)
    assert np.abs(d - want).max() < 1e-9 * amp * N * dt


def test_parseval():
    rng = np.random.default_rng(2)
    N, dt = 2048, 2.0
    x = rng.normal(size=N)
    full = np.fft.rfft(x) * dt  # as fd_series, every bin
    d = G.fd_series(x, dt, 0.0, 1, N // 2)
    assert np.allclose(d, full[1:])
    df = 1.0 / (N * dt)
    power = df * (abs(full[0]) ** 2 + 2 * np.sum(np.abs(full[1:N // 2]) ** 2) + abs(full[N // 2]) ** 2)
    assert np.isclose(np.sum(x ** 2) * dt, power, rtol=1e-12)


def test_band_round_trip():
    rng = np.random.default_rng(3)
    N, dt, t0, k_first, n_freq = 8192, 10.0, 100.0, 40, 1500
    band = rng.normal(size=(3, n_freq)) + 1j * rng.normal(size=(3, n_freq))
    xyz = G.xyz_time_series(band, N, dt, t0, k_first)
    assert xyz.shape == (3, N) and np.isrealobj(xyz)
    back = G.tdi_to_aet_fd(xyz, dt, t0, k_first, n_freq)
    assert np.abs(back - band).max() < 1e-11 * np.abs(band).max()
