"""Data ingest: TDI X, Y, Z time series -> A, E, T frequency series -- plain
FP64 oracle, TEST INFRASTRUCTURE ONLY.

Only the test-suite may import this module; the GPU library never does.

Sec. 2.1 (template generation): the TDI observables X, Y, Z have correlated
noise and are combined into the uncorrelated observables
A = (Z - X) / sqrt2, E = (X - 2Y + Z) / sqrt6, T = (X + Y + Z) / sqrt3
(the transform the paper cites), and the data are Fourier transformed before
the analysis (the likelihood of eqs. like and inner works on d~(f)).

Readings (the paper gives no numerical convention for the transform):

* the Fourier convention of the templates, d~(f) = integral d(t)
  e^{-2 pi i f t} dt, approximated on the samples t_n = t0 + n dt,
  n = 0..N-1, by dt sum_n d(t_n) e^{-2 pi i f t_n}, at the frequencies
  f_k = k / (N dt) of the discrete transform;
* an optional Tukey window (cosine tapers over a fraction alpha of the
  series, split between its two ends; alpha = 0: none) multiplies each of
  A, E, T before the transform;
* the returned band is k = k_first .. k_first + n_freq - 1 with
  k_first >= 1 (the library's grids start above zero frequency) and
  k_first + n_freq - 1 <= N / 2.

The discrete transform is numpy's real FFT (a library primitive); nothing is
blocked, fused or reordered beyond the definitions above.
"""
from __future__ import annotations

import numpy as np


def tdi_aet(x, y, z):
    """A, E, T from X, Y, Z (any array shape, elementwise)."""
    x, y, z = (np.asarray(v, dtype=np.float64) for v in (x, y, z))
    return (z - x) / np.sqrt(2.0), (x - 2.0 * y + z) / np.sqrt(6.0), (x + y + z) / np.sqrt(3.0)


def tdi_xyz(a, e, t):
    """The inverse map: X, Y, Z from A, E, T (the transform's matrix is
    orthogonal, so its inverse is its transpose)."""
    a, e, t = (np.asarray(v) for v in (a, e, t))
    x = -a / np.sqrt(2.0) + e / np.sqrt(6.0) + t / np.sqrt(3.0)
    y = -2.0 * e / np.sqrt(6.0) + t / np.sqrt(3.0)
    z = a / np.sqrt(2.0) + e / np.sqrt(6.0) + t / np.sqrt(3.0)
    return x, y, z


def tukey(n: int, alpha: float) -> np.ndarray:
    """Tukey window of n samples: 1 in the middle, 0.5 (1 - cos(pi m / e)) at
    distance m < e = alpha (n - 1) / 2 from either end."""
    if alpha <= 0.0 or n < 2:
        return np.ones(n)
    e = min(alpha, 1.0) * (n - 1) / 2.0
    k = np.arange(n, dtype=np.float64)
    m = np.minimum(k, (n - 1) - k)
    w = np.ones(n)
    lo = m < e
    w[lo] = 0.5 * (1.0 - np.cos(np.pi * m[lo] / e))
    return w


def fd_series(a, dt: float, t0: float, k_first: int, n_freq: int, alpha: float = 0.0) -> np.ndarray:
    """dt sum_n w_n a_n e^{-2 pi i f_k (t0 + n dt)} for k = k_first ..
    k_first + n_freq - 1, f_k = k / (N dt); a [..., N] real."""
    a = np.asarray(a, dtype=np.float64)
    N = a.shape[-1]
    if k_first < 1 or n_freq < 1 or k_first + n_freq - 1 > N // 2:
        raise ValueError("band outside 1 .. N/2")
    spec = np.fft.rfft(a * tukey(N, alpha), axis=-1) * dt
    k = np.arange(k_first, k_first + n_freq)
    f = k / (N * dt)
    return spec[..., k] * np.exp(-2j * np.pi * f * t0)


def tdi_to_aet_fd(xyz, dt: float, t0: float, k_first: int, n_freq: int, alpha: float = 0.0) -> np.ndarray:
    """[3][N] samples of X, Y, Z -> [3][n_freq] complex A~, E~, T~ on the band."""
    xyz = np.asarray(xyz, dtype=np.float64)
    aet = np.stack(tdi_aet(xyz[0], xyz[1], xyz[2]))
    return fd_series(aet, dt, t0, k_first, n_freq, alpha)


def xyz_time_series(aet_band, N: int, dt: float, t0: float, k_first: int) -> np.ndarray:
    """Real X, Y, Z series of N samples whose A, E, T transforms (in the
    convention above, no window) equal aet_band [3][n_freq] on the band and
    vanish elsewhere: the inverse discrete transform of each channel, then
    the inverse of the A, E, T map.  For building ingest inputs from
    frequency-domain templates."""
    aet_band = np.asarray(aet_band, dtype=np.complex128)
    n_freq = aet_band.shape[-1]
    if k_first < 1 or k_first + n_freq - 1 > N // 2 - 1:
        raise ValueError("band must lie strictly inside 1 .. N/2 - 1")
    k = np.arange(k_first, k_first + n_freq)
    f = k / (N * dt)
    spec = np.zeros((3, N // 2 + 1), dtype=np.complex128)
    spec[:, k] = aet_band * np.exp(2j * np.pi * f * t0) / dt
    aet = np.fft.irfft(spec, n=N, axis=-1)
    return np.stack(tdi_xyz(aet[0], aet[1], aet[2]))
