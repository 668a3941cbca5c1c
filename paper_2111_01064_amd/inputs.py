"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle leg.

This module holds no likelihood, waveform or response arithmetic: it draws
parameters, noise, walker clouds and request streams, and evaluates the
analytic noise PSDs that the library takes as *inputs* (the paper treats the
PSDs as known analytic functions, Sec. 2, and cites their formulas).  Anything
that needs the method itself (a template, an SNR, a curvature) is passed in
as a callable by the caller.

Seeds: numpy PCG64 with ``seed = 20211101 + 100*cfg + index``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

MSUN_S = 4.925490947641267e-6
C_SI = 299792458.0
ARM_M = 2.5e9
YEAR_S = 31557600.0
SEED_BASE = 20211101

# parameter order of a walker (Sec. 2.1): M_T, q, a1, a2, D_L, phi_ref, iota, lambda, beta, psi, t_ref
PARAM_NAMES = ("M_T", "q", "a1", "a2", "D_L", "phi_ref", "iota", "lambda", "beta", "psi", "t_ref")
NPARAM = 11


def rng_for(cfg: int, index: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + 100 * cfg + index))


# --------------------------------------------------------------------------- grids
@dataclass(frozen=True)
class Grid:
    f0: float
    df: float
    n_f: int
    t_obs: float

    @property
    def freqs(self) -> np.ndarray:
        return self.f0 + np.arange(self.n_f) * self.df


def grid_chirp() -> Grid:
    """2^14 linear bins on [1e-4, 0.1] Hz (the single-channel chirp case)."""
    n = 1 << 14
    return Grid(1e-4, (0.1 - 1e-4) / (n - 1), n, 1.0e4 * 2)


def grid_lisa(years: float = 1.0, dt: float = 10.0, n_keep: int | None = None) -> Grid:
    """rfft grid of a series of T_obs = N dt, DC dropped: f_k = (k+1)/T_obs."""
    n = int(round(years * YEAR_S / dt))
    t_obs = n * dt
    nf = n // 2 if n_keep is None else n_keep
    return Grid(1.0 / t_obs, 1.0 / t_obs, nf, t_obs)


def grid_lisa_small(n_f: int = 4096, f_hi: float = 0.05, t_obs: float = YEAR_S) -> Grid:
    """A coarse uniform grid on (0, f_hi] for fast oracle checks."""
    df = f_hi / n_f
    return Grid(df, df, n_f, t_obs)


# --------------------------------------------------------------------------- PSDs
def psd_chirp(f) -> np.ndarray:
    """S(f) = 1e-40 (1 + (f/3e-3)^-4) of the single-channel chirp case."""
    f = np.asarray(f, dtype=np.float64)
    return 1e-40 * (1.0 + (f / 3e-3) ** -4)


def psd_powerlaw(f, s0: float = 1e-40, f_ref: float = 3e-3, alpha: float = -4.0) -> np.ndarray:
    f = np.asarray(f, dtype=np.float64)
    return s0 * (f / f_ref) ** alpha


def psd_lisa_aet(f) -> np.ndarray:
    """First-generation A, E, T noise PSDs in fractional-frequency units.

    Test-mass acceleration 3e-15 m/s^2/sqrt(Hz) with the usual low/high-frequency
    reddening, optical-metrology noise 15e-12 m/sqrt(Hz), arm 2.5e9 m.
    Returns [3][n]; S_A == S_E.
    """
    f = np.asarray(f, dtype=np.float64)
    L = ARM_M / C_SI
    x = 2.0 * np.pi * f * L
    s_pm = (3e-15) ** 2 * (1.0 + (4e-4 / f) ** 2) * (1.0 + (f / 8e-3) ** 4) / (2.0 * np.pi * f * C_SI) ** 2
    s_op = (15e-12) ** 2 * (1.0 + (2e-3 / f) ** 4) * (2.0 * np.pi * f / C_SI) ** 2
    sx2 = np.sin(x) ** 2
    s_ae = 8.0 * sx2 * (2.0 * s_pm * (3.0 + 2.0 * np.cos(x) + np.cos(2.0 * x)) + s_op * (2.0 + np.cos(x)))
    sh2 = np.sin(0.5 * x) ** 2
    s_t = 32.0 * sx2 * sh2 * (4.0 * s_pm * sh2 + s_op)
    return np.stack([s_ae, s_ae.copy(), s_t])


# --------------------------------------------------------------------------- noise
def noise(psd, df: float, rng: np.random.Generator) -> np.ndarray:
    """Stationary Gaussian noise with <n(f) n*(f')> = S/2 delta (one-sided):
    Re and Im independent N(0, S/(4 df)) per channel and frequency."""
    psd = np.atleast_2d(np.asarray(psd, dtype=np.float64))
    sig = np.sqrt(psd / (4.0 * df))
    return sig * rng.standard_normal(psd.shape) + 1j * sig * rng.standard_normal(psd.shape)


# --------------------------------------------------------------------------- sources
def draw_chirp_source(rng: np.random.Generator) -> np.ndarray:
    """Chirp-model source: slots {Mc [Msun], amplitude (placeholder 1), t_c, phi_c}."""
    th = np.zeros(NPARAM)
    th[0] = rng.uniform(1e5, 1e6)
    th[1] = 1.0
    th[2] = 1.0e4
    th[3] = rng.uniform(0.0, 2.0 * np.pi)
    return th


def draw_mbhb_source(rng: np.random.Generator, t_obs: float) -> tuple[np.ndarray, float]:
    """One MBHB source (D_L placeholder 1 Gpc) and its target SNR.

    M_T log-uniform [1e5, 1e7] Msun, Q = m1/m2 ~ U[1, 10] passed as q = 1/Q,
    aligned spins U[-0.99, 0.99], angles from the prior table, t_ref in
    [0.2, 0.8] T_obs, target SNR log-uniform [100, 1000].
    """
    th = np.zeros(NPARAM)
    th[0] = math.exp(rng.uniform(math.log(1e5), math.log(1e7)))
    th[1] = 1.0 / rng.uniform(1.0, 10.0)
    th[2] = rng.uniform(-0.99, 0.99)
    th[3] = rng.uniform(-0.99, 0.99)
    th[4] = 1.0
    th[5] = rng.uniform(0.0, 2.0 * np.pi)
    th[6] = math.acos(rng.uniform(-1.0, 1.0))
    th[7] = rng.uniform(0.0, 2.0 * np.pi)
    th[8] = math.asin(rng.uniform(-1.0, 1.0))
    th[9] = rng.uniform(0.0, np.pi)
    th[10] = rng.uniform(0.2, 0.8) * t_obs
    snr = math.exp(rng.uniform(math.log(100.0), math.log(1000.0)))
    return th, snr


def table_maxll_source(rng: np.random.Generator) -> np.ndarray:
    """The injection printed in the paper's maximum-likelihood table (m1, m2, a1,
    a2, D_L, iota, lambda, beta, t_ref); phi_ref and psi are not printed and are
    drawn here."""
    m1, m2 = 2.599137e6, 1.242861e6
    th = np.zeros(NPARAM)
    th[0] = m1 + m2
    th[1] = m2 / m1
    th[2], th[3] = 7.534822e-1, 6.215875e-1
    th[4] = 5.600578e1
    th[5] = rng.uniform(0.0, 2.0 * np.pi)
    th[6], th[7], th[8] = 1.224532, 3.509097, 2.927012e-1
    th[9] = rng.uniform(0.0, np.pi)
    th[10] = 2.495997e7
    return th


def prior_draws(rng: np.random.Generator, n: int, t_obs: float,
                log_mt=(math.log(1e5), math.log(1e7))) -> np.ndarray:
    """Brute-force search draws from the prior table (M_T log-uniform)."""
    th = np.zeros((n, NPARAM))
    th[:, 0] = np.exp(rng.uniform(log_mt[0], log_mt[1], n))
    th[:, 1] = rng.uniform(0.05, 1.0, n)
    th[:, 2] = rng.uniform(-0.99, 0.99, n)
    th[:, 3] = rng.uniform(-0.99, 0.99, n)
    th[:, 4] = rng.uniform(1e-2, 1e3, n)
    th[:, 5] = rng.uniform(0.0, 2.0 * np.pi, n)
    th[:, 6] = np.arccos(rng.uniform(-1.0, 1.0, n))
    th[:, 7] = rng.uniform(0.0, 2.0 * np.pi, n)
    th[:, 8] = np.arcsin(rng.uniform(-1.0, 1.0, n))
    th[:, 9] = rng.uniform(0.0, np.pi, n)
    th[:, 10] = rng.uniform(0.0, t_obs, n)
    return th


def distance_for_snr(hh_at_unit_distance: float, snr: float, d_unit: float = 1.0) -> float:
    """The template scales as 1/D_L, so SNR = sqrt(<h|h>) scales the same way."""
    return d_unit * math.sqrt(hh_at_unit_distance) / snr


# --------------------------------------------------------------------------- walkers
def clip_walkers(th: np.ndarray) -> np.ndarray:
    """Keep walkers inside the parameter domain: wrap angles, clip q and spins."""
    th = th.copy()
    th[:, 1] = np.clip(th[:, 1], 0.05, 1.0)
    th[:, 2] = np.clip(th[:, 2], -0.99, 0.99)
    th[:, 3] = np.clip(th[:, 3], -0.99, 0.99)
    th[:, 4] = np.abs(th[:, 4])
    th[:, 5] = np.mod(th[:, 5], 2.0 * np.pi)
    th[:, 6] = np.clip(th[:, 6], 0.0, np.pi)
    th[:, 7] = np.mod(th[:, 7], 2.0 * np.pi)
    th[:, 8] = np.clip(th[:, 8], -0.5 * np.pi, 0.5 * np.pi)
    th[:, 9] = np.mod(th[:, 9], np.pi)
    return th


def walker_cloud(theta_true, sigma, temps, n_per_temp: int, rng: np.random.Generator,
                 clip: bool = True) -> np.ndarray:
    """theta ~ N(theta_true, T_k diag(sigma^2)) for each temperature rung."""
    theta_true = np.asarray(theta_true, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    out = []
    for T in temps:
        out.append(theta_true + math.sqrt(T) * sigma * rng.standard_normal((n_per_temp, theta_true.size)))
    th = np.concatenate(out, axis=0)
    return clip_walkers(th) if clip else th


def relative_cloud(theta_true, rel: float, n: int, rng: np.random.Generator) -> np.ndarray:
    """theta ~ theta_true * (1 + rel N(0,1)) per parameter."""
    theta_true = np.asarray(theta_true, dtype=np.float64)
    return theta_true * (1.0 + rel * rng.standard_normal((n, theta_true.size)))


def curvature_sigma(loglike, theta0, rel_step=None) -> np.ndarray:
    """1/sqrt(-d2 lnL / d theta_i^2) from central differences of a supplied
    batched log-likelihood callable (one batch of 2*11+1 points)."""
    theta0 = np.asarray(theta0, dtype=np.float64)
    n = theta0.size
    steps = np.array([1e-5 * theta0[0], 1e-4, 1e-3, 1e-3, 1e-4 * theta0[4], 1e-4, 1e-4,
                      1e-5, 1e-5, 1e-4, 1e-2]) if rel_step is None else np.asarray(rel_step)
    pts = [theta0]
    for i in range(n):
        for s in (+1, -1):
            t = theta0.copy()
            t[i] += s * steps[i]
            pts.append(t)
    lnl = np.asarray(loglike(np.array(pts)), dtype=np.float64)
    sig = np.zeros(n)
    for i in range(n):
        c = -(lnl[1 + 2 * i] - 2.0 * lnl[0] + lnl[2 + 2 * i]) / steps[i] ** 2
        sig[i] = 1.0 / math.sqrt(c) if c > 0 else steps[i]
    return sig


# --------------------------------------------------------------------------- batching / serving
def batch_shapes(rng: np.random.Generator, n_sources: int = 16):
    """Per-source (mode mask, N_b, W) for the ragged multi-source batch:
    a random non-empty subset of the six modes always holding (2,2),
    N_b log-uniform over [64, 512], W log-uniform over [128, 4096]."""
    shapes = []
    for _ in range(n_sources):
        k = int(rng.integers(1, 7))
        extra = rng.permutation(5)[: k - 1] + 1
        mask = 1 | int(sum(1 << int(e) for e in extra))
        nb = int(round(math.exp(rng.uniform(math.log(64), math.log(512)))))
        w = int(round(math.exp(rng.uniform(math.log(128), math.log(4096)))))
        shapes.append((mask, nb, w))
    return shapes


def per_mode_bins(rng: np.random.Generator, mask: int):
    """Bin counts of the six modes for per-mode relative binning: log-uniform
    over [64, 512] for the modes in the mask (0 for the others)."""
    out = [0] * 6
    for i in range(6):
        if mask & (1 << i):
            out[i] = int(round(math.exp(rng.uniform(math.log(64), math.log(512)))))
    return out


def poisson_requests(rng: np.random.Generator, n: int, rate_hz: float, n_samplers: int = 64,
                     n_sources: int = 4, w_max: int = 4096):
    """Open-loop Poisson arrivals: (arrival_s, sampler, source, W) with
    W = round(exp U[0, ln w_max]) and sampler s bound to source s mod n_sources."""
    gaps = rng.exponential(1.0 / rate_hz, n)
    t = np.cumsum(gaps)
    samplers = rng.integers(0, n_samplers, n)
    ws = np.rint(np.exp(rng.uniform(0.0, math.log(w_max), n))).astype(np.int64)
    ws = np.clip(ws, 1, w_max)
    return [(float(t[i]), int(samplers[i]), int(samplers[i]) % n_sources, int(ws[i])) for i in range(n)]
