"""Pins of the sampler oracle (oracle/sampler.py, Sec. 3's tempered ensemble
with stretch and sky-mode proposals) on the CPU.

pin                                          what a mistake it would catch
-------------------------------------------  ---------------------------------------------
Philox4x32-10 known-answer vectors           a wrong round, constant or key schedule
   (Random123's published test vectors)
uniforms: mean 1/2, variance 1/12            the word -> (0, 1) map
stretch move alone reproduces the mean and   the z^(d-1) factor, g(z) sampling, partner
   covariance of a correlated Gaussian          choice from the complement half
sky hops: each hop has its inverse with      asymmetric hop choice (no detailed balance)
   equal probability; a hop-invariant
   target is sampled correctly by hops alone
tempered pair: the cold rung still samples   the swap acceptance (sign, beta difference)
   the target, the hot rung its power 1/2
"""
import math

import numpy as np
import pytest

from oracle import sampler as S

LO = np.array([0.0] * 11)
HI = np.array([1.0] * 11)


def test_philox_known_answers():
    kat = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
           ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
           ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
            (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for c, k, want in kat:
        got = S.philox4x32_10(np.array(c, dtype=np.uint64), np.array(k, dtype=np.uint64))
        assert tuple(int(x) for x in got) == want


def test_uniform_moments():
    u = S.uniforms(12345, 7, np.arange(200000), S.ST_MOVE, 0).ravel()
    assert np.all((u > 0) & (u < 1))
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / u.size)
    assert abs(u.var() - 1 / 12) < 5 * 0.0745 / math.sqrt(u.size)


def _gauss(mean, cov):
    ic = np.linalg.inv(cov)

    def f(x):
        d = np.atleast_2d(x) - mean
        return -0.5 * np.einsum("ni,ij,nj->n", d, ic, d)

    return f


def _run(sampler, f, n_iter, burn):
    xs = []
    for it in range(n_iter):
        sampler.step(f)
        if it >= burn:
            xs.append(sampler.x[0].copy())
    return np.concatenate(xs)


def test_stretch_reproduces_gaussian_mean_and_covariance():
    rng = np.random.default_rng(1)
    A = rng.normal(size=(11, 11)) * 0.01
    cov = A @ A.T + np.diag(np.full(11, 0.02 ** 2))
    mean = np.full(11, 0.5)
    f = _gauss(mean, cov)
    W = 64
    x0 = mean + rng.normal(size=(1, W, 11)) * 0.05
    smp = S.Sampler([1.0], x0, f(x0[0])[None, :], LO, HI, seed=11, p_all=0.0, p_lon=0.0, p_lat=0.0)
    xs = _run(smp, f, 2500, 500)
    m, c = xs.mean(axis=0), np.cov(xs.T)
    sd = np.sqrt(np.diag(cov))
    # effective samples: ~W x iterations / autocorrelation time (~50 for d = 11)
    assert np.all(np.abs(m - mean) < 0.15 * sd), (m - mean) / sd
    rel = np.abs(np.sqrt(np.diag(c)) / sd - 1)
    assert np.all(rel < 0.12), rel
    corr_t = cov / np.outer(sd, sd)
    corr_s = c / np.outer(np.sqrt(np.diag(c)), np.sqrt(np.diag(c)))
    assert np.abs(corr_t - corr_s).max() < 0.12
    acc = smp.n_acc[0, S.STRETCH] / smp.n_prop[0, S.STRETCH]
    assert 0.1 < acc < 0.6


def test_sky_hops_are_symmetric_and_keep_an_invariant_target():
    lo, hi = S.prior_box(3.15e7)
    rng = np.random.default_rng(2)
    x = lo + (hi - lo) * rng.uniform(size=(500, 11))
    for kind in (S.SKY_ALL, S.SKY_LON, S.SKY_LAT):
        u_lon, u_lat = rng.uniform(size=500), rng.uniform(size=500)
        y = S.sky_hop(x, np.full(500, kind), u_lon, u_lat)
        # the inverse hop: 4 - k quarter turns (equally likely) and the same reflection (an involution)
        k = np.minimum(np.floor(4 * u_lon), 3)
        inv_lon = ((4 - k) % 4 + 0.5) / 4
        back = S.sky_hop(y, np.full(500, kind), inv_lon, u_lat)
        d = np.abs(back - x)
        d[:, 7] = np.minimum(d[:, 7], 2 * math.pi - d[:, 7])
        d[:, 9] = np.minimum(d[:, 9], math.pi - d[:, 9])
        assert d.max() < 1e-12, kind
        assert np.all(S.in_box(y, lo, hi))
    # a target invariant under the hops (period pi/2 in lambda and psi, even
    # in sin beta and cos iota): hops are always accepted, the marginal of
    # lambda keeps its shape
    def f(xb):
        xb = np.atleast_2d(xb)
        return np.log(1.0 + 0.8 * np.cos(4.0 * xb[:, 7])) + np.log(1.0 + 0.8 * np.cos(4.0 * xb[:, 9])) \
            - 8.0 * xb[:, 8] ** 2 - 8.0 * xb[:, 6] ** 2 - 0.5 * ((xb[:, [0, 1, 2, 3, 4, 5, 10]] - 0.5 * (
                lo + hi)[[0, 1, 2, 3, 4, 5, 10]]) ** 2 / (0.05 * (hi - lo)[[0, 1, 2, 3, 4, 5, 10]]) ** 2).sum(axis=1)
    W = 64
    x0 = 0.5 * (lo + hi) + 0.02 * (hi - lo) * rng.normal(size=(1, W, 11))
    smp = S.Sampler([1.0], x0, f(x0[0])[None, :], lo, hi, seed=5, p_all=0.2, p_lon=0.2, p_lat=0.2)
    xs = _run(smp, f, 2000, 400)
    for kd in (S.SKY_ALL, S.SKY_LON, S.SKY_LAT):
        assert smp.n_acc[0, kd] == smp.n_prop[0, kd] > 0
    # E[cos 4 lambda] under 1 + 0.8 cos(4 lambda) is 0.4
    assert abs(np.cos(4 * xs[:, 7]).mean() - 0.4) < 0.05
    assert abs(xs[:, 8].mean()) < 0.05  # symmetric in sin beta


def test_tempered_pair_samples_target_and_its_power():
    mean, sd = np.full(11, 0.5), np.full(11, 0.03)

    def f(x):
        return -0.5 * (((np.atleast_2d(x) - mean) / sd) ** 2).sum(axis=1)

    rng = np.random.default_rng(3)
    W = 48
    x0 = mean + rng.normal(size=(2, W, 11)) * 0.03
    lnl0 = np.stack([f(x0[0]), f(x0[1])])
    smp = S.Sampler([1.0, 0.5], x0, lnl0, LO, HI, seed=9, p_all=0.0, p_lon=0.0, p_lat=0.0)
    cold, hot = [], []
    for it in range(2500):
        smp.step(f)
        if it >= 500:
            cold.append(smp.x[0].copy())
            hot.append(smp.x[1].copy())
    cold, hot = np.concatenate(cold), np.concatenate(hot)
    assert smp.n_swap_acc[0] > 0
    assert np.all(np.abs(cold.std(axis=0) / sd - 1) < 0.12)
    assert np.all(np.abs(hot.std(axis=0) / (sd * math.sqrt(2)) - 1) < 0.12)
    # cold-rung mean lnL of an 11-D Gaussian: -d/2
    assert abs(f(cold).mean() + 5.5) < 0.5


def test_coordinates_round_trip():
    lo, hi = S.prior_box(3.15e7)
    rng = np.random.default_rng(4)
    x = lo + (hi - lo) * rng.uniform(size=(100, 11))
    th = S.x_to_theta(x)
    assert np.all(np.abs(S.theta_to_x(th) - x) <= 1e-12 * np.maximum(1, np.abs(x)))
