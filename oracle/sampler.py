"""Parallel-tempered ensemble sampler -- plain oracle, TEST INFRASTRUCTURE ONLY.

Only the test-suite may import this module; the GPU library never does.  It
restates the sampler of Sec. 3 of the paper (an affine-invariant ensemble
with parallel tempering; ~85 % stretch proposals and three kinds of sky-mode
hops) in plain numpy, one iteration at a time, with every random number drawn
from a Philox4x32-10 counter-based generator written here from its published
definition (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC 2011), so that the GPU sampler, which implements the same
generator on its own, can be checked decision for decision.

Readings (the paper gives the structure, not every detail):

* sampling coordinates x = (ln M_T, q, a1, a2, D_L, phi_ref, cos iota,
  lambda, sin beta, psi, t_ref), uniform prior on the box of the paper's
  prior table (spins within +-0.99, the model's domain); theta = (M_T, q,
  a1, a2, D_L, phi_ref, iota, lambda, beta, psi, t_ref) is what the
  likelihood takes;
* rung k samples L(x)^beta_k p(x), beta_0 = 1 > beta_1 > ... >= 0;
* each rung's walkers are split in two halves; the first half moves with the
  second as complement, then the second with the updated first;
* each walker draws its move: stretch (Goodman & Weare: partner j from the
  complement, z from g(z) ~ 1/sqrt(z) on [1/a, a], y = x_j + z (x - x_j),
  acceptance z^(d-1) with d = 11), or a sky-mode hop: to one of the eight
  modes at random (lambda + k pi/2 and psi + k pi/2 for k = 0..3, times the
  reflection beta -> -beta, cos iota -> -cos iota, cos psi -> -cos psi), a
  longitudinal hop alone, or the latitudinal reflection alone; the hops are
  measure-preserving bijections chosen independently of the state, so the
  proposal is symmetric;
* after both halves, adjacent rungs k, k+1 exchange walkers: walker i of k
  with walker (i + s) mod W of k+1 (s uniform per iteration and rung pair),
  accepted with probability min(1, exp((beta_k - beta_k+1)(lnL_k+1 - lnL_k)));
* random numbers: Philox4x32-10 with key (seed low, seed high) and counter
  (iteration, index, stream, half) -> four 32-bit words, each turned into a
  uniform in (0, 1) as (w + 0.5) / 2^32.
"""
from __future__ import annotations

import math

import numpy as np

NDIM = 11
M32 = 0xFFFFFFFF
# Philox4x32 round multipliers and Weyl key increments (the published constants)
PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85

# streams of the counter's third word
ST_MOVE, ST_SWAP = 1, 2
# move kinds
STRETCH, SKY_ALL, SKY_LON, SKY_LAT = 0, 1, 2, 3


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on arrays of counters ctr [..., 4] and keys
    key [..., 2] (uint32): each round multiplies words 0 and 2 by the round
    constants, forms the new words from the high and low halves of the
    products xor'ed with words 1, 3 and the key, and bumps the key by the
    Weyl constants."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64)
    k1 = np.asarray(key[..., 1], dtype=np.uint64)
    for r in range(10):
        p0 = c[0] * PHILOX_M0
        p1 = c[2] * PHILOX_M1
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(M32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(M32)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        if r < 9:
            k0 = (k0 + np.uint64(PHILOX_W0)) & np.uint64(M32)
            k1 = (k1 + np.uint64(PHILOX_W1)) & np.uint64(M32)
    return np.stack(c, axis=-1).astype(np.uint32)


def uniforms(seed: int, iteration: int, index, stream: int, half: int):
    """Four uniforms in (0, 1) per index for counter (iteration, index,
    stream, half)."""
    index = np.asarray(index, dtype=np.uint64)
    ctr = np.zeros(index.shape + (4,), dtype=np.uint64)
    ctr[..., 0] = iteration & M32
    ctr[..., 1] = index
    ctr[..., 2] = stream
    ctr[..., 3] = half
    key = np.zeros(index.shape + (2,), dtype=np.uint64)
    key[..., 0] = seed & M32
    key[..., 1] = (seed >> 32) & M32
    w = philox4x32_10(ctr, key).astype(np.float64)
    return (w + 0.5) / 4294967296.0


def prior_box(t_obs: float):
    """Lower and upper bounds of x (the paper's prior table, spins within
    the model's +-0.99)."""
    lo = np.array([math.log(1e5), 0.05, -0.99, -0.99, 1e-2, 0.0, -1.0, 0.0, -1.0, 0.0, 0.0])
    hi = np.array([math.log(1e8), 1.0, 0.99, 0.99, 1e3, 2 * math.pi, 1.0, 2 * math.pi, 1.0, math.pi, t_obs])
    return lo, hi


def x_to_theta(x):
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    th = x.copy()
    th[:, 0] = np.exp(x[:, 0])
    th[:, 6] = np.arccos(np.clip(x[:, 6], -1.0, 1.0))
    th[:, 8] = np.arcsin(np.clip(x[:, 8], -1.0, 1.0))
    return th


def theta_to_x(th):
    th = np.atleast_2d(np.asarray(th, dtype=np.float64))
    x = th.copy()
    x[:, 0] = np.log(th[:, 0])
    x[:, 6] = np.cos(th[:, 6])
    x[:, 8] = np.sin(th[:, 8])
    return x


def in_box(x, lo, hi):
    return np.all((x >= lo) & (x <= hi), axis=-1)


def sky_hop(x, kind, u_lon, u_lat):
    """Sky-mode hops of walkers x [n][11] of the given kinds: longitudinal
    k = floor(4 u_lon) quarter turns of lambda (mod 2 pi) and psi (mod pi);
    the latitudinal reflection beta -> -beta, cos iota -> -cos iota,
    psi -> pi - psi (cos psi -> -cos psi) when u_lat < 1/2 (SKY_ALL) or always
    (SKY_LAT).  Stretch walkers (kind 0) are returned unchanged."""
    y = np.array(x, dtype=np.float64)
    lon = (kind == SKY_ALL) | (kind == SKY_LON)
    k = np.minimum(np.floor(4.0 * u_lon), 3.0)
    y[lon, 7] = np.fmod(y[lon, 7] + k[lon] * 0.5 * math.pi, 2.0 * math.pi)
    y[lon, 9] = np.fmod(y[lon, 9] + k[lon] * 0.5 * math.pi, math.pi)
    lat = (kind == SKY_LAT) | ((kind == SKY_ALL) & (u_lat < 0.5))
    y[lat, 8] = -y[lat, 8]
    y[lat, 6] = -y[lat, 6]
    y[lat, 9] = math.pi - y[lat, 9]
    return y


class Sampler:
    """State: x [K][W][11] (K rungs of W walkers), lnL [K][W]; lnlike(x_batch)
    returns lnL of an [n][11] batch of sampling coordinates."""

    def __init__(self, betas, x0, lnL0, lo, hi, seed: int, a: float = 2.0, p_all=0.04, p_lon=0.03, p_lat=0.08):
        self.betas = np.asarray(betas, dtype=np.float64)
        self.x = np.array(x0, dtype=np.float64)
        self.lnL = np.array(lnL0, dtype=np.float64)
        self.K, self.W = self.x.shape[:2]
        assert self.W % 2 == 0 and self.W >= 4
        self.lo, self.hi = np.asarray(lo), np.asarray(hi)
        self.seed, self.a = int(seed), float(a)
        self.p = (p_all, p_lon, p_lat)
        self.it = 0
        self.n_acc = np.zeros((self.K, 4))
        self.n_prop = np.zeros((self.K, 4))
        self.n_swap_acc = np.zeros(max(self.K - 1, 1))

    def _move_uniforms(self, half: int):
        K, W, H = self.K, self.W, self.W // 2
        idx = np.arange(K)[:, None] * W + half * H + np.arange(H)[None, :]
        return uniforms(self.seed, self.it, idx, ST_MOVE, half), uniforms(self.seed, self.it, idx, ST_MOVE, half + 2)

    def propose(self, half: int):
        """Proposals for the walkers of one half of every rung: (y [K][W/2][11],
        kind [K][W/2], log of the stretch factor z^(d-1) (0 for hops))."""
        K, W, H = self.K, self.W, self.W // 2
        u, _ = self._move_uniforms(half)
        pa, pl, pt = self.p
        kind = np.full((K, H), STRETCH, dtype=np.int64)
        kind[u[..., 0] < pa + pl + pt] = SKY_LAT
        kind[u[..., 0] < pa + pl] = SKY_LON
        kind[u[..., 0] < pa] = SKY_ALL
        xi = self.x[:, half * H:(half + 1) * H]
        comp = self.x[:, (1 - half) * H:(2 - half) * H]
        j = np.minimum(np.floor(u[..., 1] * H).astype(np.int64), H - 1)
        xj = np.take_along_axis(comp, j[..., None], axis=1)
        z = ((self.a - 1.0) * u[..., 2] + 1.0) ** 2 / self.a
        st = kind == STRETCH
        y = np.where(st[..., None], xj + z[..., None] * (xi - xj), 0.0)
        lz = np.where(st, (NDIM - 1) * np.log(z), 0.0)
        hop = sky_hop(xi.reshape(-1, NDIM), kind.ravel(), u[..., 1].ravel(), u[..., 2].ravel()).reshape(K, H, NDIM)
        y = np.where(st[..., None], y, hop)
        return y, kind, lz

    def accept(self, half: int, y, kind, lz, lnL_y):
        """Metropolis decisions for one half given the proposals' lnL: accept
        when ln v < ln z^(d-1) + beta (lnL_y - lnL), inside the prior box and
        with a finite lnL_y (a walker with a non-finite lnL takes any finite
        proposal)."""
        K, W, H = self.K, self.W, self.W // 2
        _, v = self._move_uniforms(half)
        sl = slice(half * H, (half + 1) * H)
        cur = self.lnL[:, sl]
        ok = in_box(y, self.lo, self.hi) & np.isfinite(lnL_y)
        with np.errstate(invalid="ignore"):
            log_a = np.where(np.isfinite(cur), lz + self.betas[:, None] * (lnL_y - cur), np.inf)
        acc = ok & (np.log(v[..., 0]) < log_a)
        for kd in range(4):
            self.n_prop[:, kd] += (kind == kd).sum(axis=1)
            self.n_acc[:, kd] += ((kind == kd) & acc).sum(axis=1)
        self.x[:, sl] = np.where(acc[..., None], y, self.x[:, sl])
        self.lnL[:, sl] = np.where(acc, lnL_y, cur)
        return acc

    def swap(self):
        """Exchanges between adjacent rungs, k = 0, 1, ... in turn."""
        K, W = self.K, self.W
        for k in range(K - 1):
            s = min(int(uniforms(self.seed, self.it, np.array(k), ST_SWAP, 0)[0] * W), W - 1)
            v = uniforms(self.seed, self.it, k * W + np.arange(W), ST_SWAP, 1)[:, 0]
            j = (np.arange(W) + s) % W
            a, b = self.lnL[k].copy(), self.lnL[k + 1, j].copy()
            with np.errstate(invalid="ignore"):
                log_a = (self.betas[k] - self.betas[k + 1]) * (b - a)
            acc = np.log(v) < np.where(np.isnan(log_a), -np.inf, log_a)
            xa, xb = self.x[k].copy(), self.x[k + 1, j].copy()
            self.x[k] = np.where(acc[:, None], xb, xa)
            self.lnL[k] = np.where(acc, b, a)
            xk1 = self.x[k + 1].copy()
            lk1 = self.lnL[k + 1].copy()
            xk1[j] = np.where(acc[:, None], xa, xb)
            lk1[j] = np.where(acc, a, b)
            self.x[k + 1], self.lnL[k + 1] = xk1, lk1
            self.n_swap_acc[k] += acc.sum()

    def step(self, lnlike):
        """One iteration: both halves of every rung, then the swaps."""
        for half in (0, 1):
            y, kind, lz = self.propose(half)
            ly = np.full(kind.shape, -np.inf)
            ok = in_box(y, self.lo, self.hi)
            if ok.any():
                ly[ok] = lnlike(y[ok])
            self.accept(half, y, kind, lz, ly)
        self.swap()
        self.it += 1
