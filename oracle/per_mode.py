"""Per-mode relative binning -- plain FP64 oracle, TEST INFRASTRUCTURE ONLY.

Only the test-suite and the CPU-baseline leg of the benchmark may import this
module; the GPU library never does.  It is written from Sec. 2.2 of the paper
(relative binning: the ratio of a template to a fixed reference is replaced by
a complex line across each frequency bin, eqs. d_h_rel_bin and h_h_rel_bin,
contracted with per-bin sums of the data and the reference) applied to every
harmonic mode on its own, and it reuses only the pinned C oracle for the
single-mode templates (``oracle.template`` with a one-mode mask).

Reading of the paper for higher modes (the paper heterodynes the (2,2) mode
only):

* each mode L = (l, m) of the reference h0 has its own band (first and last
  grid frequency where h0_L is non-zero in any channel), its own number of
  log-spaced bins N_L and its own ratio r_L = h_L / h0_L, fitted by a complex
  line across each of its bins (value r0 at the arithmetic bin centre, slope
  r1), exactly as for the (2,2) mode;
* <d|h> = sum_L Z(d, h_L) uses the mode's own bins (A0_L, A1_L of eq.
  d_h_rel_bin with h0_L in place of h0);
* <h|h> = sum_L sum_L' Z(h_L, h_L').  The diagonal terms use the mode's own
  bins (B0_L, B1_L of eq. h_h_rel_bin, the |r1|^2 term dropped as the paper
  does).  A cross term L != L' is summed on the merged grid of the two modes
  (the union of their edges inside the overlap of their bands): in merged
  bin m both lines are evaluated at the merged centre f_m, r_L(f_m), with the
  slope of the mode's own bin, and the product r_L r_L'^* is linearised about
  f_m, dropping the (f - f_m)^2 r1_L r1_L'^* term like the diagonal |r1|^2
  term.  C0 = sum h0_L h0_L'^* / S df and C1 = the same times (f - f_m).
* grid frequency f_k belongs to bin [F_b, F_b+1) (the last bin closed), as
  for the single-mode reference; the merged bins follow the same rule on the
  grid points of the overlap.

Parity status: pinned by tests/test_oracle_per_mode.py (h = h0, a constant
ratio per mode from a phi_ref shift and a distance change -- exact, where the
mode-summed ratio is not --, the residual form, one mode against the C
oracle's single-mode reference, and convergence towards the full-grid
likelihood as the bins are refined).
"""
from __future__ import annotations

import math

import numpy as np

from . import EBAND, EINVAL, MODEL_IMR, OK, Data, template

N_MODES = 6
MODE_M = (2, 3, 4, 1, 2, 3)


def _log_edges(F0: float, FN: float, n: int) -> np.ndarray:
    """n log-spaced bins between F0 and FN (ends exact), with the C library's
    exp and log (Python's math module), as the C oracle does."""
    e = np.empty(n + 1)
    e[0], e[n] = F0, FN
    a, b = math.log(F0), math.log(FN)
    for j in range(1, n):
        e[j] = math.exp(a + j * (b - a) / n)
    return e


def _assign(f_grid: np.ndarray, lo: int, hi: int, edges: np.ndarray) -> np.ndarray:
    """First grid index of each bin: kb[b] = first k in [lo, hi] with f_k >=
    F_b (b >= 1), kb[0] = lo, kb[n] = hi + 1 -- bins [F_b, F_b+1), the last
    closed."""
    n = edges.size - 1
    kb = np.empty(n + 1, dtype=np.int64)
    kb[0], kb[n] = lo, hi + 1
    seg = f_grid[lo:hi + 1]
    for b in range(1, n):
        kb[b] = lo + int(np.searchsorted(seg, edges[b], side="left"))
    for b in range(n - 1, 0, -1):  # bins never run backwards
        kb[b] = min(kb[b], kb[b + 1])
    return kb


def _bin_sums(x, kb, f_grid, centres):
    """sum over each bin of x and of x (f - f_b): x [C][N] -> ([C][nb], [C][nb])."""
    C = x.shape[0]
    nb = kb.size - 1
    s0 = np.zeros((C, nb), dtype=x.dtype)
    s1 = np.zeros((C, nb), dtype=x.dtype)
    for b in range(nb):
        a, e = kb[b], kb[b + 1]
        if e <= a:
            continue
        dx = f_grid[a:e] - centres[b]
        s0[:, b] = x[:, a:e].sum(axis=1)
        s1[:, b] = (x[:, a:e] * dx).sum(axis=1)
    return s0, s1


class ModeBins:
    """One mode's band, edges, bin assignment, sums and reference at the edges."""

    def __init__(self, L: int, k_lo: int, k_hi: int, edges, kb, A0, A1, Ares0, Ares1, B0, B1, h0_edges):
        self.L, self.k_lo, self.k_hi = L, k_lo, k_hi
        self.edges, self.kb = edges, kb
        self.centres = 0.5 * (edges[:-1] + edges[1:])
        self.A0, self.A1, self.Ares0, self.Ares1 = A0, A1, Ares0, Ares1
        self.B0, self.B1, self.h0_edges = B0, B1, h0_edges

    @property
    def n_bins(self):
        return self.edges.size - 1

    def bin_of(self, f: float) -> int:
        """the bin [F_b, F_b+1) (last closed) containing frequency f"""
        return int(min(max(np.searchsorted(self.edges, f, side="right") - 1, 0), self.n_bins - 1))


class PairBins:
    """Merged grid of two modes over the overlap of their bands."""

    def __init__(self, La: int, Lb: int, edges, kb, ba, bb, C0, C1):
        self.La, self.Lb = La, Lb
        self.edges, self.kb = edges, kb
        self.centres = 0.5 * (edges[:-1] + edges[1:])
        self.ba, self.bb = ba, bb  # each mode's own bin holding merged bin m
        self.C0, self.C1 = C0, C1


class PerModeReference:
    """Per-mode heterodyne reference of an IMR source (3 channels)."""

    def __init__(self, modes: int, theta0, data: Data, n_bins_mode):
        self.modes, self.data = int(modes), data
        self.theta0 = np.asarray(theta0, dtype=np.float64)
        self.n_bins_mode = [int(n) for n in n_bins_mode]
        f = data.freqs
        w = 1.0 / data.psd * data.df  # sums are sum (.) / S df; the factor 4 is applied in the contraction
        h0 = {}
        for L in range(N_MODES):
            if modes & (1 << L):
                h0[L] = template(MODEL_IMR, 1 << L, self.theta0, f, data.t_obs)
        h0_tot = sum(h0.values())
        d = data.d
        self.dd = float(np.sum(4.0 * np.abs(d) ** 2 * w))
        r0 = d - h0_tot
        self.lnL0 = -0.5 * float(np.sum(4.0 * np.abs(r0) ** 2 * w))  # eq. like at h = h0
        self.dh0 = float(np.sum(4.0 * (d.conj() * h0_tot).real * w))
        self.hh0 = float(np.sum(4.0 * np.abs(h0_tot) ** 2 * w))
        self.status = OK
        self.mode_bins: dict[int, ModeBins] = {}
        for L, hL in h0.items():
            nz = np.flatnonzero(np.any(hL != 0.0, axis=0))
            if nz.size < 2:
                continue  # the mode has no band on this grid: it takes no part
            lo, hi = int(nz[0]), int(nz[-1])
            nb = self.n_bins_mode[L]
            if nb < 1:
                raise ValueError("bin count must be >= 1")
            edges = _log_edges(f[lo], f[hi], nb)
            kb = _assign(f, lo, hi, edges)
            centres = 0.5 * (edges[:-1] + edges[1:])
            A0, A1 = _bin_sums(d * hL.conj() * w, kb, f, centres)
            Ar0, Ar1 = _bin_sums(r0 * hL.conj() * w, kb, f, centres)
            B0, B1 = _bin_sums(np.abs(hL) ** 2 * w, kb, f, centres)
            he = template(MODEL_IMR, 1 << L, self.theta0, edges, data.t_obs)
            if not np.all(np.abs(he) > 0.0):
                self.status = EBAND  # the ratio h_L / h0_L must exist at every edge of the mode
            self.mode_bins[L] = ModeBins(L, lo, hi, edges, kb, A0, A1, Ar0, Ar1, B0.real, B1.real, he)
        if not self.mode_bins:
            self.status = EBAND
        self.pairs: list[PairBins] = []
        Ls = sorted(self.mode_bins)
        for i, La in enumerate(Ls):
            for Lb in Ls[i + 1:]:
                a, b = self.mode_bins[La], self.mode_bins[Lb]
                lo, hi = max(a.k_lo, b.k_lo), min(a.k_hi, b.k_hi)
                if hi < lo:
                    continue
                Flo, Fhi = f[lo], f[hi]
                e = np.union1d(a.edges[(a.edges >= Flo) & (a.edges <= Fhi)],
                               b.edges[(b.edges >= Flo) & (b.edges <= Fhi)])
                if e.size < 2:  # an overlap of one grid point: one bin of zero width
                    e = np.array([Flo, Fhi if Fhi > Flo else Flo])
                kb = _assign(f, lo, hi, e)
                centres = 0.5 * (e[:-1] + e[1:])
                ba = np.array([a.bin_of(x) for x in e[:-1]], dtype=np.int64)
                bb = np.array([b.bin_of(x) for x in e[:-1]], dtype=np.int64)
                C0, C1 = _bin_sums(h0[La] * h0[Lb].conj() * w, kb, f, centres)
                self.pairs.append(PairBins(La, Lb, e, kb, ba, bb, C0, C1))

    # ------------------------------------------------------------ evaluation
    def _fits(self, theta):
        """per mode: (r at the edges [C][E], r0 at the bin centres, slope r1)"""
        out = {}
        for L, mb in self.mode_bins.items():
            h = template(MODEL_IMR, 1 << L, theta, mb.edges, self.data.t_obs)
            r = h / mb.h0_edges
            r0 = 0.5 * (r[:, :-1] + r[:, 1:])
            r1 = (r[:, 1:] - r[:, :-1]) / np.diff(mb.edges)
            out[L] = (r0, r1)
        return out

    def _line_at(self, L, fits, b, f):
        """mode L's line of bin b (per channel) at frequency f, and its slope"""
        r0, r1 = fits[L]
        mb = self.mode_bins[L]
        return r0[:, b] + r1[:, b] * (f - mb.centres[b]), r1[:, b]

    def core(self, theta):
        """(lnL, Z[d,h], Z[h,h]) in the paper's form (eqs. d_h_rel_bin,
        h_h_rel_bin, like) for one walker."""
        fits = self._fits(theta)
        zdh = 0.0
        zhh = 0.0
        for L, mb in self.mode_bins.items():
            r0, r1 = fits[L]
            zdh += 4.0 * float(np.sum((mb.A0 * r0.conj() + mb.A1 * r1.conj()).real))
            zhh += 4.0 * float(np.sum(mb.B0 * np.abs(r0) ** 2 + 2.0 * mb.B1 * (r0 * r1.conj()).real))
        for p in self.pairs:
            for m in range(p.centres.size):
                fm = p.centres[m]
                ra, sa = self._line_at(p.La, fits, p.ba[m], fm)
                rb, sb = self._line_at(p.Lb, fits, p.bb[m], fm)
                P0 = ra * rb.conj()
                P1 = sa * rb.conj() + ra * sb.conj()
                # both orders (L, L') and (L', L): twice the real part
                zhh += 2.0 * 4.0 * float(np.sum((p.C0[:, m] * P0 + p.C1[:, m] * P1).real))
        lnL = -0.5 * (self.dd + zhh - 2.0 * zdh)  # eq. like
        return lnL, zdh, zhh

    def core_residual(self, theta):
        """lnL in the residual form: lnL(h0) plus terms in delta_L = r_L - 1 only
        (algebraically identical to core)."""
        fits = self._fits(theta)
        acc = 0.0
        for L, mb in self.mode_bins.items():
            r0, r1 = fits[L]
            d0, d1 = r0 - 1.0, r1
            acc += 4.0 * float(np.sum((mb.Ares0 * d0.conj() + mb.Ares1 * d1.conj()).real))
            acc -= 2.0 * float(np.sum(mb.B0 * np.abs(d0) ** 2 + 2.0 * mb.B1 * (d0 * d1.conj()).real))
        for p in self.pairs:
            for m in range(p.centres.size):
                fm = p.centres[m]
                ra, sa = self._line_at(p.La, fits, p.ba[m], fm)
                rb, sb = self._line_at(p.Lb, fits, p.bb[m], fm)
                da, db = ra - 1.0, rb - 1.0
                P0 = da * db.conj()
                P1 = sa * db.conj() + da * sb.conj()
                acc -= 4.0 * float(np.sum((p.C0[:, m] * P0 + p.C1[:, m] * P1).real))
        return self.lnL0 + acc

    def loglike(self, theta):
        th = np.atleast_2d(np.asarray(theta, dtype=np.float64))
        out = np.zeros((3, th.shape[0]))
        for i, t in enumerate(th):
            if not _imr_valid(t):
                out[:, i] = (-np.inf, 0.0, 0.0)
                continue
            out[:, i] = self.core(t)
        return out[0], out[1], out[2]


def _imr_valid(t) -> bool:
    return bool(np.all(np.isfinite(t)) and t[0] > 0.0 and 0.05 <= t[1] <= 1.0 and abs(t[2]) <= 0.99
                and abs(t[3]) <= 0.99 and t[4] > 0.0)
