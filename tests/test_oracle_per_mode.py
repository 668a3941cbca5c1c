"""Pins of the per-mode relative-binning oracle (oracle/per_mode.py, Sec. 2.2
applied to each harmonic mode) against exact special cases, the independently
pinned single-mode C oracle and the full-grid likelihood (CPU only).

pin                                        what a mistake it would catch
-----------------------------------------  ---------------------------------------------
one mode == the C oracle's single-mode      band, edges, bin assignment, A0..B1 per mode
   reference (edges, k_b, sums, lnL)
het == full at h = h0 (all modes)           dropped cross term, wrong factor 2 or 4
h_L = c_L h0_L (phi_ref shift: c_L =        cross-term conj placement and sign; the
   e^{i m dphi}, distance: real c) => exact    merged-grid linearisation at constant r
   (the mode-summed ratio is not)
residual form == paper form                 algebra of the residual rewrite (A - B per
                                               mode, cross terms in delta only)
|het - full| falls ~N_b^-2 for walkers      the merged bin's lookup of each mode's own
   near the truth                              bin and centre offset (a wrong lookup
                                               leaves an O(1) error that does not fall)
"""
import numpy as np
import pytest

import oracle as O
from oracle import per_mode as PM
from paper_2111_01064_amd import inputs as I

ALL = O.ALL_MODES


def _hm_setup(n_f=8192, snr=150.0, seed=3, noisy=True, modes=ALL):
    g = I.grid_lisa_small(n_f, 0.05)
    rng = I.rng_for(2, 80 + seed)
    th, _ = I.draw_mbhb_source(rng, g.t_obs)
    th[0], th[1], th[6] = 1.5e6, 0.3, 1.1  # unequal masses and an inclined orbit: all six modes present
    psd = I.psd_lisa_aet(g.freqs)
    h = O.template(O.MODEL_IMR, modes, th, g.freqs, g.t_obs)
    th[4] = I.distance_for_snr(O.inner(h, h, psd, g.df), snr)
    h = O.template(O.MODEL_IMR, modes, th, g.freqs, g.t_obs)
    d = h + (I.noise(psd, g.df, rng) if noisy else 0.0)
    return g, th, O.Data(d, psd, g.f0, g.df, g.t_obs), rng


def _nb(n):
    return [n] * 6


@pytest.fixture(scope="module")
def hm():
    g, th, data, rng = _hm_setup()
    ref = PM.PerModeReference(ALL, th, data, [48, 40, 36, 56, 44, 32])
    assert ref.status == O.OK
    assert len(ref.mode_bins) == 6 and len(ref.pairs) == 15
    return g, th, data, rng, ref


def test_one_mode_matches_single_mode_oracle():
    g, th, data, rng = _hm_setup(modes=O.MODE_22)
    pm = PM.PerModeReference(O.MODE_22, th, data, _nb(64))
    ref = O.Reference(O.MODEL_IMR, O.MODE_22, th, data, 64)
    mb = pm.mode_bins[0]
    assert (mb.k_lo, mb.k_hi) == (ref.k_lo, ref.k_hi)
    assert np.array_equal(mb.edges, ref.edges)
    assert np.array_equal(mb.kb, ref.kb)
    for a, b in ((mb.A0, ref.A0c), (mb.A1, ref.A1c), (mb.B0, ref.B0), (mb.B1, ref.B1)):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    assert not pm.pairs
    sig = I.curvature_sigma(lambda x: ref.loglike(x)[0], th)
    w = I.walker_cloud(th, sig, (1, 16, 256), 4, rng)
    a, b = pm.loglike(w)[0], ref.loglike(w)[0]
    assert np.all(np.abs(a - b) <= 1e-9 * np.abs(b))


def test_het_equals_full_at_reference(hm):
    g, th, data, _, ref = hm
    lf = O.loglike_full(O.MODEL_IMR, ALL, th, data)[0][0]
    lh, zdh, zhh = ref.core(th)
    assert abs(lh - lf) <= 1e-10 * abs(lf)
    assert abs(ref.lnL0 - lf) <= 1e-10 * abs(lf)
    assert abs(zhh - ref.hh0) <= 1e-10 * ref.hh0


def test_constant_ratio_per_mode_is_exact(hm):
    """A phi_ref shift multiplies mode (l, m) by e^{i m dphi} and a distance
    change every mode by one real factor: each mode's ratio is constant, so
    per-mode binning reproduces the full-grid likelihood exactly; the
    mode-summed ratio of the single-reference scheme is not constant and
    does not."""
    g, th, data, _, ref = hm
    w = np.array(th)
    w[5] += 0.7
    w[4] *= 1.3
    lf, dhf, hhf = O.loglike_full(O.MODEL_IMR, ALL, w, data)
    lh, zdh, zhh = ref.core(w)
    print(f"[pm] constant ratios: |het - full| = {abs(lh - lf[0]):.3e}", flush=True)
    assert abs(lh - lf[0]) <= 1e-9 * max(abs(lf[0]), 1.0) + 1e-6
    assert abs(zdh - dhf[0]) <= 1e-9 * abs(hhf[0]) + 1e-6
    assert abs(zhh - hhf[0]) <= 1e-9 * abs(hhf[0]) + 1e-6
    summed = O.Reference(O.MODEL_IMR, ALL, th, data, 48)
    ls = summed.loglike(w)[0][0]
    print(f"[pm] same walker, mode-summed ratio: |het - full| = {abs(ls - lf[0]):.3e}", flush=True)
    assert abs(ls - lf[0]) > 100 * abs(lh - lf[0])


def test_residual_form_matches_paper_form(hm):
    g, th, data, rng, ref = hm
    sig = np.abs(th) * 1e-5 + 1e-6
    w = I.walker_cloud(th, sig, (1, 100, 10000), 3, rng)
    for t in w:
        a = ref.core(t)[0]
        b = ref.core_residual(t)
        scale = abs(ref.lnL0) + abs(a - ref.lnL0)
        assert abs(a - b) <= 1e-11 * scale, (a, b)


def test_binning_error_falls_with_bin_count():
    g, th, data, rng = _hm_setup(n_f=16384, noisy=False)
    sig = np.abs(th) * 3e-6 + 1e-7
    w = I.walker_cloud(th, sig, (1, 4), 3, rng)
    lf = O.loglike_full(O.MODEL_IMR, ALL, w, data)[0]
    errs = []
    for nb in (16, 32, 64):
        ref = PM.PerModeReference(ALL, th, data, _nb(nb))
        errs.append(np.abs(ref.loglike(w)[0] - lf).max())
    print(f"[pm] max |het - full| at 16/32/64 bins per mode: {errs}", flush=True)
    assert errs[1] < errs[0] / 2.5 and errs[2] < errs[1] / 2.5
