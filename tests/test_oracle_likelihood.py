"""Pins of the oracle's likelihoods (eq. like, eq. inner) and of its
heterodyne (Sec. 2.2) against invariants, exact special cases, brute force
and the paper's printed numbers (CPU only).

pin                                   what a mistake it would catch
------------------------------------  ---------------------------------------------
d = h, no noise => lnL = 0 (Sec. 2)   wrong sign / factor in eq. (like)
het == full at h = h0                 dropped term in A0/B0, wrong 4 or 1/2
h = c h0 (D_L, phi_ref)  => exact     r0 / r1 construction, conj placement
h = h0 (a + b f)  => Z[d,h] exact,    A1 / B1 sign, bin-centre f_b, the paper's
   Z[h,h] = <h|h> - 4 sum B2 |b|^2       dropped |r1|^2 term
one grid point per bin => Z[d,h] =    bin assignment (half-open bins), A1 offset
   <d|h>
|het - full| ~ N_b^-2                 wrong interpolation order
residual form == paper form           algebra of the residual rewrite
bin assignment / band by brute force  off-by-one in k_b, band ends
E<n|n> = 2 N_f per channel            noise normalisation (one-sided S/2 delta)
lnL + <d|d>/2 ~ SNR^2/2 (76005 for    the 4 Re and 1/2 factors (maximum-likelihood
   SNR ~390)                             table: 76005 vs 390^2/2 = 76050)
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2111_01064_amd import inputs as I

TOL_REL = 1e-10


def _lisa_setup(seed=0, n_f=6000, snr=200.0, noisy=True, modes=O.MODE_22):
    g = I.grid_lisa_small(n_f, 0.05)
    rng = I.rng_for(2, 50 + seed)
    th, _ = I.draw_mbhb_source(rng, g.t_obs)
    th[0] = 2e6
    psd = I.psd_lisa_aet(g.freqs)
    h = O.template(O.MODEL_IMR, modes, th, g.freqs, g.t_obs)
    th[4] = I.distance_for_snr(O.inner(h, h, psd, g.df), snr)
    h = O.template(O.MODEL_IMR, modes, th, g.freqs, g.t_obs)
    d = h + (I.noise(psd, g.df, rng) if noisy else 0)
    return g, th, O.Data(d, psd, g.f0, g.df, g.t_obs), rng


def _chirp_setup(noisy=True, seed=0):
    g = I.grid_chirp()
    rng = I.rng_for(1, seed)
    th = I.draw_chirp_source(rng)
    psd = I.psd_chirp(g.freqs)
    h = O.template(O.MODEL_TF2, 0, th, g.freqs, g.t_obs)
    th[1] = 100.0 / math.sqrt(O.inner(h, h, psd, g.df))
    h = O.template(O.MODEL_TF2, 0, th, g.freqs, g.t_obs)
    d = h + (I.noise(psd, g.df, rng) if noisy else 0)
    return g, th, O.Data(d, psd, g.f0, g.df, g.t_obs), rng


def test_noiseless_maximum_is_zero():
    g, th, data, _ = _lisa_setup(noisy=False)
    lf, dh, hh = O.loglike_full(O.MODEL_IMR, O.MODE_22, th, data)
    assert lf[0] == 0.0
    assert abs(dh[0] - hh[0]) < 1e-12 * hh[0]
    ref = O.Reference(O.MODEL_IMR, O.MODE_22, th, data, 64)
    lh, _, _ = ref.loglike(th)
    assert abs(lh[0]) < 1e-12 * ref.dd


@pytest.mark.parametrize("modes", [O.MODE_22, O.MODE_22 | O.MODE_33 | O.MODE_21])
def test_het_equals_full_at_reference(modes):
    g, th, data, _ = _lisa_setup(modes=modes)
    ref = O.Reference(O.MODEL_IMR, modes, th, data, 96)
    assert ref.status == O.OK
    lh, dh, hh = ref.loglike(th)
    lf, dhf, hhf = O.loglike_full(O.MODEL_IMR, modes, th, data)
    assert abs(lh[0] - lf[0]) < TOL_REL * ref.dd
    assert abs(dh[0] - dhf[0]) < TOL_REL * ref.dd
    assert abs(hh[0] - hhf[0]) < TOL_REL * ref.dd


def test_constant_ratio_is_exact():
    g, th, data, _ = _lisa_setup()
    ref = O.Reference(O.MODEL_IMR, O.MODE_22, th, data, 64)
    walkers = []
    for dl in (0.7, 1.3):
        t = th.copy()
        t[4] *= dl
        walkers.append(t)
    for dphi in (0.4, 2.9):  # (2,2) only: h ~ e^{2 i phi_ref}
        t = th.copy()
        t[5] += dphi
        walkers.append(t)
    walkers = np.array(walkers)
    lh, dh, hh = ref.loglike(walkers)
    lf, dhf, hhf = O.loglike_full(O.MODEL_IMR, O.MODE_22, walkers, data)
    assert np.all(np.abs(lh - lf) < TOL_REL * ref.dd)
    assert np.all(np.abs(dh - dhf) < TOL_REL * ref.dd)


def test_affine_ratio_identity():
    g, th, data, _ = _lisa_setup()
    ref = O.Reference(O.MODEL_IMR, O.MODE_22, th, data, 64)
    f = g.freqs
    h0 = O.template(O.MODEL_IMR, O.MODE_22, th, f, g.t_obs)
    a, b = 0.9 - 0.2j, (0.3 + 0.5j) / 0.01
    h = h0 * (a + b * f)
    h_edges = ref.h0c * (a + b * ref.edges)
    lnl, zdh, zhh = ref.core(h_edges)
    _, dh, hh = O.loglike_of(data.d, h, data.psd, g.df)
    assert abs(zdh - dh) < TOL_REL * ref.dd
    dropped = 4.0 * abs(b) ** 2 * ref.B2.sum()
    assert dropped > 1e-6 * hh  # the dropped term is not negligible here
    assert abs(zhh - (hh - dropped)) < TOL_REL * ref.dd


def test_one_grid_point_per_bin_gives_exact_overlap():
    g, th, data, rng = _chirp_setup()
    f = g.freqs
    h0 = O.template(O.MODEL_TF2, 0, th, f, g.t_obs)
    t1 = th.copy()
    t1[0] *= 1.0 + 3e-3   # far from the reference: r is not linear at all
    t1[3] += 1.0
    h = O.template(O.MODEL_TF2, 0, t1, f, g.t_obs)
    lo, hi = 100, 900
    edges = f[lo:hi + 2]
    ref = O.Reference.from_edges(data, h0, edges, lo, hi, h0[:, lo:hi + 2])
    assert np.array_equal(ref.kb, np.arange(lo, hi + 2))
    _, zdh, _ = ref.core(h[:, lo:hi + 2])
    sl = slice(lo, hi + 1)
    dh = O.inner(data.d[:, sl], h[:, sl], data.psd[:, sl], g.df)
    assert abs(zdh - dh) < 1e-12 * abs(O.inner(data.d, data.d, data.psd, g.df))


def test_binning_error_converges_quadratically():
    g, th, data, rng = _chirp_setup()
    t1 = th.copy()
    t1[0] *= 1 + 2e-5
    t1[2] += 0.5
    lf, _, _ = O.loglike_full(O.MODEL_TF2, 0, t1, data)
    errs = []
    for nb in (16, 32, 64, 128, 256):
        ref = O.Reference(O.MODEL_TF2, 0, th, data, nb)
        lh, _, _ = ref.loglike(t1)
        errs.append(abs(lh[0] - lf[0]))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(2.5 < r < 6.5 for r in ratios[1:]), (errs, ratios)


def test_residual_form_matches_paper_form():
    g, th, data, rng = _lisa_setup(modes=O.MODE_22 | O.MODE_44)
    ref = O.Reference(O.MODEL_IMR, O.MODE_22 | O.MODE_44, th, data, 128)
    for k in range(4):
        t = th.copy()
        t[0] *= 1 + 2e-5 * rng.standard_normal()
        t[10] += 3.0 * rng.standard_normal()
        t[7] += 1e-3 * rng.standard_normal()
        h_e = O.template(O.MODEL_IMR, O.MODE_22 | O.MODE_44, t, ref.edges, g.t_obs)
        lp, _, _ = ref.core(h_e)
        lr = ref.core(h_e, residual=True)
        assert abs(lp - lr) < TOL_REL * ref.dd


def test_bin_assignment_and_band_brute_force():
    g, th, data, _ = _lisa_setup()
    ref = O.Reference(O.MODEL_IMR, O.MODE_22, th, data, 128)
    f = g.freqs
    h0 = O.template(O.MODEL_IMR, O.MODE_22, th, f, g.t_obs)
    nz = np.nonzero(np.any(h0 != 0, axis=0))[0]
    assert ref.k_lo == nz[0] and ref.k_hi == nz[-1]
    assert ref.edges[0] == f[ref.k_lo] and ref.edges[-1] == f[ref.k_hi]
    assert np.all(np.diff(ref.edges) > 0)
    r = np.log(ref.edges[1:] / ref.edges[:-1])
    assert np.allclose(r, r[0], rtol=1e-9)
    nb = ref.n_bins
    for k in range(ref.k_lo, ref.k_hi + 1):
        b = int(np.searchsorted(ref.kb, k, side="right") - 1)
        assert ref.kb[b] <= k < ref.kb[b + 1]
        if b < nb - 1:
            assert ref.edges[b] <= f[k] < ref.edges[b + 1]
        else:
            assert ref.edges[b] <= f[k] <= ref.edges[b + 1]
    assert ref.kb[0] == ref.k_lo and ref.kb[-1] == ref.k_hi + 1


def test_linearity_in_data():
    g, th, data, rng = _lisa_setup()
    psd = data.psd
    n2 = I.noise(psd, g.df, rng)
    da = O.Data(data.d, psd, g.f0, g.df, g.t_obs)
    db = O.Data(n2, psd, g.f0, g.df, g.t_obs)
    dc = O.Data(data.d + n2, psd, g.f0, g.df, g.t_obs)
    ra, rb, rc = (O.Reference(O.MODEL_IMR, O.MODE_22, th, x, 64) for x in (da, db, dc))
    assert np.allclose(ra.A0 + rb.A0, rc.A0, rtol=1e-12, atol=1e-12 * np.abs(rc.A0).max())
    assert np.allclose(ra.A1 + rb.A1, rc.A1, rtol=1e-12, atol=1e-12 * np.abs(rc.A1).max())
    assert np.array_equal(ra.B0, rc.B0)


def test_invalid_walkers_give_minus_infinity():
    g, th, data, _ = _lisa_setup()
    ref = O.Reference(O.MODEL_IMR, O.MODE_22, th, data, 64)
    bad = np.tile(th, (5, 1))
    bad[0, 1] = 1.5
    bad[1, 2] = 1.2
    bad[2, 4] = -1.0
    bad[3, 0] = float("nan")
    bad[4, 1] = 0.01
    lh, _, _ = ref.loglike(bad)
    lf, _, _ = O.loglike_full(O.MODEL_IMR, O.MODE_22, bad, data)
    assert np.all(np.isneginf(lh)) and np.all(np.isneginf(lf))


def test_noise_normalisation():
    g = I.grid_lisa_small(4096, 0.05)
    psd = I.psd_lisa_aet(g.freqs)
    vals = []
    for s in range(6):
        n = I.noise(psd, g.df, I.rng_for(9, s))
        vals.append(O.inner(n, n, psd, g.df))
    N = 3 * g.n_f
    sigma = 2.0 * math.sqrt(N)
    for v in vals:
        assert abs(v - 2 * N) < 5 * sigma
    assert abs(np.mean(vals) - 2 * N) < 5 * sigma / math.sqrt(len(vals))


def test_paper_printed_peak_likelihood_convention():
    """Maximum-likelihood table: with <d|d> removed, the noisy run peaked at
    ~+76005 for a source of SNR ~390 (Sec. 3.3; values in
    tests/golden/paper_ldc1a_maxll.json).  At h = s, lnL + <d|d>/2 =
    <d|h> - <h|h>/2 = SNR^2/2 + <n|h>, with <n|h> ~ N(0, SNR^2)."""
    import json
    import os

    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_ldc1a_maxll.json")))
    snr, peak = gold["injected_snr"], gold["max_lnL_without_dd"]
    assert abs(peak - 0.5 * snr ** 2) < 1.0 * snr  # the printed pair is self-consistent
    vals = []
    for s in range(4):
        g, th, data, _ = _lisa_setup(seed=s, snr=snr)
        lf, dh, hh = O.loglike_full(O.MODEL_IMR, O.MODE_22, th, data)
        dd = O.inner(data.d, data.d, data.psd, g.df)
        assert abs(math.sqrt(hh[0]) - snr) < 1e-9 * snr
        v = lf[0] + 0.5 * dd
        assert abs(v - (dh[0] - 0.5 * hh[0])) < 1e-9 * dd
        assert abs(v - 0.5 * snr ** 2) < 5 * snr
        vals.append(v)
    assert abs(np.mean(vals) - peak) < 5 * snr


def test_chirp_het_vs_full_method_error_is_small_near_truth():
    g, th, data, rng = _chirp_setup()
    ref = O.Reference(O.MODEL_TF2, 0, th, data, 64)
    assert ref.edges[0] == g.freqs[0] and ref.edges[-1] == g.freqs[-1]
    w = I.relative_cloud(th, 1e-4, 16, rng)
    w[:, 4:] = 0.0
    lh, _, _ = ref.loglike(w)
    lf, _, _ = O.loglike_full(O.MODEL_TF2, 0, w, data)
    near = (lf - lf.max()) > -50
    # method (not implementation) error of 64 bins near the peak: a few 1e-2
    assert np.all(np.abs(lh - lf)[near] < 0.1)


# ----------------------------------------------------------------- reference update (Sec. 3.2)
def _best_by_definition(v):
    """Brute force: the first index i with v[i] finite and no finite value above it."""
    fin = [i for i in range(len(v)) if math.isfinite(v[i])]
    for i in fin:
        if all(v[j] <= v[i] for j in fin):
            return i
    return -1


def test_best_walker_brute_force():
    rng = np.random.default_rng(5)
    specials = [np.nan, np.inf, -np.inf]
    for trial in range(300):
        n = int(rng.integers(0, 12))
        v = rng.integers(-3, 3, size=n).astype(np.float64)  # many ties
        for i in range(n):
            if rng.random() < 0.25:
                v[i] = specials[int(rng.integers(0, 3))]
        assert O.best_walker(v) == _best_by_definition(list(v)), v
    assert O.best_walker([]) == -1
    assert O.best_walker([np.nan, -np.inf, np.inf]) == -1
    assert O.best_walker([np.inf, 1.0, 1.0]) == 1
    assert O.best_walker([-5.0, 2.0, np.nan, 2.0]) == 1


def test_refresh_reference_rebuilds_at_the_best_walker():
    g = I.grid_lisa_small(2048, 0.05)
    rng = I.rng_for(2, 11)
    th, _ = I.draw_mbhb_source(rng, g.t_obs)
    psd = I.psd_lisa_aet(g.freqs)
    d = O.template(O.MODEL_IMR, O.MODE_22, th, g.freqs, g.t_obs)
    data = O.Data(d, psd, g.f0, g.df, g.t_obs)
    ref = O.Reference(O.MODEL_IMR, O.MODE_22, th, data, 32)
    w = I.walker_cloud(th, np.abs(th) * 1e-4 + 1e-6, (1, 4), 4, rng)
    lnl, _, _ = ref.loglike(w)
    st, pick, new = O.refresh_reference(ref, w, lnl)
    assert st == O.OK and pick == int(np.argmax(lnl))
    direct = O.Reference(O.MODEL_IMR, O.MODE_22, w[pick], data, 32)
    assert new.n_bins == 32 and new.k_lo == direct.k_lo and new.k_hi == direct.k_hi
    for name in ("edges", "kb", "A0", "A1", "B0", "B1", "h0_edges"):
        assert np.array_equal(getattr(new, name), getattr(direct, name)), name
    # failures leave the caller with the old reference
    assert O.refresh_reference(ref, w, np.full(len(w), -np.inf))[:2] == (O.EINVAL, -1)
    bad = w.copy()
    bad[0, 1] = 2.0  # q outside (0.05, 1]
    assert O.refresh_reference(ref, bad, np.arange(len(w))[::-1].astype(float))[:2] == (O.EINVAL, 0)
    late = w.copy()
    late[0, 10] = -1e3 * g.t_obs  # the whole signal lies before the observation
    st, pick, new = O.refresh_reference(ref, late, np.arange(len(w))[::-1].astype(float))
    assert (st, pick, new) == (O.EBAND, 0, None)
