"""Parity at the benchmark's full size, on the benchmark's own workload: the
1-yr grid at dt = 10 s (1 577 880 Fourier bins x 3 channels), 128 bins, the
eight sources of the benchmark step (the same seeds and recipe, SNR 107-948)
with 8 temperatures x 64 walkers each (4096 walkers), launched the way
bench.py launches the step (one batch issued with mbh_batch_launch_direct,
flattened mapping).  The data, references and walkers come from the oracle
and the input generators only (the benchmark sets D_L from the library's
<h|h>; here it is the oracle's, so the data agree with the benchmark's to
rounding, not bit for bit).

Every heterodyned result of the batch is checked against the oracle's
heterodyned likelihood (cheap per walker at any grid size) in both
precisions; the reference build (coefficients, band, lnL(h0) against the
oracle's full grid) and three full-grid walkers per source (cold, warm and
hot rungs), which cost the oracle about half a second each at this size,
are checked too.
"""
import numpy as np
import pytest

import oracle as O
from paper_2111_01064_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-3
N_SOURCES = 8  # the benchmark step's sources
TEMPS = (1, 2, 4, 8, 16, 32, 64, 128)
PER_TEMP = 64
N_BINS = 128


@pytest.fixture(scope="module")
def M():
    from paper_2111_01064_amd import mbh

    return mbh


@pytest.fixture(scope="module")
def ctx(M):
    return M.Context(0)


@pytest.fixture(scope="module")
def full(M, ctx):
    import torch

    g = I.grid_lisa()
    psd = I.psd_lisa_aet(g.freqs)
    out = []
    for s in range(N_SOURCES):
        rng = I.rng_for(2, s)  # the benchmark step's seeds
        th, snr = I.draw_mbhb_source(rng, g.t_obs)
        # the template scales as 1/D_L (placeholder 1 Gpc)
        h = O.template(O.MODEL_IMR, O.MODE_22, th, g.freqs, g.t_obs)
        th[4] = I.distance_for_snr(O.inner(h, h, psd, g.df), snr)
        d = h * (1.0 / th[4]) + I.noise(psd, g.df, rng)
        del h
        data = O.Data(d, psd, g.f0, g.df, g.t_obs)
        ref = O.Reference(O.MODEL_IMR, O.MODE_22, th, data, N_BINS)
        assert ref.status == O.OK
        sig = I.curvature_sigma(lambda x: ref.loglike(x)[0], th)
        w = I.walker_cloud(th, sig, TEMPS, PER_TEMP, rng)
        gd = M.data_create(ctx, torch.as_tensor(d, device="cuda"), torch.as_tensor(psd, device="cuda"), g.f0, g.df,
                           g.t_obs)
        gr = M.build_reference_coeffs(ctx, gd, M.MODEL_IMR, M.MODE_22, th, N_BINS)
        print(f"[fullsize] source {s}: SNR {snr:.0f}, M_T {th[0]:.3g} Msun, band bins {ref.k_lo}..{ref.k_hi}",
              flush=True)
        out.append(dict(th=th, snr=snr, data=data, ref=ref, walkers=w, gdata=gd, gref=gr))
    return g, out


def test_fullsize_reference(full):
    _, srcs = full
    for c in srcs:
        r, gr = c["ref"], c["gref"]
        ex, info = gr.export(), gr.info
        assert info["k_lo"] == r.k_lo and info["k_hi"] == r.k_hi
        assert np.array_equal(ex["kb"], r.kb)
        for name, a, b in (("A0", ex["A0"], r.A0c), ("A1", ex["A1"], r.A1c), ("B0", ex["B0"], r.B0),
                           ("B1", ex["B1"], r.B1)):
            err = np.abs(a - b).max() / np.abs(b).max()
            print(f"[fullsize] reference {name}: max rel err {err:.2e}", flush=True)
            assert err < 1e-9
        lf, _, _ = O.loglike_full(O.MODEL_IMR, O.MODE_22, c["th"], c["data"])
        print(f"[fullsize] lnL(h0): library {info['lnL0']:.6f} oracle full grid {lf[0]:.6f}", flush=True)
        assert abs(info["lnL0"] - lf[0]) < TOL


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fullsize_batch_heterodyned(M, ctx, full, prec):
    import torch

    _, srcs = full
    p = M.FP64 if prec == "fp64" else M.MIXED
    M.set_lanes(ctx, N_BINS, 1, p, 0)
    thetas = [torch.as_tensor(c["walkers"], device="cuda") for c in srcs]
    lnls = [torch.empty(len(c["walkers"]), dtype=torch.float64, device="cuda") for c in srcs]
    b = M.Batch(ctx, [c["gref"] for c in srcs], thetas, lnls, prec=p)
    b.launch_direct()
    torch.cuda.synchronize()
    b.close()
    for c, l in zip(srcs, lnls):
        got = l.cpu().numpy()
        ref_l, _, _ = c["ref"].loglike(c["walkers"])
        err = np.abs(got - ref_l)
        print(f"[fullsize] het {prec}: n={got.size} max|dlnL|={err.max():.3e} median={np.median(err):.3e} "
              f"lnL range=[{ref_l.min():.4g}, {ref_l.max():.4g}]", flush=True)
        assert np.all(err <= TOL)
        if prec == "fp64":
            assert np.all(err <= 1e-6 + 1e-12 * np.abs(ref_l))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fullsize_full_grid(M, ctx, full, prec):
    import torch

    _, srcs = full
    p = M.FP64 if prec == "fp64" else M.MIXED
    for c in srcs:
        w = c["walkers"][[0, 200, 511]]  # cold, warm and hot rungs
        got = M.loglike_full(ctx, c["gdata"], M.MODEL_IMR, M.MODE_22, torch.as_tensor(w, device="cuda"),
                             p).cpu().numpy()
        ref_l, _, _ = O.loglike_full(O.MODEL_IMR, O.MODE_22, w, c["data"])
        err = np.abs(got - ref_l)
        print(f"[fullsize] full {prec}: max|dlnL|={err.max():.3e} lnL range=[{ref_l.min():.4g}, {ref_l.max():.4g}]",
              flush=True)
        assert np.all(err <= 1e-6 + 1e-11 * np.abs(ref_l))


def test_fullsize_full_grid_walker_groups(M, ctx, full):
    """A full-grid call larger than one group of walkers (the partial sums of
    a group are capped at 1 GiB: 7258 walkers with <d|h>, <h|h> on this grid)
    gives, walker for walker, the results of smaller calls bit for bit, and
    the oracle's on a sample."""
    import torch

    g, srcs = full
    c = srcs[0]
    draws = I.prior_draws(I.rng_for(3, 0), 7500, g.t_obs)
    td = torch.as_tensor(draws, device="cuda")
    dh_all = torch.empty((len(draws), 2), dtype=torch.float64, device="cuda")
    big = M.loglike_full(ctx, c["gdata"], M.MODEL_IMR, M.MODE_22, td, M.FP64, dh_hh=dh_all).cpu().numpy()
    parts, dhs = [], []
    for a, b in ((0, 4000), (4000, 7500)):
        dh = torch.empty((b - a, 2), dtype=torch.float64, device="cuda")
        parts.append(M.loglike_full(ctx, c["gdata"], M.MODEL_IMR, M.MODE_22, td[a:b].contiguous(), M.FP64,
                                    dh_hh=dh).cpu().numpy())
        dhs.append(dh.cpu().numpy())
    assert np.array_equal(big, np.concatenate(parts), equal_nan=True)
    assert np.array_equal(dh_all.cpu().numpy(), np.concatenate(dhs))
    sample = [0, 7257, 7258, 7499]
    ref_l, _, _ = O.loglike_full(O.MODEL_IMR, O.MODE_22, draws[sample], c["data"])
    ok = np.isfinite(ref_l)
    err = np.abs(big[sample] - ref_l)[ok]
    print(f"[fullsize] full grid, 7500 draws in two groups: sample max|dlnL|={err.max():.3e}", flush=True)
    assert np.all(err <= 1e-6 + 1e-11 * np.abs(ref_l[ok]))
