"""GPU ingest (mbh_tdi_to_aet_fd, mbh_data_create_tdi; Sec. 2.1) against the
ingest oracle (oracle/ingest.py).

Parity: the A, E, T band of seeded X, Y, Z series, element by element, for
even and odd series lengths, with and without a window, within 1e-12 of the
band's largest value (the transform's rounding grows like log N).

End to end: a frequency-domain source with noise (the oracle's template)
is turned into X, Y, Z time series by the oracle's inverse; data ingested
from them on the GPU must give the likelihoods of the frequency-domain data:
<d|d>, full-grid and heterodyned lnL, to FP64 rounding.
"""
import numpy as np
import pytest

import oracle as O
from oracle import ingest as OI
from paper_2111_01064_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    from paper_2111_01064_amd import mbh

    return mbh


@pytest.fixture(scope="module")
def ctx(M):
    return M.Context(0)


def _t(x):
    import torch

    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


@pytest.mark.parametrize("N,alpha,t0", [(15360, 0.0, 0.0), (15360, 0.1, 1234.5), (10001, 0.25, -77.0)])
def test_tdi_to_aet_matches_oracle(M, ctx, N, alpha, t0):
    rng = I.rng_for(9, N)
    dt = 5.0
    xyz = rng.normal(size=(3, N)) * np.array([[1.0], [0.7], [1.3]])
    for k_first, n_freq in ((1, N // 2), (17, 900)):
        want = OI.tdi_to_aet_fd(xyz, dt, t0, k_first, n_freq, alpha)
        got = M.tdi_to_aet_fd(ctx, _t(xyz), dt, t0, k_first, n_freq, alpha).cpu().numpy()
        err = np.abs(got - want).max() / np.abs(want).max()
        print(f"[ingest] N={N} alpha={alpha} band {k_first}+{n_freq}: max rel err {err:.2e}", flush=True)
        assert err < 1e-12


def test_ingest_full_size_matches_oracle(M, ctx):
    """The bench's ingest workload: one year at dt = 10 s (N = 3 155 760 =
    2^4 3^4 5 487, so the transform takes rocFFT's Bluestein path), the whole
    band k = 1 .. N/2, with a Tukey window and a start time, against the
    oracle element by element within 1e-11 of the band's largest value."""
    dt, t0, alpha = 10.0, 12345.6, 0.1
    N = int(round(I.YEAR_S / dt))
    rng = I.rng_for(9, 77)
    xyz = rng.normal(size=(3, N)) * np.array([[1.0], [0.7], [1.3]])
    want = OI.tdi_to_aet_fd(xyz, dt, t0, 1, N // 2, alpha)
    got = M.tdi_to_aet_fd(ctx, _t(xyz), dt, t0, 1, N // 2, alpha).cpu().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"[ingest] full size N={N}: max rel err {err:.2e}", flush=True)
    assert err < 1e-11


def test_ingest_plan_shared_by_streams(M, ctx):
    """The context keeps one transform plan per length; calls on two streams
    in flight together (each with its own work area) give the results of
    calls made one at a time."""
    import torch

    N, dt = 12288, 5.0
    xs = [I.rng_for(10, k).normal(size=(3, N)) for k in range(2)]
    want = [OI.tdi_to_aet_fd(x, dt, 0.0, 1, N // 2, 0.05) for x in xs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ins = [_t(x) for x in xs]
    torch.cuda.synchronize()
    outs = [torch.empty((3, N // 2), dtype=torch.complex128, device="cuda") for _ in xs]
    for rep in range(3):
        for x, o, st in zip(ins, outs, streams):
            M.tdi_to_aet_fd(ctx, x, dt, 0.0, 1, N // 2, 0.05, stream=st, out=o)
        torch.cuda.synchronize()
        for o, w in zip(outs, want):
            assert np.abs(o.cpu().numpy() - w).max() < 1e-12 * np.abs(w).max(), rep


def test_ingest_rejects_bad_arguments(M, ctx):
    xyz = _t(np.zeros((3, 1000)))
    for args in ((5.0, 0.0, 0, 10, 0.0), (5.0, 0.0, 1, 501, 0.0), (-1.0, 0.0, 1, 10, 0.0), (5.0, 0.0, 1, 10, 1.5),
                 (5.0, 0.0, 1, 1, 0.0)):
        with pytest.raises(M.MbhError):
            M.tdi_to_aet_fd(ctx, xyz, *args[:4], alpha=args[4])


def test_ingested_data_give_the_frequency_domain_likelihood(M, ctx):
    import torch

    dt = 50.0
    n = int(round(I.YEAR_S / dt))
    g = I.grid_lisa(1.0, dt, n_keep=n // 2 - 1)  # f_k = k / (N dt), k = 1 .. N/2 - 1
    rng = I.rng_for(9, 1)
    th, _ = I.draw_mbhb_source(rng, g.t_obs)
    th[0] = 1.5e6
    psd = I.psd_lisa_aet(g.freqs)
    h = O.template(O.MODEL_IMR, O.MODE_22, th, g.freqs, g.t_obs)
    th[4] = I.distance_for_snr(O.inner(h, h, psd, g.df), 300.0)
    d = O.template(O.MODEL_IMR, O.MODE_22, th, g.freqs, g.t_obs) + I.noise(psd, g.df, rng)
    xyz = OI.xyz_time_series(d, n, dt, 0.0, 1)
    # the oracle's own round trip
    assert np.abs(OI.tdi_to_aet_fd(xyz, dt, 0.0, 1, g.n_f) - d).max() < 1e-10 * np.abs(d).max()
    gfd = M.data_create(ctx, _t(d), _t(psd), g.f0, g.df, g.t_obs)
    gtd = M.data_create_tdi(ctx, _t(xyz), dt, 0.0, 1, g.n_f, _t(psd), g.t_obs)
    assert gtd.f0 == g.f0 and gtd.df == g.df and gtd.n_f == g.n_f
    dd_fd, dd_td = gfd.inner_dd(), gtd.inner_dd()
    print(f"[ingest] <d|d> frequency-domain {dd_fd:.10e} ingested {dd_td:.10e}", flush=True)
    assert abs(dd_fd - dd_td) <= 1e-10 * dd_fd
    data = O.Data(d, psd, g.f0, g.df, g.t_obs)
    ref = O.Reference(O.MODEL_IMR, O.MODE_22, th, data, 128)
    w = I.walker_cloud(th, I.curvature_sigma(lambda x: ref.loglike(x)[0], th), (1, 4), 8, rng)
    tw = _t(w)
    l_fd = M.loglike_full(ctx, gfd, M.MODEL_IMR, M.MODE_22, tw, M.FP64).cpu().numpy()
    l_td = M.loglike_full(ctx, gtd, M.MODEL_IMR, M.MODE_22, tw, M.FP64).cpu().numpy()
    assert np.all(np.abs(l_td - l_fd) <= 1e-6 + 1e-12 * np.abs(l_fd))
    l_or, _, _ = O.loglike_full(O.MODEL_IMR, O.MODE_22, w[:4], data)
    assert np.all(np.abs(l_td[:4] - l_or) <= 1e-6 + 1e-12 * np.abs(l_or))
    r_fd = M.build_reference_coeffs(ctx, gfd, M.MODEL_IMR, M.MODE_22, th, 128)
    r_td = M.build_reference_coeffs(ctx, gtd, M.MODEL_IMR, M.MODE_22, th, 128)
    h_fd = M.loglike_heterodyned(ctx, r_fd, tw, M.FP64).cpu().numpy()
    h_td = M.loglike_heterodyned(ctx, r_td, tw, M.FP64).cpu().numpy()
    print(f"[ingest] max |lnL ingested - frequency-domain|: full {np.abs(l_td - l_fd).max():.2e}, "
          f"heterodyned {np.abs(h_td - h_fd).max():.2e}", flush=True)
    assert np.all(np.abs(h_td - h_fd) <= 1e-6 + 1e-12 * np.abs(h_fd))
    for x in (r_fd, r_td, gfd, gtd):
        x.close()
    torch.cuda.synchronize()
