"""The no-allocation heterodyned entry point (mbh_loglike_heterodyned_noalloc)
against the allocating one (mbh_loglike_heterodyned), through the C ABI.

Both run the same kernels on the same inputs, so their results must be
identical bit for bit; the allocating entry point is itself held to the
oracle by the parity tests.  Two calls in a row, the second with fewer
walkers (the shared device array then holds the first call's contents), in
both precisions, with and without <d|h>, <h|h>; and a call above the
scratch maximum is refused before any work is issued.
"""
import numpy as np
import pytest

import oracle as O
from paper_2111_01064_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    import torch

    from paper_2111_01064_amd import mbh as M

    g = I.grid_lisa_small(16384, 0.05)
    rng = I.rng_for(2, 3)
    th, _ = I.draw_mbhb_source(rng, g.t_obs)
    psd = I.psd_lisa_aet(g.freqs)
    h = O.template(O.MODEL_IMR, O.MODE_22, th, g.freqs, g.t_obs)
    th[4] = I.distance_for_snr(O.inner(h, h, psd, g.df), 400.0)
    d = O.template(O.MODEL_IMR, O.MODE_22, th, g.freqs, g.t_obs) + I.noise(psd, g.df, rng)
    oref = O.Reference(O.MODEL_IMR, O.MODE_22, th, O.Data(d, psd, g.f0, g.df, g.t_obs), 128)
    sig = I.curvature_sigma(lambda x: oref.loglike(x)[0], th)
    w = I.walker_cloud(th, sig, (1, 4, 16, 64), 128, rng)
    ctx = M.Context(0)
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")
    gd = M.data_create(ctx, dev(d, torch.complex128), dev(psd, torch.float64), g.f0, g.df, g.t_obs)
    gr = M.build_reference_coeffs(ctx, gd, M.MODEL_IMR, M.MODE_22, th, 128)
    return dict(M=M, ctx=ctx, gd=gd, gr=gr, w=w, dev=dev)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("want_dh", [False, True])
def test_noalloc_matches_allocating_entry_point(case, prec, want_dh):
    import torch

    M, ctx, gr, w = case["M"], case["ctx"], case["gr"], case["w"]
    for W in (len(w), 37):  # the second call is smaller than the first
        tw = case["dev"](w[:W], torch.float64)
        dh_ref = torch.empty((W, 2), dtype=torch.float64, device="cuda") if want_dh else None
        ref = M.loglike_heterodyned(ctx, gr, tw, prec, dh_hh=dh_ref)
        got_l = torch.full((W,), np.nan, dtype=torch.float64, device="cuda")
        got_dh = torch.full((W, 2), np.nan, dtype=torch.float64, device="cuda") if want_dh else None
        M.loglike_heterodyned_noalloc(ctx, gr, tw, got_l, prec, dh_hh=got_dh)
        torch.cuda.synchronize()
        a, b = got_l.cpu().numpy(), ref.cpu().numpy()
        print(f"[noalloc] prec={prec} dh={want_dh} W={W}: max|diff|={np.abs(a - b).max():.3e}", flush=True)
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b)
        if want_dh:
            assert np.array_equal(got_dh.cpu().numpy(), dh_ref.cpu().numpy())


def test_noalloc_refuses_calls_above_the_maximum(case):
    import torch

    M, ctx, gr = case["M"], case["ctx"], case["gr"]
    W = 40000  # 40000 x (568 + 32 x 4) bytes > 24 MiB at 128 bins
    tw = torch.zeros((W, 11), dtype=torch.float64, device="cuda")
    out = torch.zeros(W, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MbhError) as e:
        M.loglike_heterodyned_noalloc(ctx, gr, tw, out, M.FP64)
    assert e.value.status == M.MBH_EINVAL
    assert "maximum" in str(e.value)
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0  # nothing was written
