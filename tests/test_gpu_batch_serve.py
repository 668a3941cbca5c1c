"""Batching (one device-resident work list over ragged items, replayed as a graph
or as stream launches) and
serving (continuous batching), checked against single calls and the oracle.

Every walker's result depends only on its inputs, its reference and the lanes
per walker of its reference's shape, so results must be bit-identical between
a single call, a batch, a graph replay and any serving mix; a subsample is also
checked against the FP64 oracle to the 1e-3 bar.
"""
import numpy as np
import pytest

import oracle as O
from paper_2111_01064_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-3


@pytest.fixture(scope="module")
def M():
    from paper_2111_01064_amd import mbh

    return mbh


@pytest.fixture(scope="module")
def ctx(M):
    return M.Context(0)


def _t(x):
    import torch

    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.fixture(scope="module")
def sources(M, ctx):
    """Sixteen sources on a coarse grid with ragged modes, bin and walker counts."""
    import torch

    g = I.grid_lisa_small(8192, 0.05)
    shapes = I.batch_shapes(I.rng_for(4, 0), 16)
    out = []
    for s, (modes, nb, W) in enumerate(shapes):
        rng = I.rng_for(4, 1 + s)
        th, snr = I.draw_mbhb_source(rng, g.t_obs)
        th[0] = float(np.exp(rng.uniform(np.log(3e5), np.log(5e6))))
        psd = I.psd_lisa_aet(g.freqs)
        h = O.template(O.MODEL_IMR, modes, th, g.freqs, g.t_obs)
        th[4] = I.distance_for_snr(O.inner(h, h, psd, g.df), min(snr, 300.0))
        d = O.template(O.MODEL_IMR, modes, th, g.freqs, g.t_obs) + I.noise(psd, g.df, rng)
        data = O.Data(d, psd, g.f0, g.df, g.t_obs)
        ref = O.Reference(O.MODEL_IMR, modes, th, data, nb)
        if ref.status != O.OK:
            continue
        sig = I.curvature_sigma(lambda x: ref.loglike(x)[0], th)
        w = I.walker_cloud(th, sig, (1, 4, 16), (W + 2) // 3, rng)[:W]
        gd = M.data_create(ctx, torch.as_tensor(d, device="cuda"), torch.as_tensor(psd, device="cuda"), g.f0, g.df,
                           g.t_obs)
        gr = M.build_reference_coeffs(ctx, gd, M.MODEL_IMR, modes, th, nb)
        out.append(dict(modes=modes, nb=nb, W=W, th=th, ref=ref, walkers=w, gdata=gd, gref=gr))
    assert len(out) >= 12
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_graph_replays_match_single_calls_and_oracle(M, ctx, sources, prec):
    import torch

    p = M.FP64 if prec == "fp64" else M.MIXED
    thetas = [_t(s["walkers"]) for s in sources]
    lnls = [torch.empty(s["W"], dtype=torch.float64, device="cuda") for s in sources]
    dhs = [torch.empty((s["W"], 2), dtype=torch.float64, device="cuda") for s in sources]
    batch = M.Batch(ctx, [s["gref"] for s in sources], thetas, lnls, dhs, prec=p)
    single = [M.loglike_heterodyned(ctx, s["gref"], t, p).cpu().numpy() for s, t in zip(sources, thetas)]
    for rep in range(3):
        if rep == 2:  # walkers move between replays: the graph reads theta in place
            for s, t in zip(sources, thetas):
                t[:, 10] += 0.5
            single = [M.loglike_heterodyned(ctx, s["gref"], t, p).cpu().numpy() for s, t in zip(sources, thetas)]
        for l in lnls:
            l.fill_(np.nan)
        batch.launch()
        torch.cuda.synchronize()
        _ = torch.randn(1000, device="cuda").sum().item()  # eager work between replays
        for s, l, ref_single in zip(sources, lnls, single):
            got = l.cpu().numpy()
            assert np.array_equal(got, ref_single), (s["modes"], s["nb"], s["W"])
    # the three stages launched one by one are the same work
    for l in lnls:
        l.fill_(np.nan)
    for stage in (M.STAGE_SETUP, M.STAGE_MAIN, M.STAGE_FINISH):
        batch.launch_stage(stage)
    torch.cuda.synchronize()
    for l, ref_single in zip(lnls, single):
        assert np.array_equal(l.cpu().numpy(), ref_single)
    # stream launches of the same work (no graph) agree bit for bit
    for l in lnls:
        l.fill_(np.nan)
    batch.launch_direct()
    torch.cuda.synchronize()
    for l, ref_single in zip(lnls, single):
        assert np.array_equal(l.cpu().numpy(), ref_single)
    # oracle parity on a subsample of every item (last positions)
    worst = 0.0
    for s, t, l in zip(sources, thetas, lnls):
        idx = np.linspace(0, s["W"] - 1, 12).astype(int)
        ref_l, _, _ = s["ref"].loglike(t.cpu().numpy()[idx])
        err = np.abs(l.cpu().numpy()[idx] - ref_l)
        worst = max(worst, err.max())
        assert np.all(err <= TOL), (s["modes"], s["nb"], err.max())
    print(f"[batch] {prec}: {len(sources)} items, {sum(s['W'] for s in sources)} walkers, oracle max|dlnL| {worst:.2e}")


def test_batch_per_item_precision_matches_single_calls(M, ctx, sources):
    """mbh_batch_create_prec: items of one batch in different precisions, each
    bit-identical to a single call in its own precision (replay and stream
    launches); a per-mode-free batch only, and a bad precision is refused."""
    import torch

    precs = [M.MIXED if i % 3 else M.FP64 for i in range(len(sources))]
    thetas = [_t(s["walkers"]) for s in sources]
    lnls = [torch.empty(s["W"], dtype=torch.float64, device="cuda") for s in sources]
    dhs = [torch.empty((s["W"], 2), dtype=torch.float64, device="cuda") for s in sources]
    batch = M.Batch(ctx, [s["gref"] for s in sources], thetas, lnls, dhs, precs=precs)
    single = [M.loglike_heterodyned(ctx, s["gref"], t, p).cpu().numpy() for s, t, p in zip(sources, thetas, precs)]
    for launch in (batch.launch, batch.launch_direct, batch.launch):
        for l in lnls:
            l.fill_(np.nan)
        launch()
        torch.cuda.synchronize()
        for s, l, want, p in zip(sources, lnls, single, precs):
            assert np.array_equal(l.cpu().numpy(), want), (p, s["modes"], s["nb"], s["W"])
    with pytest.raises(M.MbhError):
        M.Batch(ctx, [sources[0]["gref"]], thetas[:1], lnls[:1], precs=[7])
    print(f"[batch] per-item precision: {sum(p == M.MIXED for p in precs)} mixed, "
          f"{sum(p == M.FP64 for p in precs)} FP64 items, bit-identical to single calls", flush=True)


def test_server_alone_equals_mix_and_backpressure(M, ctx, sources):
    import time

    refs = [s["gref"] for s in sources[:4]]
    srv = M.Server(ctx, refs, max_inflight=2, max_batch_walkers=8192, hbm_budget_bytes=64 << 20, prec=M.MIXED)
    rng = I.rng_for(5, 0)
    probe = sources[1]["walkers"][:37]
    rid = srv.submit(1, probe)
    alone, lat = srv.wait(rid, len(probe))
    assert lat > 0
    single = M.loglike_heterodyned(ctx, refs[1], _t(probe), M.MIXED).cpu().numpy()
    assert np.array_equal(alone, single)
    # a burst of requests with the probe in the middle
    reqs = []
    for k in range(60):
        src = int(rng.integers(0, 4))
        W = int(np.clip(np.rint(np.exp(rng.uniform(0, np.log(2000)))), 1, 2000))
        pool = sources[src]["walkers"]
        th = pool[rng.integers(0, len(pool), W)]
        reqs.append((src, th, srv.submit(src, th)))
        if k == 30:
            reqs.append((1, probe, srv.submit(1, probe)))
    for src, th, r in reqs:
        out, lat = srv.wait(r, len(th))
        ref = M.loglike_heterodyned(ctx, refs[src], _t(th), M.MIXED).cpu().numpy()
        assert np.array_equal(out, ref)
    st = srv.stats()
    assert st["completed"] == st["submitted"] == len(reqs) + 1
    assert st["batches"] < st["submitted"]  # requests were batched together
    srv.close()

    # a budget that fits ~600-900 walkers per slot (the per-walker footprint
    # includes the partial sums, up to ~1.2 kB at 512 bins): work queues,
    # nothing fails
    small = M.Server(ctx, refs, max_inflight=2, max_batch_walkers=8192, hbm_budget_bytes=2 * 600 * 1200,
                     prec=M.FP64)
    ids = [(small.submit(0, sources[0]["walkers"][:500]), 500) for _ in range(6)]
    for r, W in ids:
        out, _ = small.wait(r, W)
        assert np.all(np.isfinite(out))
    st = small.stats()
    assert st["max_walkers_in_flight"] <= 2 * 900
    with pytest.raises(M.MbhError) as e:
        small.submit(0, sources[0]["walkers"][:1000])
    assert e.value.status == M.MBH_EAGAIN
    small.close()


def test_server_replay_and_wait_capacity(M, ctx, sources):
    """A Poisson trace replayed from native threads (mbh_server_replay): every
    result equals the single call on the same walkers bit for bit, latencies
    are positive; mbh_server_wait refuses output buffers smaller than the
    request."""
    import ctypes as ct

    refs = [s["gref"] for s in sources[:4]]
    srv = M.Server(ctx, refs, max_inflight=3, max_batch_walkers=16384, hbm_budget_bytes=256 << 20, prec=M.MIXED)
    rng = I.rng_for(5, 2)
    trace = I.poisson_requests(rng, 200, 20000.0, 64, 4, 512)
    pools = [sources[k]["walkers"] for k in range(4)]
    rows, theta = [], []
    off = 0
    for (_, _, src, W) in trace:
        sel = pools[src][rng.integers(0, len(pools[src]), W)]
        theta.append(sel)
        rows.append(off)
        off += W
    theta = np.concatenate(theta)
    out = srv.replay([t for (t, _, _, _) in trace], [src for (_, _, src, _) in trace],
                     [W for (_, _, _, W) in trace], rows, theta, want_lnL=True)
    assert np.all(out["latency_s"] > 0) and np.all(np.isfinite(out["latency_s"]))
    assert out["wall_s"] > 0
    k = 0
    for (t, _, src, W), r0 in zip(trace, rows):
        ref = M.loglike_heterodyned(ctx, refs[src], _t(theta[r0:r0 + W]), M.MIXED).cpu().numpy()
        assert np.array_equal(out["lnL"][k:k + W], ref)
        k += W
    print(f"[serve] replay of {len(trace)} requests: p50 {np.percentile(out['latency_s'], 50) * 1e3:.3f} ms, "
          f"p99 {np.percentile(out['latency_s'], 99) * 1e3:.3f} ms, wall {out['wall_s']:.3f} s", flush=True)
    # output capacity below the request's walker count: refused, the request kept
    rid = srv.submit(0, pools[0][:10])
    buf = np.zeros(9)
    lat = ct.c_double()
    st = M._L.mbh_server_wait(srv.h, rid, -1, buf.ctypes.data_as(M._dp), None, 9, ct.byref(lat))
    assert st == M.MBH_EINVAL
    res, _ = srv.wait(rid)
    assert res.shape == (10,) and np.all(np.isfinite(res))
    st = srv.stats()
    assert st["completed"] == st["submitted"] == len(trace) + 1
    srv.close()


def test_autotuner_records_a_valid_choice(M, ctx, sources, tmp_path):
    s = sources[0]
    lanes = M.autotune_heterodyned(ctx, s["gref"], _t(s["walkers"]), M.MIXED)
    assert lanes in (0, 16, 32, 64)
    assert M.autotune_heterodyned(ctx, s["gref"], 2048, M.FP64) in (0, 16, 32, 64)
    nm = bin(s["modes"]).count("1")
    assert M.lanes_for(ctx, s["nb"], nm, M.MIXED) == lanes
    path = str(tmp_path / "lanes.txt")
    M.autotune_save(ctx, path)
    ctx2 = M.Context(0)
    M.autotune_load(ctx2, path)
    assert M.lanes_for(ctx2, s["nb"], nm, M.MIXED) == lanes


def test_batch_without_walkers_is_refused(M, ctx, sources):
    """A batch whose items all hold zero walkers is refused at creation (it
    would have no walker tile for the setup and totals kernels to read);
    one empty item among others is fine."""
    import torch

    s = sources[0]
    empty = torch.empty((0, 11), dtype=torch.float64, device="cuda")
    out = torch.empty(0, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MbhError) as e:
        M.Batch(ctx, [s["gref"], sources[1]["gref"]], [empty, empty], [out, out], prec=M.FP64)
    assert e.value.status == M.MBH_EINVAL
    tw = _t(s["walkers"][:5])
    lnl = torch.empty(5, dtype=torch.float64, device="cuda")
    b = M.Batch(ctx, [sources[1]["gref"], s["gref"]], [empty, tw], [out, lnl], prec=M.FP64)
    b.launch()
    torch.cuda.synchronize()
    single = M.loglike_heterodyned(ctx, s["gref"], tw, M.FP64).cpu().numpy()
    assert np.array_equal(lnl.cpu().numpy(), single)
    b.close()
