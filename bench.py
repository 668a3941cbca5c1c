#!/usr/bin/env python3
"""Benchmark of the heterodyned MBHB likelihood on one MI355X.

Workload (one step): heterodyned lnL of 8 sources x (8 temperatures x 64
walkers) = 4096 walkers against their references, (2,2) IMR-lite + LISA TDI
A/E/T, 1 yr at dt = 10 s (1 577 880 Fourier bins, 3 channels), 128 bins,
SNR log-uniform in [100, 1000], seeded synthetic noise; evaluated as one
device-resident batch (mbh_batch) launched on a stream per step (its graph
replay is timed beside it).  The timed value is the
mixed-precision path; the plain-FP64 path is timed the same way and reported
beside it, together with the largest |dlnL| between the two.

Also measured (not part of the step): the full-grid likelihood on a prior-draw
sweep, the reference build, a higher-mode ragged 16-source batch, and a
Poisson request stream through the continuous-batching server (p50/p99).
The CPU baseline is the FP64 oracle timed on a bounded sample on the host.

Prints ONE JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2111_01064_amd import inputs as I  # noqa: E402

METRIC = "heterodyned lnL evals/s (mixed vs FP64, |ΔlnL|≤1e-3); p50/p99 request latency"
PEAK_ALU_TFLOPS = 78.6   # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, unpacked FP32 and FP64 alike
PEAK_HBM_GBS = 8000.0
N_SOURCES, TEMPS, PER_TEMP, N_BINS = 8, tuple(2.0 ** k for k in range(8)), 64, 128
# Algorithmic work of one heterodyned evaluation (roofline "achieved"): the
# per-unit figure of the measurement plan, 5e4 flops per evaluation for the
# (2,2) mode, three channels and 129 bin edges (waveform ~60 flops, response
# ~200 flops and ~13 transcendentals per edge, contraction ~30 per bin;
# transcendental = 1 flop, FMA = 2); the design notes derive it.  The bytes
# an evaluation must move are its 11 parameters in and one lnL out (96 B).
ALGO_FLOPS_PER_EVAL = 5.0e4
ALGO_BYTES_PER_EVAL = 96.0
# Algorithmic work of the full-grid likelihood per (walker, grid point): the
# template (~250 flops and ~15 transcendentals for (2,2) and three channels)
# and the residual contraction; the data and weights (32 B per point) are
# read once per walker tile.
ALGO_FULL_FLOPS_PER_POINT = 250.0
# Hardware counter figures of the current kernels (rocprofv3): VALU flops per
# (walker, edge) of the mixed main pass (SQ_INSTS_VALU_FLOPS_* x 64 lanes,
# FMA = 2), VALU flops per (walker, point) of the FP64 full grid, and HBM
# bytes per launch of the mixed main pass (FETCH_SIZE and WRITE_SIZE divided by
# their reading for a 64 MiB device copy: factors 0.5002 and 1.000).  Valid
# only for the kernel sources they were measured on (sha256 over
# KERNEL_SOURCES); reported as null otherwise.
COUNTERS = {"src_sha256": "17bbbc549db901cc88ac28f6f2325a6d2a5d878639a571fba0855cc90e2ce08d",
            "valu_flops_per_edge": 850.7, "full_valu_flops_per_point": 504.7, "bytes_per_launch": 5.495e6}


# the sources that define the device code of the main pass and the order
# its tiles are launched in (which sets what each XCD's L2 holds)
KERNEL_SOURCES = ("mbh_device.hpp", "mbh_kernels.hpp", "mbh_work.hpp", "mbh_serve.hip")


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2111_01064_amd", "csrc")
    for fn in KERNEL_SOURCES:
        with open(os.path.join(d, fn), "rb") as f:
            h.update(fn.encode() + b"\0" + f.read())
    return h.hexdigest()


def walker_segments(W: int, E: int, lanes: int) -> int:
    """Partial-sum segments of W walkers with E bin edges: the 63-bin chunks
    each walker's bins touch (flattened mapping) or one per walker."""
    if lanes:
        return W
    return sum((w * E + E - 2) // 63 - (w * E) // 63 + 1 for w in range(W))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Sources:
    """Synthetic LISA sources built through the library (no oracle)."""

    def __init__(self, M, ctx, grid, n_sources, modes_list=None, n_bins_list=None, snr_cap=None, cfg=2):
        import torch

        self.M, self.ctx, self.grid = M, ctx, grid
        f = grid.freqs
        self.psd = torch.as_tensor(I.psd_lisa_aet(f), device="cuda")
        zeros = torch.zeros((3, grid.n_f), dtype=torch.complex128, device="cuda")
        grid_data = M.data_create(ctx, zeros, self.psd, grid.f0, grid.df, grid.t_obs)
        self.items = []
        for s in range(n_sources):
            rng = I.rng_for(cfg, s)
            th, snr = I.draw_mbhb_source(rng, grid.t_obs)
            if snr_cap:
                snr = min(snr, snr_cap)
            modes = modes_list[s] if modes_list else M.MODE_22
            nb = n_bins_list[s] if n_bins_list else N_BINS
            h = M.template_full(ctx, grid_data, M.MODEL_IMR, modes, th)
            # <h|h> at D_L = 1 Gpc through the library's own full-grid kernel
            dsig = M.data_create(ctx, h, self.psd, grid.f0, grid.df, grid.t_obs)
            dh = torch.empty((1, 2), dtype=torch.float64, device="cuda")
            M.loglike_full(ctx, dsig, M.MODEL_IMR, modes, torch.as_tensor(th[None, :], device="cuda"), M.FP64,
                           dh_hh=dh)
            hh1 = float(dh[0, 1])
            dsig.close()
            th[4] = I.distance_for_snr(hh1, snr)
            noise = torch.as_tensor(I.noise(I.psd_lisa_aet(f), grid.df, rng), device="cuda")
            d = h * (1.0 / th[4]) + noise
            del h, noise
            data = M.data_create(ctx, d, self.psd, grid.f0, grid.df, grid.t_obs)
            ref = M.build_reference_coeffs(ctx, data, M.MODEL_IMR, modes, th, nb)
            self.items.append(dict(th=th, snr=snr, data=data, ref=ref, modes=modes, nb=nb, rng=rng, d=d))
        grid_data.close()

    def walkers(self, item, temps, per_temp):
        import torch

        M, ctx = self.M, self.ctx

        def het(x):
            return M.loglike_heterodyned(ctx, item["ref"], torch.as_tensor(x, device="cuda"), M.FP64).cpu().numpy()

        sig = I.curvature_sigma(het, item["th"])
        w = I.walker_cloud(item["th"], sig, temps, per_temp, item["rng"])
        return w


def time_batch(M, ctx, batch, steps, warmup, stream, mode="direct"):
    """Wall time of `steps` batch launches queued back to back on `stream`
    (bracketed by device synchronisation), and the device time between two
    events around them, per step.  mode: "direct" (mbh_batch_launch_direct:
    stream launches) or "graph" (mbh_batch_launch: one graph replay)."""
    import torch

    fn = batch.launch_direct if mode == "direct" else batch.launch
    for _ in range(warmup):
        fn(stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        a.record(stream)
        for _ in range(steps):
            fn(stream)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, a.elapsed_time(b) * 1e-3 / steps


def time_stage(batch, stage, steps, stream):
    """Mean duration of one stage of the batch (mbh_batch_launch_stage):
    `steps` launches queued back to back between two events on the launch
    stream, so that the host-side launch latency overlaps the device work;
    the stage's inputs come from a preceding full launch."""
    import torch

    batch.launch(stream)
    for _ in range(3):
        batch.launch_stage(stage, stream)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        a.record(stream)
        for _ in range(steps):
            batch.launch_stage(stage, stream)
        b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) * 1e-3 / steps


def copy_calibration():
    """A plain device copy of 64 MiB (read 64 MiB, write 64 MiB), run so that
    HBM byte counters can be scaled against a kernel of known traffic."""
    import torch

    src = torch.ones(8 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


LOUDEST_SOURCE = 1  # the step's loudest source (SNR ~950)


def cpu_baseline(M, ctx, budget_s: float = 15.0):
    """The FP64 oracle (OpenMP over walkers) on one source of the step's
    workload, its loudest: its own data, reference and walker cloud (the
    step's seed and recipe, built by the oracle), timed on the host.  The
    library then evaluates the same oracle-made walkers on the same data
    (one batch, launched as the step is, in both precisions) and the largest
    |dlnL| against the oracle is reported."""
    import torch

    import oracle as O

    g = I.grid_lisa()
    rng = I.rng_for(2, LOUDEST_SOURCE)
    th, snr = I.draw_mbhb_source(rng, g.t_obs)
    f = g.freqs
    psd = I.psd_lisa_aet(f)
    t0 = time.perf_counter()
    h = O.template(O.MODEL_IMR, O.MODE_22, th, f, g.t_obs)
    th[4] = I.distance_for_snr(O.inner(h, h, psd, g.df), snr)
    d = h / th[4] + I.noise(psd, g.df, rng)
    del h
    data = O.Data(d, psd, g.f0, g.df, g.t_obs)
    ref = O.Reference(O.MODEL_IMR, O.MODE_22, th, data, N_BINS)
    sig = I.curvature_sigma(lambda x: ref.loglike(x)[0], th)
    w = I.walker_cloud(th, sig, TEMPS, PER_TEMP, rng)
    setup_s = time.perf_counter() - t0
    n_done, t_start = 0, time.perf_counter()
    while time.perf_counter() - t_start < budget_s:
        lo, _, _ = ref.loglike(w)
        n_done += len(w)
    el = time.perf_counter() - t_start
    # the same on one core (a shorter sample)
    n_threads = O.max_threads()
    O.set_threads(1)
    n1, t1s = 0, time.perf_counter()
    while time.perf_counter() - t1s < budget_s / 5:
        ref.loglike(w)
        n1 += len(w)
    single = n1 / (time.perf_counter() - t1s)
    O.set_threads(n_threads)
    # one full-grid evaluation for the per-evaluation cost of the direct likelihood
    t1 = time.perf_counter()
    O.loglike_full(O.MODEL_IMR, O.MODE_22, w[: O.max_threads()], data)
    full_s = (time.perf_counter() - t1) / O.max_threads()
    # the library on the oracle's inputs
    gd = M.data_create(ctx, torch.as_tensor(d, device="cuda"), torch.as_tensor(psd, device="cuda"), g.f0, g.df,
                       g.t_obs)
    gr = M.build_reference_coeffs(ctx, gd, M.MODEL_IMR, M.MODE_22, th, N_BINS)
    tw = torch.as_tensor(w, device="cuda")
    vs_oracle = {}
    for name, prec in (("fp64", M.FP64), ("mixed", M.MIXED)):
        lb = torch.empty(len(w), dtype=torch.float64, device="cuda")
        b = M.Batch(ctx, [gr], [tw], [lb], prec=prec)
        b.launch_direct()
        torch.cuda.synchronize()
        b.close()
        vs_oracle[name] = float(np.max(np.abs(lb.cpu().numpy() - lo)))
    gr.close()
    gd.close()
    return dict(value=n_done / el, unit="evals/s", cores=O.max_threads(), kind="oracle",
                sample=f"source {LOUDEST_SOURCE} of the step (SNR {snr:.0f}), {len(w)} walkers (8 temps x 64) "
                       f"x {n_done // len(w)} passes, 1.58e6-bin grid, 128 bins, {el:.1f} s",
                full_grid_s_per_eval_per_core=full_s * O.max_threads(), setup_s=setup_s,
                single_core_value=single, vs_oracle=vs_oracle, lnL_range=[float(lo.min()), float(lo.max())])


def chirp_case(M, ctx):
    """The single-channel 0PN chirp case (2^14 linear bins on [1e-4, 0.1] Hz,
    64 bins, 32 walkers at 1e-4 relative scatter), noiseless data and a
    seeded noisy variant: the oracle's heterodyned and full-grid lnL, their
    difference and CPU seconds, and the library's FP64 heterodyned lnL
    against the oracle's."""
    import torch

    import oracle as O

    out = {}
    for variant in ("noiseless", "noisy"):
        g = I.grid_chirp()
        rng = I.rng_for(1, 0)
        th = I.draw_chirp_source(rng)
        psd = I.psd_chirp(g.freqs)
        h = O.template(O.MODEL_TF2, 0, th, g.freqs, g.t_obs)
        th[1] = 100.0 / math.sqrt(O.inner(h, h, psd, g.df))
        d = O.template(O.MODEL_TF2, 0, th, g.freqs, g.t_obs)
        if variant == "noisy":
            d = d + I.noise(psd, g.df, rng)
        data = O.Data(d, psd, g.f0, g.df, g.t_obs)
        t0 = time.perf_counter()
        ref = O.Reference(O.MODEL_TF2, 0, th, data, 64)
        w = I.relative_cloud(th, 1e-4, 32, rng)
        w[:, 4:] = 0.0
        lh, _, _ = ref.loglike(w)
        t_het = time.perf_counter() - t0
        t0 = time.perf_counter()
        lf, _, _ = O.loglike_full(O.MODEL_TF2, 0, w, data)
        t_full = time.perf_counter() - t0
        gd = M.data_create(ctx, torch.as_tensor(np.atleast_2d(d), device="cuda"),
                           torch.as_tensor(np.atleast_2d(psd), device="cuda"), g.f0, g.df, g.t_obs)
        gr = M.build_reference_coeffs(ctx, gd, M.MODEL_TF2, 0, th, 64)
        lg = M.loglike_heterodyned(ctx, gr, torch.as_tensor(w, device="cuda"), M.FP64).cpu().numpy()
        gr.close()
        gd.close()
        out[variant] = dict(walkers=len(w), bins=64, grid=g.n_f,
                            max_abs_het_minus_full=float(np.max(np.abs(lh - lf))), oracle_het_s=t_het,
                            oracle_full_s=t_full, cores=O.max_threads(),
                            max_abs_gpu_fp64_minus_oracle_het=float(np.max(np.abs(lg - lh))))
    return out


def serve_run(M, ctx, refs, pools, prec, rate_hz, n_req, warm, update=None):
    """Poisson request stream replayed through the server by its native trace
    replay (mbh_server_replay: submission at the arrival times and collection
    in the library's own threads).  With update = (datas, lnls, every) a
    reference update of the request's source is queued (from Python, while
    the replay runs) at the arrival of every `every`-th request."""
    rng = I.rng_for(5, 1)
    reqs = I.poisson_requests(rng, n_req + warm, rate_hz, 64, len(refs), 4096)
    srv = M.Server(ctx, refs, max_inflight=3, max_batch_walkers=65536, hbm_budget_bytes=2 << 30, prec=prec)
    rows, theta, off = [], [], 0
    for (_, _, src, W) in reqs:
        pool = pools[src]
        theta.append(pool[rng.integers(0, len(pool), W)])
        rows.append(off)
        off += W
    theta = np.concatenate(theta)
    t_arr = [r[0] for r in reqs]
    result = {}

    def run():
        result["out"] = srv.replay(t_arr, [r[2] for r in reqs], [r[3] for r in reqs], rows, theta)

    th = threading.Thread(target=run)
    t0 = time.perf_counter()
    th.start()
    upd_ids = []
    if update is not None:
        for i in range(update[2] - 1, len(reqs), update[2]):
            while th.is_alive() and time.perf_counter() - t0 < t_arr[i]:
                time.sleep(0.0002)
            src = reqs[i][2]
            upd_ids.append(srv.refresh(src, update[0][src], pools[src], update[1][src]))
    th.join()
    if "out" not in result:
        raise RuntimeError("server replay failed")
    for u in upd_ids:
        srv.wait(u, 0)
    out_r = result["out"]
    st = srv.stats()
    srv.close()
    l = out_r["latency_s"][warm:] * 1e3
    walkers = sum(r[3] for r in reqs)
    wall = out_r["wall_s"]
    out = dict(p50_ms=float(np.percentile(l, 50)), p99_ms=float(np.percentile(l, 99)),
               throughput_evals_s=walkers / wall, requests_per_s=len(reqs) / wall, requests=n_req,
               rate_hz=rate_hz, achieved_over_offered=(len(reqs) / wall) / rate_hz, batches=st["batches"],
               mean_walkers_per_batch=st["walkers"] / max(1, st["batches"]),
               max_submit_lag_ms=float(out_r["submit_lag_s"].max() * 1e3))
    if update is not None:
        out["reference_updates"] = len(upd_ids)
        out["max_ms"] = float(l.max())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 2000 timed steps (~50 ms) after 200 warm-up steps: with 200 after 20 the
    # timed region (~5.5 ms) ends before the step reaches its steady rate
    # (measured 27.4 against 26.2 us per mixed step, 1.38e8 against 1.52e8
    # FP64 evals/s)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--quick", action="store_true", help="skip the side measurements")
    ap.add_argument("--mapping", type=int, default=None,
                    help="fix the heterodyned mapping (0 = flattened, or lanes per walker) instead of autotuning; "
                         "for profiler runs, whose timings would mislead the autotuner")
    ap.add_argument("--full-grid-only", type=int, default=0, metavar="DRAWS",
                    help="time only the full-grid likelihood on this many prior draws of the first source "
                         "(default tile, FP64; for profiler runs) and exit")
    ap.add_argument("--sampler-only", action="store_true",
                    help="run only the sampler search on the loudest source and exit (for profiler runs)")
    ap.add_argument("--ingest-only", action="store_true",
                    help="time only the TDI ingest (X, Y, Z -> A, E, T band) and exit (for profiler runs)")
    ap.add_argument("--hm-only", action="store_true",
                    help="time only the 16-source higher-mode batch (mode-summed and per-mode binning) and exit "
                         "(for profiler runs; with --mapping, no autotuning)")
    ap.add_argument("--mixed-tol", type=float, default=None,
                    help="estimated-error tolerance of the mixed path (library default 9e-4; inf: no FP64 "
                         "recomputation, 0: everything in FP64)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: every walker batch fits one MI355X and this build has no "
              "multi-GPU path (see the sharding notes in the design document)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2111_01064_amd import mbh as M

    ctx = M.Context(0)
    if args.mixed_tol is not None:
        M.set_mixed_tolerance(ctx, args.mixed_tol)
    grid = I.grid_lisa()
    if args.ingest_only:
        print(json.dumps(ingest_leg(M, ctx)))
        return
    if args.hm_only:
        print(json.dumps(hm_batch_leg(M, ctx, grid, args.mapping, method_error=False), default=float))
        return
    if args.sampler_only:
        S = Sources(M, ctx, grid, 2)
        print(json.dumps(sampler_search(M, ctx, S.items[1]), default=float))
        return
    if args.full_grid_only:
        S = Sources(M, ctx, grid, 1)
        draws = torch.as_tensor(I.prior_draws(I.rng_for(3, 0), args.full_grid_only, grid.t_obs), device="cuda")
        M.loglike_full(ctx, S.items[0]["data"], M.MODEL_IMR, M.MODE_22, draws[:64], M.FP64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            M.loglike_full(ctx, S.items[0]["data"], M.MODEL_IMR, M.MODE_22, draws, M.FP64)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        print(json.dumps({"metric": "full-grid lnL evals/s", "value": len(draws) / dt, "unit": "evals/s",
                          "draws": len(draws), "shape": list(M.full_shape(ctx, False)), "steps": args.steps}))
        return
    t0 = time.perf_counter()
    S = Sources(M, ctx, grid, N_SOURCES)
    log(f"[bench] built {N_SOURCES} sources on {grid.n_f} bins in {time.perf_counter() - t0:.1f} s")
    walkers = [S.walkers(it, TEMPS, PER_TEMP) for it in S.items]
    thetas = [torch.as_tensor(w, device="cuda") for w in walkers]
    W_total = sum(len(w) for w in walkers)
    stream = torch.cuda.Stream()
    res = {}
    for name, prec in (("fp64", M.FP64), ("mixed", M.MIXED)):
        # autotune the mapping for this shape once, on the step's own walkers
        if args.mapping is None:
            M.autotune_heterodyned(ctx, S.items[0]["ref"], torch.cat(thetas), prec)
        else:
            M.set_lanes(ctx, N_BINS, 1, prec, args.mapping)
        lnls = [torch.empty(len(w), dtype=torch.float64, device="cuda") for w in walkers]
        batch = M.Batch(ctx, [it["ref"] for it in S.items], thetas, lnls, prec=prec)
        wall, mean_s = time_batch(M, ctx, batch, args.steps, args.warmup, stream, "direct")
        fp64_segs = batch.fp64_segments() / (args.steps + args.warmup)
        res[name] = dict(wall=wall, kernel_s=mean_s, lnl=np.concatenate([l.cpu().numpy() for l in lnls]),
                         lanes=M.lanes_for(ctx, N_BINS, 1, prec), fp64_segs=fp64_segs)
        gwall, gmean = time_batch(M, ctx, batch, args.steps, args.warmup, stream, "graph")
        res[name]["graph_us"] = gwall / args.steps * 1e6
        stages = [time_stage(batch, st, max(20, args.steps // 4), stream)
                  for st in (M.STAGE_SETUP, M.STAGE_MAIN, M.STAGE_FINISH)]
        res[name]["stages_s"] = stages
        batch.close()
        res[name]["segments"] = sum(walker_segments(len(w), N_BINS + 1, res[name]["lanes"]) for w in walkers)
        log(f"[bench] {name}: {W_total} walkers/step, {wall / args.steps * 1e6:.1f} us/step "
            f"(graph replay {res[name]['graph_us']:.1f}), {mean_s * 1e6:.1f} us/step (events), wall {wall:.3f} s, "
            f"lanes {res[name]['lanes']}, FP64 segments/step {fp64_segs:.1f} of {res[name]['segments']}, "
            f"stages (us) "
            + " / ".join(f"{x * 1e6:.1f}" for x in stages))
    dmix = float(np.max(np.abs(res["mixed"]["lnl"] - res["fp64"]["lnl"])))
    # |dlnL| against the distance below each source's best walker
    dist = np.concatenate([l.max() - l for l in np.split(res["fp64"]["lnl"], np.cumsum([len(w) for w in walkers])[:-1])])
    dabs = np.abs(res["mixed"]["lnl"] - res["fp64"]["lnl"])
    by_dist = []
    for lo, hi in ((0, 10), (10, 100), (100, 1e3), (1e3, 1e4), (1e4, np.inf)):
        m = (dist >= lo) & (dist < hi)
        if m.any():
            by_dist.append({"below_max": [lo, None if np.isinf(hi) else hi], "walkers": int(m.sum()),
                            "max_abs_dlnL": float(dabs[m].max())})
    ms_per_step = res["mixed"]["wall"] / args.steps * 1e3
    value = W_total * args.steps / res["mixed"]["wall"]
    fp64_value = W_total * args.steps / res["fp64"]["wall"]
    E = N_BINS + 1
    flops = W_total * ALGO_FLOPS_PER_EVAL
    # the main pass's duration: its own launches back to back between two
    # events on the launch stream (the stage timing).  Also reported: the
    # step's time less the setup and totals stages, whose own back-to-back
    # timings are bound by the host's launch rate (a few microseconds per
    # launch for kernels that run about that long), so that this difference
    # reads short.
    def main_in_step(r):
        return r["wall"] / args.steps - r["stages_s"][0] - r["stages_s"][2]

    t_main = res["mixed"]["stages_s"][1]
    achieved = flops / t_main / 1e12
    counters_ok = COUNTERS["src_sha256"] == kernel_sources_hash()
    traffic = COUNTERS["bytes_per_launch"] if counters_ok else None
    hw_flops = W_total * E * COUNTERS["valu_flops_per_edge"] if counters_ok else None
    out = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64 (mixed)", "data": "synthetic",
        "config": {"workload": "8 sources x (8 temps x 64 walkers), (2,2) IMR-lite + TDI A/E/T, "
                               "1 yr dt=10 s (1577880 bins x 3 ch), 128 bins, SNR 100-1000, noisy",
                   "walkers_per_step": W_total, "n_bins": N_BINS,
                   "launch": "mbh_batch_launch_direct (work list resident, stream launches)"},
        "fp64_evals_per_s": fp64_value, "fp64_ms_per_step": res["fp64"]["wall"] / args.steps * 1e3,
        "mixed_speedup_vs_fp64": value / fp64_value, "max_abs_dlnL_mixed_vs_fp64": dmix,
        "dlnL_mixed_vs_fp64_by_distance": by_dist,
        "mixed_fp64_recomputed_fraction": res["mixed"]["fp64_segs"] / res["mixed"]["segments"],
        "mixed_tolerance": M.mixed_tolerance(ctx),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_ALU_TFLOPS, "traffic": traffic,
                     "kernel": "k_het_tiles<float> (main pass, mixed)", "kernel_us": t_main * 1e6,
                     "kernel_us_in_step": main_in_step(res["mixed"]) * 1e6,
                     "flops_per_launch": flops, "algorithmic_flops_per_eval": ALGO_FLOPS_PER_EVAL,
                     "frac_hw": (hw_flops / t_main / 1e12 / PEAK_ALU_TFLOPS) if hw_flops else None,
                     "algorithmic_bytes_per_launch": W_total * ALGO_BYTES_PER_EVAL,
                     "traffic_over_algorithmic": (traffic / (W_total * ALGO_BYTES_PER_EVAL)) if traffic else None},
        "stages_us": {k: {"setup": v["stages_s"][0] * 1e6, "main": v["stages_s"][1] * 1e6,
                          "finish": v["stages_s"][2] * 1e6, "step_events": v["kernel_s"] * 1e6,
                          "step_graph_replay": v["graph_us"]} for k, v in res.items()},
        "fp64_roofline_frac": flops / res["fp64"]["stages_s"][1] / 1e12 / PEAK_ALU_TFLOPS,
        "roofline_counters_current": counters_ok,
        "paper_context": {"het_evals_per_s": 2e5, "note": "~5 us per heterodyned lnL, unnamed GPU, PhenomD"},
    }
    copy_calibration()
    if not args.quick:
        out.update(side_measurements(M, ctx, S, walkers, grid))
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle) ...")
        cb = cpu_baseline(M, ctx)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["max_abs_dlnL_vs_oracle"] = {**cb["vs_oracle"], "source": LOUDEST_SOURCE, "walkers": len(TEMPS) * PER_TEMP,
                                         "oracle_lnL_range": cb["lnL_range"]}
        log(f"[bench] vs oracle (loudest source, 512 walkers): {out['max_abs_dlnL_vs_oracle']}")
        out["cpu_baseline_full_grid_s_per_eval_per_core"] = cb["full_grid_s_per_eval_per_core"]
        out["cpu_baseline_single_core_evals_per_s"] = cb["single_core_value"]
        out["chirp_case"] = chirp_case(M, ctx)
        log(f"[bench] chirp case: {out['chirp_case']}")
    print(json.dumps(out), flush=True)


def served_samplers(M, ctx, S5, refs, prec, n_iter=200, warm=5):
    """Samplers as clients of the request server (Sec. 3's search with its
    likelihood calls served, mbh_sampler_step_served): 16 tempered samplers on
    the 4 resident sources (sampler i on source i mod 4), 8 rungs (T_k = 2^k)
    of 8, 32, 128 or 512 walkers, so that each half step is one request of
    32, 128, 512 or 2048 walkers; each sampler runs in a thread of its own on
    its own stream, `warm` iterations, then n_iter timed."""
    import torch

    K, sizes, n_smp = 8, (8, 32, 128, 512), 16
    lo = np.array([math.log(1e5), 0.05, -0.99, -0.99, 1e-2, 0.0, -1.0, 0.0, -1.0, 0.0, 0.0])
    hi = np.array([math.log(1e8), 1.0, 0.99, 0.99, 1e3, 2 * math.pi, 1.0, 2 * math.pi, 1.0, math.pi,
                   S5.items[0]["data"].t_obs])
    betas = 1.0 / 2.0 ** np.arange(K)
    sigs = []
    for item in S5.items:
        sigs.append(I.curvature_sigma(lambda x, r=item["ref"]: M.loglike_heterodyned(
            ctx, r, torch.as_tensor(x, device="cuda"), M.FP64).cpu().numpy(), item["th"]))
    srv = M.Server(ctx, refs, max_inflight=3, max_batch_walkers=65536, hbm_budget_bytes=2 << 30, prec=prec)
    smps, Ws = [], []
    for i in range(n_smp):
        src, W = i % 4, sizes[(i // 4) % 4]
        item = S5.items[src]
        cloud = I.walker_cloud(item["th"], sigs[src], tuple(2.0 ** k for k in range(K)), W, I.rng_for(7, i))
        x0 = cloud.copy()
        x0[:, 0] = np.log(cloud[:, 0])
        x0[:, 6] = np.cos(cloud[:, 6])
        x0[:, 8] = np.sin(cloud[:, 8])
        smp = M.Sampler(ctx, betas, W, lo, hi, seed=20211101 + i, prec=prec)
        smp.set_walkers(np.clip(x0, lo, hi), M.Sampler.likelihood(ref=item["ref"]))
        smps.append(smp)
        Ws.append(W)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(n_smp)]
    res = {}

    def run(i, n):
        t0 = time.perf_counter()
        lat = smps[i].step_served(srv, i % 4, n, stream=streams[i])
        res[i] = (lat, time.perf_counter() - t0)

    def all_threads(n):
        th = [threading.Thread(target=run, args=(i, n)) for i in range(n_smp)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        if len(res) != n_smp:
            raise RuntimeError("a served sampler failed")

    all_threads(warm)
    res.clear()
    b0 = srv.stats()
    t0 = time.perf_counter()
    all_threads(n_iter)
    wall = time.perf_counter() - t0
    b1 = srv.stats()
    lat = np.concatenate([res[i][0] for i in range(n_smp)]) * 1e3
    evals = sum(n_iter * K * W for W in Ws)
    batches = b1["batches"] - b0["batches"]
    out = {"samplers": n_smp, "rungs": K, "request_walkers": [K * w // 2 for w in sizes], "iterations_each": n_iter,
           "wall_s": wall, "evals_per_s": evals / wall, "requests_per_s": 2 * n_iter * n_smp / wall,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "iteration_ms_median": float(np.median([res[i][1] / n_iter for i in range(n_smp)]) * 1e3),
           "requests_per_batch": 2 * n_iter * n_smp / max(1, batches)}
    for smp in smps:
        smp.close()
    srv.close()
    log(f"[bench] samplers as server clients ({'fp64' if prec == M.FP64 else 'mixed'}): {out}")
    return out


def ingest_leg(M, ctx, reps=20):
    """TDI X, Y, Z -> A, E, T band (Sec. 2.1) on the step's data grid: one
    year of samples at dt = 10 s (N = 3 155 760), the band k = 1 .. N/2 that
    the 1.58e6-bin grid holds; the plan is made by a first, untimed call.
    Algorithmic bytes: the three series read once (24 N) and the band written
    once (48 n_freq)."""
    import torch

    def run(n, dt, alpha):
        nf = n // 2
        g = torch.Generator(device="cuda").manual_seed(7)
        xyz = torch.randn((3, n), dtype=torch.float64, device="cuda", generator=g)
        st = torch.cuda.Stream()
        out = torch.empty((3, nf), dtype=torch.complex128, device="cuda")
        M.tdi_to_aet_fd(ctx, xyz, dt, 0.0, 1, nf, alpha, out=out, stream=st)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        for _ in range(reps):
            M.tdi_to_aet_fd(ctx, xyz, dt, 0.0, 1, nf, alpha, out=out, stream=st)
        b.record(st)
        torch.cuda.synchronize()
        sec = a.elapsed_time(b) * 1e-3 / reps
        gbs = (24.0 * n + 48.0 * nf) / sec * 1e-9
        return {"samples": n, "dt": dt, "band_bins": nf, "tukey_alpha": alpha, "ms_per_call": sec * 1e3,
                "algorithmic_GB_per_s": gbs, "frac_hbm": gbs / PEAK_HBM_GBS}

    n = int(round(I.YEAR_S / 10.0))  # 2^4 3^4 5 487: the transform takes rocFFT's Bluestein path
    res = {"year_dt10": run(n, 10.0, 0.0), "year_dt10_tukey0.1": run(n, 10.0, 0.1),
           # the same year in 2^22 samples, for the cost of the odd length
           "year_pow2": run(1 << 22, I.YEAR_S / (1 << 22), 0.0)}
    log(f"[bench] ingest: {res}")
    return res


def sampler_search(M, ctx, item, prec=None, mixed_rungs=0):
    import torch

    # FP64: at 2000 walkers per half-ensemble launch the heterodyned pass is
    # latency-bound, so FP32 gains nothing while hot rungs recompute many
    # segments in FP64 (measured: 87.7 us per iteration FP64, 110-123 mixed)
    prec = M.FP64 if prec is None else prec

    K, W = 10, 400
    lo = np.array([math.log(1e5), 0.05, -0.99, -0.99, 1e-2, 0.0, -1.0, 0.0, -1.0, 0.0, 0.0])
    hi = np.array([math.log(1e8), 1.0, 0.99, 0.99, 1e3, 2 * math.pi, 1.0, 2 * math.pi, 1.0, math.pi, item["data"].t_obs])
    th = item["th"]

    def het(x):
        return M.loglike_heterodyned(ctx, item["ref"], torch.as_tensor(x, device="cuda"), M.FP64).cpu().numpy()

    sig = I.curvature_sigma(het, th)
    cloud = I.walker_cloud(th, sig, tuple(4.0 ** k for k in range(K)), W, I.rng_for(2, 900))
    x0 = cloud.copy()
    x0[:, 0] = np.log(cloud[:, 0])
    x0[:, 6] = np.cos(cloud[:, 6])
    x0[:, 8] = np.sin(cloud[:, 8])
    x0 = np.clip(x0, lo, hi)
    ref = M.build_reference_coeffs(ctx, item["data"], M.MODEL_IMR, M.MODE_22, cloud[-1], N_BINS)
    like = M.Sampler.likelihood(ref=ref)
    betas = 1.0 / 1.6 ** np.arange(K)
    smp = M.Sampler(ctx, betas, W, lo, hi, seed=20211101, prec=prec, mixed_rungs=mixed_rungs)
    smp.set_walkers(x0, like)
    r = smp.run(like, check_every=150, lnl_tol=1.0, lnl_checks=30, refresh_every=1000, refresh_data=item["data"],
                max_iter=30000)
    st = smp.stats()
    # the best walker of the cold rung and the source, on the full grid
    fin = smp.get()
    xb = fin["x"][int(np.argmax(fin["lnL"][:W]))]
    tb = xb.copy()
    tb[0], tb[6], tb[8] = math.exp(xb[0]), math.acos(xb[6]), math.asin(xb[8])
    lf = M.loglike_full(ctx, item["data"], M.MODEL_IMR, M.MODE_22,
                        torch.as_tensor(np.stack([tb, th]), device="cuda"), M.FP64).cpu().numpy()
    acc = st["accepted"].astype(float)
    prop = np.maximum(st["proposed"].astype(float), 1.0)
    l_true = float(het(th[None, :])[0])
    out = dict(rungs=K, walkers_per_rung=W, precision="fp64" if prec == M.FP64 else "mixed",
               mixed_rungs=mixed_rungs, iterations=r["iterations"],
               stop={0: "max_iter", 1: "snr", 2: "converged"}[r["reason"]], reference_updates=r["refreshes"],
               seconds=r["seconds"], us_per_iteration=r["seconds"] / max(1, r["iterations"]) * 1e6,
               lnL_evals_per_s=2 * (K * W // 2) * r["iterations"] / r["seconds"],
               max_lnL=r["max_lnL"], lnL_at_source=l_true, best_extracted_snr=r["best_snr"],
               full_grid_lnL_best=float(lf[0]), full_grid_lnL_source=float(lf[1]),
               source_snr=item["snr"], cold_acceptance={"stretch": acc[0, 0] / prop[0, 0],
                                                        "sky_hops": acc[0, 1:].sum() / prop[0, 1:].sum()},
               swap_acceptance_cold_pair=float(st["swaps"][0]) / (W * max(1, r["iterations"])))
    smp.close()
    ref.close()
    log(f"[bench] sampler search: {out}")
    return out


def hm_batch_leg(M, ctx, grid, mapping=None, method_error=True):
    """Ragged higher-mode batch: 16 sources, modes 1-6, N_b 64-512, W
    128-4096, with the mode-summed ratio (both precisions) and with per-mode
    binning (FP64).  ``mapping`` fixes the mapping of every item instead of
    autotuning it (profiler runs); ``method_error`` adds the comparison with
    the full-grid likelihood on a walker subset."""
    import torch

    shapes = I.batch_shapes(I.rng_for(4, 0), 16)
    S4 = Sources(M, ctx, grid, 16, modes_list=[s[0] for s in shapes], n_bins_list=[s[1] for s in shapes], cfg=4)
    th4 = []
    for item, (_, _, W) in zip(S4.items, shapes):
        th4.append(torch.as_tensor(S4.walkers(item, (1, 4, 16, 64), (W + 3) // 4)[:W], device="cuda"))
    W4 = sum(len(t) for t in th4)
    hm = {"sources": 16, "walkers": W4, "shapes": [[int(m), int(nb), int(w)] for (m, nb, w) in shapes]}
    st = torch.cuda.Stream()
    lnl4 = {}
    for name, prec in (("fp64", M.FP64), ("mixed", M.MIXED)):
        chosen = []
        for it4, t4, sh in zip(S4.items, th4, shapes):
            if mapping is None:
                chosen.append(int(M.autotune_heterodyned(ctx, it4["ref"], t4, prec)))
            else:
                M.set_lanes(ctx, int(sh[1]), bin(int(sh[0])).count("1"), prec, mapping)
                chosen.append(mapping)
        # lanes per walker the autotuner picked per item (0 = flattened, one lane per walker and edge)
        hm[f"{name}_autotuned_lanes"] = chosen
        ln4 = [torch.empty(len(t), dtype=torch.float64, device="cuda") for t in th4]
        b4 = M.Batch(ctx, [x["ref"] for x in S4.items], th4, ln4, prec=prec)
        # 200 timed launches after 20 (steady state, as for the step)
        wall, mean_s = time_batch(M, ctx, b4, 200, 20, st)
        hm[f"{name}_evals_per_s"] = W4 * 200 / wall
        hm[f"{name}_us_per_launch"] = mean_s * 1e6
        hm[f"{name}_fp64_segments_per_launch"] = b4.fp64_segments() / 220
        lnl4[name] = np.concatenate([l.cpu().numpy() for l in ln4])
        b4.close()
        log(f"[bench] HM batch {name}: {W4} walkers, {W4 * 200 / wall:.3g} evals/s")
    hm["mixed_speedup_vs_fp64"] = hm["mixed_evals_per_s"] / hm["fp64_evals_per_s"]
    ok = np.isfinite(lnl4["fp64"])
    hm["max_abs_dlnL_mixed_vs_fp64"] = float(np.max(np.abs(lnl4["mixed"][ok] - lnl4["fp64"][ok])))
    # the same sources and walkers with per-mode relative binning (each mode
    # its own bins, log-uniform 64-512 per mode; FP64), and the method error
    # of both schemes against the full-grid likelihood on a walker subset
    nbm = [I.per_mode_bins(I.rng_for(4, 200 + k), sh[0]) for k, sh in enumerate(shapes)]
    pm_refs = [M.build_reference_coeffs_pm(ctx, it4["data"], M.MODEL_IMR, it4["modes"], it4["th"], nb)
               for it4, nb in zip(S4.items, nbm)]
    lnp = [torch.empty(len(t), dtype=torch.float64, device="cuda") for t in th4]
    bp = M.Batch(ctx, pm_refs, th4, lnp, prec=M.FP64)
    wall, mean_s = time_batch(M, ctx, bp, 200, 20, st)
    hm["per_mode_fp64_evals_per_s"] = W4 * 200 / wall
    hm["per_mode_fp64_us_per_launch"] = mean_s * 1e6
    hm["per_mode_bins"] = nbm
    bp.close()
    lnp = [l.cpu().numpy() for l in lnp]
    if not method_error:
        for r in pm_refs:
            r.close()
        return hm
    err_sum, err_pm = [], []
    for k, (it4, t4) in enumerate(zip(S4.items, th4)):
        idx = np.arange(0, len(t4), max(1, len(t4) // 32))[:32]
        sub = t4[torch.as_tensor(idx, device="cuda")].contiguous()
        lf = M.loglike_full(ctx, it4["data"], M.MODEL_IMR, it4["modes"], sub, M.FP64).cpu().numpy()
        off = sum(len(x) for x in th4[:k])
        err_sum.append(np.abs(lnl4["fp64"][off + idx] - lf))
        err_pm.append(np.abs(lnp[k][idx] - lf))
    es, ep = np.concatenate(err_sum), np.concatenate(err_pm)
    hm["method_error_vs_full_grid"] = {
        "walkers": int(es.size),
        "mode_summed": {"max": float(es.max()), "median": float(np.median(es))},
        "per_mode": {"max": float(ep.max()), "median": float(np.median(ep))}}
    for r in pm_refs:
        r.close()
    log(f"[bench] HM batch per-mode FP64: {hm['per_mode_fp64_evals_per_s']:.3g} evals/s; method error "
        f"{hm['method_error_vs_full_grid']}")
    return hm


def side_measurements(M, ctx, S, walkers, grid):
    import torch

    out = {}
    # full-grid likelihood: brute-force prior draws on the 1.58e6-bin grid,
    # FP64 (MBH_MIXED runs the same path), with the tile the autotuner picks
    # on the first 2048 draws
    it = S.items[0]
    draws = I.prior_draws(I.rng_for(3, 0), 16384, grid.t_obs)
    td = torch.as_tensor(draws, device="cuda")
    out["full_grid_shape_default"] = list(M.full_shape(ctx, False))
    M.loglike_full(ctx, it["data"], M.MODEL_IMR, M.MODE_22, td[:64], M.FP64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M.loglike_full(ctx, it["data"], M.MODEL_IMR, M.MODE_22, td, M.FP64)
    torch.cuda.synchronize()
    out["full_grid_default_shape_evals_per_s"] = len(draws) / (time.perf_counter() - t0)
    out["full_grid_shape"] = list(M.autotune_full(ctx, it["data"], M.MODEL_IMR, M.MODE_22, td[:2048]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lf = M.loglike_full(ctx, it["data"], M.MODEL_IMR, M.MODE_22, td, M.FP64)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["full_grid_evals_per_s"] = len(draws) / dt
    # algorithmic work per (walker, grid point); the counter figure beside it
    out["full_grid_roofline_frac"] = len(draws) * grid.n_f * ALGO_FULL_FLOPS_PER_POINT / dt / 1e12 / PEAK_ALU_TFLOPS
    if COUNTERS["src_sha256"] == kernel_sources_hash() and COUNTERS["full_valu_flops_per_point"]:
        out["full_grid_roofline_frac_hw"] = (len(draws) * grid.n_f * COUNTERS["full_valu_flops_per_point"] / dt
                                             / 1e12 / PEAK_ALU_TFLOPS)
    lm = M.loglike_full(ctx, it["data"], M.MODEL_IMR, M.MODE_22, td, M.MIXED)
    out["full_grid_mixed_equals_fp64"] = bool(torch.equal(lm, lf))
    log(f"[bench] full grid: {out['full_grid_evals_per_s']:.1f} evals/s with tile {out['full_grid_shape']} "
        f"(default {out['full_grid_shape_default']}: {out['full_grid_default_shape_evals_per_s']:.1f})")
    # reference build (a9)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = M.build_reference_coeffs(ctx, it["data"], M.MODEL_IMR, M.MODE_22, it["th"], N_BINS)
    out["reference_build_ms"] = (time.perf_counter() - t0) * 1e3
    r.close()
    # reference update on the device (Sec. 3.2): the best walker of the
    # population becomes the reference, rebuilt in place with no host sync
    r = M.build_reference_coeffs(ctx, it["data"], M.MODEL_IMR, M.MODE_22, it["th"], N_BINS)
    tw = torch.as_tensor(walkers[0], device="cuda")
    lw = M.loglike_heterodyned(ctx, r, tw, M.FP64)
    r.refresh(it["data"], tw, lw)  # the first update allocates the staging buffers
    torch.cuda.synchronize()
    st_r = torch.cuda.Stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n_rep = 20
    t0 = time.perf_counter()
    e0.record(st_r)
    for _ in range(n_rep):
        r.refresh(it["data"], tw, lw, stream=st_r)
    e1.record(st_r)
    t_issue = time.perf_counter() - t0
    torch.cuda.synchronize()
    res = r.refresh_result()
    out["reference_refresh"] = {"device_us": e0.elapsed_time(e1) * 1e3 / n_rep, "host_issue_us": t_issue * 1e6 / n_rep,
                                "status": res["status"], "generation": res["generation"]}
    log(f"[bench] reference refresh on the device: {out['reference_refresh']}")
    # a sampler-like loop (one batch per step, results read on the host) with
    # the reference moved to the best walker every 10th step: per-step
    # latency with the update on the device vs a host rebuild (new reference
    # handle, hence a new batch)
    lat = {}
    for mode in ("device", "host"):
        ref = M.build_reference_coeffs(ctx, it["data"], M.MODEL_IMR, M.MODE_22, it["th"], N_BINS)
        if mode == "device":
            ref.prepare_refresh()  # once, when the sampler starts
        lb = torch.empty(len(walkers[0]), dtype=torch.float64, device="cuda")
        b = M.Batch(ctx, [ref], [tw], [lb], prec=M.MIXED)
        b.launch_direct(st_r)
        torch.cuda.synchronize()
        ts = []
        for step in range(200):
            t0 = time.perf_counter()
            if step % 10 == 9:
                if mode == "device":
                    ref.refresh(it["data"], tw, lb, stream=st_r)
                else:
                    best = int(torch.argmax(lb).item())
                    new = M.build_reference_coeffs(ctx, it["data"], M.MODEL_IMR, M.MODE_22,
                                                   walkers[0][best], N_BINS, stream=st_r)
                    b.close()
                    ref.close()
                    ref = new
                    b = M.Batch(ctx, [ref], [tw], [lb], prec=M.MIXED)
            b.launch_direct(st_r)
            st_r.synchronize()
            ts.append(time.perf_counter() - t0)
        ts = np.array(ts) * 1e3
        upd = ts[9::10]
        lat[mode] = {"p50_ms": float(np.percentile(ts, 50)), "p99_ms": float(np.percentile(ts, 99)),
                     "update_step_mean_ms": float(upd.mean()), "plain_step_mean_ms": float(np.delete(ts, np.s_[9::10]).mean())}
        b.close()
        ref.close()
    out["reference_update_step_latency"] = lat
    log(f"[bench] steps with a reference update every 10th step: {lat}")
    r.close()
    out["hm_batch"] = hm_batch_leg(M, ctx, grid)
    # a heterodyned search (Sec. 3's second module) on the loudest source of
    # the step: 10 rungs x 400 walkers from a wide cloud around the source,
    # the reference starting at a hot walker and moved to the best walker on
    # the device every 1000 iterations (the paper: 5000, in runs of 1e4+
    # iterations), stopped when the maximum lnL has moved by less than 1 over
    # 30 checks 150 iterations apart
    out["sampler_search"] = sampler_search(M, ctx, S.items[1])
    out["ingest"] = ingest_leg(M, ctx)
    # serving: 4 resident sources (the step's physics with 1-6 modes each and
    # 64 / 128 / 256 / 512 bins), a Poisson stream from 64 samplers with
    # request sizes log-uniform in 1-4096 walkers, at fractions of the
    # measured capacity, in both precisions
    masks = [sh[0] for sh in I.batch_shapes(I.rng_for(5, 0), 4)]
    nbs = [64, 128, 256, 512]
    S5 = Sources(M, ctx, grid, 4, modes_list=masks, n_bins_list=nbs, cfg=5)
    refs = [x["ref"] for x in S5.items]
    pools = [S5.walkers(x, (1, 4, 16, 64), 64) for x in S5.items]
    serve = {"sources": [{"modes": int(m), "bins": nb} for m, nb in zip(masks, nbs)]}
    # capacity of each precision: the request rate the server sustains when
    # every request arrives at once (native replay: no interpreter in the loop)
    caps = {}
    for name, prec in (("mixed", M.MIXED), ("fp64", M.FP64)):
        cap = serve_run(M, ctx, refs, pools, prec, rate_hz=1e9, n_req=20000, warm=1000)
        caps[name] = cap["requests_per_s"]
        serve[f"{name}_capacity_req_per_s"] = cap["requests_per_s"]
        serve[f"{name}_capacity_evals_per_s"] = cap["throughput_evals_s"]
        log(f"[bench] serving capacity {name}: {cap['requests_per_s']:.0f} req/s, {cap['throughput_evals_s']:.3g} evals/s")
    serve["capacity_req_per_s"] = serve["mixed_capacity_req_per_s"]
    serve["capacity_evals_per_s"] = serve["mixed_capacity_evals_per_s"]
    for rho in (0.5, 0.8, 0.95):
        for name, prec in (("mixed", M.MIXED), ("fp64", M.FP64)):
            r = serve_run(M, ctx, refs, pools, prec, rate_hz=rho * caps[name], n_req=20000, warm=1000)
            serve[f"{name}_rho{rho}"] = r
            log(f"[bench] serve {name} at {rho} x capacity: {r}")
    # the same stream (0.5 x capacity, mixed) with a reference update (best
    # walker of the source's pool, rebuilt on the device) queued after every
    # 100th request
    datas = [x["data"] for x in S5.items]
    for rf in refs:
        rf.prepare_refresh()
    lnls = [M.loglike_heterodyned(ctx, rf, torch.as_tensor(pl, device="cuda"), M.FP64).cpu().numpy()
            for rf, pl in zip(refs, pools)]
    r = serve_run(M, ctx, refs, pools, M.MIXED, rate_hz=0.5 * caps["mixed"], n_req=20000, warm=1000,
                  update=(datas, lnls, 100))
    serve["mixed_rho0.5_with_reference_updates"] = r
    log(f"[bench] serve mixed at 0.5 x capacity with a reference update every 100 requests: {r}")
    for name, prec in (("mixed", M.MIXED), ("fp64", M.FP64)):
        serve[f"samplers_as_clients_{name}"] = served_samplers(M, ctx, S5, refs, prec)
    out["serving"] = serve
    return out


if __name__ == "__main__":
    main()
