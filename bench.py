#!/usr/bin/env python3
"""Throughput of the back-projection hot path on one MI355X.

A step is one pass of the online path over one frame of synthetic sensor data
(512 sensors x 2048 samples at 25 MHz) for the paper-scale geometry
(256x256 grid, h = 0.2 mm, random skull, 21336 region-of-interest pixels):
the fused UBP filter + delay-and-sum gather, launched through the C ABI with
the per-sensor delay table already resident in HBM.  The table itself is built
once beforehand by pat_eikonal_tables (the paper's offline step) and its build
time is reported separately.

Also timed (extra keys of the same JSON line): the 16.16-table and FP16
variants, 64-frame batched launches replayed from a HIP graph, and a short
serving mix (Poisson frames over three resident maps plus table builds).

--config selects another workload: "large" (1024x1024 grid, 1024 sensors),
the serving geometries, or the 3-D "head3" (64^3 voxel grid, 256 sensors on a
sphere; tables from pat_eikonal_tables_3d, the same gather with voxels as
pixels).

Prints one JSON line.  Usage:
    python bench.py [--steps K] [--warmup W] [--gpus 1] [--config NAME] [--no-cpu] [--no-variants]
                    [--serve SECONDS]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BP pixel·sensor gathers/s, frames/s, p50/p99 frame latency @512 sensors"
VOLUME_CONFIGS = ("tiny3", "head3")  # 3-D geometries: voxels are gathered like pixels
HBM_PEAK_GBS = 8000.0

# Memory traffic of the single-frame gather kernel per launch, from two
# rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch, mean over the dispatches of `--only headline` or, for the table
# streamed from HBM, `--only rotated`), each scaled by the same counter's
# reading for a plain 256 MB device copy (--copy-calibration 256: FETCH_SIZE
# reads 125012 KiB of 250000 KiB moved, factor 2.0; WRITE_SIZE reads 250000,
# factor 1.0).  FETCH_SIZE counts L2 read requests to the fabric, so reads
# served by the Infinity Cache count as well.  Valid only for the kernel
# sources they were taken on: the SHA-256 of the files below; any change makes
# the field null until the counters are taken again.  The 1024^2 workload's
# figures are those of the wave-window kernel (the plain table), the others
# of the split-sensor kernel (the interleaved table).  Summaries:
# profiles/k_bp_*_hbm_counters.md.
TRAFFIC_SOURCES = ("paper_1501_03869_amd/csrc/gather_px.hip", "paper_1501_03869_amd/csrc/gather_win.hip",
                   "paper_1501_03869_amd/csrc/gather_common.h")
TRAFFIC_SHA = "8c446ee2bd9ad5d338dc358c7e9cf6af010f9d7089517fe2ee51b7a2be52e815:" \
              "c13158e00f16cba69f8a19eda1d010ce6c8b0114344cf69ee605494d0366cedc:" \
              "04563295b4cefa9191f8ce39ecab8507bf4861fdb66ec84263b3126532f5fa18"
FETCH_FACTOR = 250000.0 / 125012.32
WRITE_FACTOR = 1.0
TRAFFIC_KIB = {"paper": (24265.93, 83.34), "large": (1725405.76, 3242.61),
               "paper_rotated": (24236.94, 83.36), "head3": (23670.92, 174.69),
               "head3_rotated": (23666.41, 174.69)}  # (FETCH_SIZE, WRITE_SIZE) per dispatch


def measured_traffic(config: str):
    """Bytes per launch from the stored counters, or None if the kernel changed."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    sha = ":".join(hashlib.sha256(open(os.path.join(here, f), "rb").read()).hexdigest() for f in TRAFFIC_SOURCES)
    if sha != TRAFFIC_SHA or config not in TRAFFIC_KIB:
        return None
    fetch, write = TRAFFIC_KIB[config]
    return (fetch * FETCH_FACTOR + write * WRITE_FACTOR) * 1024.0


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else float("nan")


def cpu_baseline(geo, vol, budget_s=12.0):
    """The FP64 oracle (filter + gather) on the host cores, timed on a bounded
    sample of the same workload: whole frames, repeated for about budget_s.
    Its inputs are its own: the oracle's delay table of the geometry (built
    before the timed region) and frames synthesised from it."""
    from paper_1501_03869_amd import inputs
    from oracle import oracle as orc
    tb = time.perf_counter()
    if vol:
        T = orc.tables3(geo.speed, geo.h, geo.sensors, geo.pix)
        build_s = time.perf_counter() - tb
        frames = [inputs.frame_for3(geo, T, f) for f in range(2)]
    else:
        T = orc.tables(geo.speed, geo.h, geo.sensors, geo.pix)
        build_s = time.perf_counter() - tb
        phantom = "points" if geo.nx * geo.ny > 512 * 512 else "segments"
        frames = [inputs.frame_for(geo, T, f, phantom=phantom) for f in range(2)]
    n = 0
    t0 = time.perf_counter()
    while True:
        orc.backproject(T, frames[n % len(frames)], geo.dt, geo.t0)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    gathers = n * geo.S * geo.P
    return {"value": gathers / el, "unit": "gathers/s", "cores": orc.max_threads(), "kind": "oracle",
            "sample": f"{n} whole frames ({geo.S} sensors x {geo.P} {'voxels' if vol else 'pixels'}) of the same "
                      f"workload (the oracle's own table and frames), FP64 filter + gather, {el:.1f} s",
            "table_build_s": build_s,
            "table_build_note": "the oracle's first-order fast marching (FP64, heap) for all sensors, parallel over "
                                "sensors on the same threads; not part of value"}


def rotated_tables(ctx, geo, table, frames, img, stream, steps):
    """The headline gather with its table forced out of the 256 MB Infinity
    Cache: K distinct resident copies of the interleaved table (K x table >
    512 MiB), one per launch in turn, so that every launch streams its table
    from HBM.  Mean launch duration from HIP events around back-to-back
    launches.  None when one table alone exceeds 128 MiB (it streams anyway)."""
    import torch
    S, P, N = geo.S, geo.P, geo.n_samples
    tbytes = S * P * 4
    if tbytes >= (128 << 20):
        return None
    K = max(8, -(-(512 << 20) // tbytes))
    copies = [ctx.table_to_x4(table) for _ in range(K)]
    R = frames.shape[0]
    torch.cuda.synchronize()

    def rot(i):
        r = i % R
        ctx.backproject(copies[i % K], frames[r], geo.dt, geo.t0, filtered=False, out=img[r], stream=stream)
    for i in range(2 * K):
        rot(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    steps = max(steps, 4 * K)
    e0.record(stream)
    for i in range(steps):
        rot(i)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / steps
    b = 4 * S * P + 4 * S * N + 4 * P
    del copies
    return {"bound": "hbm", "achieved": b / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": b / t / 1e9 / HBM_PEAK_GBS, "traffic": measured_traffic(geo.name + "_rotated"),
            "tables_rotated": K, "resident_table_bytes": K * tbytes, "device_ms_per_frame_mean": t * 1e3,
            "gathers_per_s": S * P / t, "algorithmic_bytes_per_launch": b,
            "timing_note": "HIP events around back-to-back launches, each on the next of K copies of the "
                           "interleaved table (K x table > 512 MiB), so every launch streams its table from HBM",
            "traffic_note": "FETCH_SIZE + WRITE_SIZE of the same rotated launches (bench.py --only rotated), "
                            "scaled by a plain copy's counters; FETCH_SIZE counts L2 read requests to the "
                            "fabric, Infinity Cache hits included"}


def large_hbm(ctx, stream, steps=50, warmup=10):
    """The 1024^2 workload's table (1024 sensors x 823 592 pixels, 3.37 GB,
    built here by pat_eikonal_tables) gathered by pat_backproject in the form
    it is fastest with (the plain [S][P] table: the wave-window kernel), one
    launch per frame: a table that always streams from HBM.  One white-noise
    frame (the content does not change the work).  Mean launch duration from
    HIP events around back-to-back launches."""
    import torch
    from paper_1501_03869_amd import inputs, pat
    geo = inputs.config("large")
    geo.pix = pat.tile_order(geo.nx, geo.ny, geo.pix, 32, 32)
    dev = torch.device("cuda")
    S, P, N = geo.S, geo.P, geo.n_samples
    t = time.perf_counter()
    table = ctx.eikonal_tables(torch.from_numpy(geo.speed).to(dev), geo.h, geo.sensors,
                               torch.from_numpy(geo.pix).to(dev))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t
    frame = torch.from_numpy(inputs.random_signals(11, S, N)).to(dev)
    img = torch.empty(P, dtype=torch.float32, device=dev)

    def one():
        ctx.backproject(table, frame, geo.dt, geo.t0, filtered=False, out=img, stream=stream)
    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        one()
    e1.record(stream)
    torch.cuda.synchronize()
    tl = e0.elapsed_time(e1) * 1e-3 / steps
    b = 4 * S * P + 4 * S * N + 4 * P
    del table, frame, img
    torch.cuda.empty_cache()
    return {"bound": "hbm", "achieved": b / tl / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": b / tl / 1e9 / HBM_PEAK_GBS, "traffic": measured_traffic("large"),
            "workload": "large: 1024x1024 grid h=0.05 mm, 1024 sensors, 823592 ROI pixels, 4096 samples at 40 MHz, "
                        "FP32 table [S][P] (3.37 GB) + FP32 signals, fused filter+gather, one frame per launch",
            "kernel": "pat_backproject (k_bp_win at this shape)", "device_ms_per_frame_mean": tl * 1e3,
            "gathers_per_s": S * P / tl, "algorithmic_bytes_per_launch": b, "table_build_s": build_s,
            "timing_note": "HIP events around back-to-back launches on one resident table that does not fit the "
                           "256 MB Infinity Cache (one white-noise frame)",
            "traffic_note": "FETCH_SIZE + WRITE_SIZE of bench.py --config large --only headline, scaled by a plain "
                            "copy's counters; null when not measured for this kernel source"}


def _frame_worker(args):
    from paper_1501_03869_amd import inputs
    parts, N, dt, t0, f, snr = args
    return inputs.frame_from_parts(parts, N, dt, t0, f, snr)


def batch_frames(geo, table_h, F=64, snr_db=20.0):
    """F distinct frames: each its own seeded phantom plus white Gaussian
    noise at snr_db (the batched-frames configuration).  The pulse sums run in
    worker processes started fresh (spawn: they never touch the GPU); the
    phantoms' table columns are gathered here."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    from paper_1501_03869_amd import inputs
    phantom = "points" if geo.nx * geo.ny > 512 * 512 else "segments"
    jobs = [(inputs.frame_parts(geo, table_h, f, phantom), geo.n_samples, geo.dt, geo.t0, f, snr_db) for f in range(F)]
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 4), mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_frame_worker, jobs))


def run_batch64(ctx, geo, table, frames, frames_h, stream, timed, args,
                names=("batch64_v0_f32", "batch64_v3_q16_f16", "batch64_v4_r16_f16"), table_h=None):
    """64 frames per launch, table read once per launch (per 16 frames for
    tables past the cache), replayed from a HIP graph.  With table_h (2-D
    geometries) the 64 frames are distinct phantoms with 20 dB noise;
    otherwise the resident frames are cycled."""
    import torch
    S, P, N = geo.S, geo.P, geo.n_samples
    dev = table.device
    if table_h is not None:
        t = time.perf_counter()
        frames_h = batch_frames(geo, table_h)
        frames = torch.from_numpy(np.stack(frames_h)).to(dev)
        print(f"[bench] {len(frames_h)} noisy frames synthesised in {time.perf_counter() - t:.1f} s",
              file=sys.stderr, flush=True)
    R = len(frames_h)
    p = np.stack(frames_h).astype(np.float32)
    scale = (np.abs(p).reshape(R, -1).max(1) / 2.0 ** 14).astype(np.float32)
    half = torch.from_numpy((p / scale[:, None, None]).astype(np.float16)).to(dev)
    scale_d = torch.from_numpy(scale).to(dev)
    tabs = {"batch64_v0_f32": table}
    if "batch64_v3_q16_f16" in names:
        tabs["batch64_v3_q16_f16"] = ctx.table_to_q16(table, geo.dt, N, geo.t0)
    if "batch64_v4_r16_f16" in names:
        tabs["batch64_v4_r16_f16"] = ctx.table_to_r16(table, geo.dt, N, geo.t0)
    F = 64
    idx = np.arange(F) % R
    sigs = {"f32": frames[torch.from_numpy(idx).to(dev)].contiguous(),
            "f16": half[torch.from_numpy(idx).to(dev)].contiguous()}
    scl = scale_d[torch.from_numpy(idx).to(dev)].contiguous()
    outF = torch.empty((F, P), dtype=torch.float32, device=dev)
    res = {}
    for name in names:
        tab = tabs[name]
        sk = "f32" if name.endswith("f32") else "f16"
        sig = sigs[sk]
        sc = scl if sk == "f16" else None
        ctx.reserve(S, P, F)
        g = torch.cuda.CUDAGraph()
        s2 = torch.cuda.Stream()
        s2.wait_stream(stream)
        with torch.cuda.stream(s2):
            ctx.backproject(tab, sig, geo.dt, geo.t0, filtered=False, frame_scale=sc, out=outF, stream=s2)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            ctx.backproject(tab, sig, geo.dt, geo.t0, filtered=False, frame_scale=sc, out=outF)
        steps = max(20, args.steps // 8)
        wall, ms = timed(lambda i: g.replay(), steps, 5)
        res[name] = {"frames_per_launch": F, "gathers_per_s": steps * F * S * P / wall,
                     "frames_per_s": steps * F / wall, "device_ms_p50": percentile(ms, 50),
                     "device_ms_p99": percentile(ms, 99), "hip_graph": True,
                     "frames": ("64 distinct phantoms, 20 dB white noise" if table_h is not None
                                else f"{R} resident frames cycled")}
    return res


def run_variants(ctx, geo, table, frames, frames_h, stream, timed, args, table_h=None):
    """Reduced-precision and batched variants on the same geometry and frames."""
    import torch
    S, P, N = geo.S, geo.P, geo.n_samples
    dev = table.device
    q16 = ctx.table_to_q16(table, geo.dt, N, geo.t0)
    R = len(frames_h)
    p = np.stack(frames_h).astype(np.float32)
    scale = (np.abs(p).reshape(R, -1).max(1) / 2.0 ** 14).astype(np.float32)
    half = torch.from_numpy((p / scale[:, None, None]).astype(np.float16)).to(dev)
    scale_d = torch.from_numpy(scale).to(dev)
    img = torch.empty((R, P), dtype=torch.float32, device=dev)
    res = {}

    def single(name, tab, sig, sc):
        def fn(i):
            r = i % R
            ctx.backproject(tab, sig[r], geo.dt, geo.t0, filtered=False, frame_scale=None if sc is None else sc[r:r + 1],
                            out=img[r], stream=stream)
        wall, ms = timed(fn, args.steps, args.warmup)
        res[name] = {"frames_per_launch": 1, "gathers_per_s": args.steps * S * P / wall,
                     "frames_per_s": args.steps / wall,
                     "timing_note": "eager single-frame launches (wall time); device_ms_*: HIP events around each",
                     "device_ms_p50": percentile(ms, 50), "device_ms_p99": percentile(ms, 99)}

    r16 = ctx.table_to_r16(table, geo.dt, N, geo.t0)
    single("v0_f32_table_f32_signal", table, frames, None)
    single("v0x4_interleaved_f32_table_f32_signal", ctx.table_to_x4(table), frames, None)
    single("v1_q16_table_f32_signal", q16, frames, None)
    single("v2_f32_table_f16_signal", table, half, scale_d)
    single("v3_q16_table_f16_signal", q16, half, scale_d)
    single("v4_r16_table_f16_signal", r16, half, scale_d)
    single("v4a_r16_table_f32_signal", r16, frames, None)

    # the conventional back projection (straight rays at 1540 m/s computed per
    # gather, no table) on the same frames
    pix_d = torch.from_numpy(np.ascontiguousarray(geo.pix)).to(dev)

    def conv(i):
        r = i % R
        if hasattr(geo, "nz"):
            ctx.backproject_const_3d(geo.nx, geo.ny, geo.nz, geo.h, 1540.0, geo.sensors, pix_d, frames[r], geo.dt,
                                     geo.t0, filtered=False, out=img[r], stream=stream)
        else:
            ctx.backproject_const(geo.nx, geo.ny, geo.h, 1540.0, geo.sensors, pix_d, frames[r], geo.dt, geo.t0,
                                  filtered=False, out=img[r], stream=stream)
    wall, ms = timed(conv, args.steps, args.warmup)
    res["conventional_bp_straight_rays"] = {
        "frames_per_launch": 1, "gathers_per_s": args.steps * S * P / wall, "frames_per_s": args.steps / wall,
        "timing_note": "eager single-frame launches (wall time, including the per-call sensor upload); "
                       "device_ms_*: HIP events around each", "device_ms_p50": percentile(ms, 50),
        "device_ms_p99": percentile(ms, 99)}

    # (the same single-frame gather with the table forced out of the 256 MB
    # Infinity Cache is reported as roofline_hbm)

    # the UBP filter alone (pat_filter): one pass over the frame, 4 B read and
    # 4 B written per sample
    fout = torch.empty_like(frames[0])
    pat_f = lambda i: ctx.filter(frames[i % R], geo.dt, geo.t0, out=fout, stream=stream)
    timed(pat_f, 20, 0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(args.steps):
        pat_f(i)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / args.steps
    res["filter_only"] = {"device_ms_mean": t * 1e3, "algorithmic_bytes": 8 * S * N,
                          "achieved_GBps": 8 * S * N / t / 1e9, "frac_hbm_peak": 8 * S * N / t / 1e9 / HBM_PEAK_GBS,
                          "timing_note": "HIP events around back-to-back pat_filter launches on one frame each"}

    # batched: F frames per launch, table read once; replayed from a HIP graph
    res.update(run_batch64(ctx, geo, table, frames, frames_h, stream, timed, args, table_h=table_h))
    return res


def run_serving(ctx, seconds, variant, rate_hz=200.0, new_map_every_s=2.0):
    """Serving mix: Poisson frame stream over three resident speed maps (128^2
    with 128 sensors, 256^2 with 512, 512^2 with 512) plus a new paper-scale
    speed map every few seconds that triggers a table build; then a saturation
    burst with all slots busy.  Returns the server's statistics."""
    import threading
    import torch
    from paper_1501_03869_amd import inputs, pat
    dev = torch.device("cuda:0")
    geos = [inputs.config("serve_a"), inputs.config("paper"), inputs.config("serve_c")]
    for g in geos:
        g.pix = pat.tile_order(g.nx, g.ny, g.pix, 32, 32)
    frames = []
    for g in geos:
        T = ctx.eikonal_tables(torch.from_numpy(g.speed).to(dev), g.h, g.sensors,
                               torch.from_numpy(g.pix).to(dev)).cpu().numpy()
        fr = [inputs.frame_for(g, T, 100 + k, noise_snr_db=20.0) for k in range(2)]
        frames.append(fr)
    q16 = variant == "v3"
    srv = pat.Server(ctx, table_fmt=pat.TABLE_Q16 if q16 else pat.TABLE_F32,
                     sig_fmt=pat.SIG_F16 if q16 else pat.SIG_F32, max_batch=64, max_inflight=3, max_slots=512)

    def enc(p):
        if not q16:
            return p, 1.0
        sc = float(np.abs(p).max() / 2.0 ** 14)
        return (p / sc).astype(np.float16), sc

    encoded = [[enc(p) for p in fr] for fr in frames]
    ids = [srv.add_map(g.speed, g.h, g.sensors, g.pix, g.n_samples, g.dt, g.t0) for g in geos]
    t_wait = time.perf_counter()
    while any(srv.map_state(i) != pat.MAP_READY for i in ids):
        if time.perf_counter() - t_wait > 120:
            raise RuntimeError("maps not ready")
        time.sleep(0.01)
    build_s = time.perf_counter() - t_wait
    kinds = {i: k for k, i in enumerate(ids)}  # map id -> frame set
    P_of = {i: geos[k].P for k, i in enumerate(ids)}
    rng = np.random.default_rng(inputs.SEED_ARRIVALS)
    arrivals = inputs.poisson_arrivals(rate_hz, seconds)
    q = []
    lock = threading.Lock()
    done = threading.Event()
    errors = []

    def collector():
        while True:
            with lock:
                item = q.pop(0) if q else None
            if item is None:
                if done.is_set():
                    return
                time.sleep(0.0002)
                continue
            try:
                srv.wait(item[0], P=item[1], timeout_ms=60000)
            except Exception as e:  # noqa: BLE001
                errors.append(repr(e))

    th = threading.Thread(target=collector)
    th.start()
    srv.reset_stats()
    t0 = time.perf_counter()
    next_map_t = new_map_every_s
    seed = 5000
    new_ids = []
    for a in arrivals:
        while True:
            now = time.perf_counter() - t0
            if now >= next_map_t:
                g = geos[1]
                sp = inputs.paper_like_speed(seed, g.nx, g.ny, g.h)
                seed += 1
                try:
                    mid = srv.add_map(sp, g.h, g.sensors, g.pix, g.n_samples, g.dt, g.t0)
                    kinds[mid] = 1
                    P_of[mid] = g.P
                    new_ids.append(mid)
                except pat.PatError:
                    pass
                next_map_t += new_map_every_s
            if now >= a:
                break
            time.sleep(min(a - now, 0.0005))
        ready = [i for i in kinds if srv.map_state(i) == pat.MAP_READY]
        mid = ready[int(rng.integers(0, len(ready)))]
        p, sc = encoded[kinds[mid]][int(rng.integers(0, 2))]
        t = srv.submit(mid, p, sc)
        with lock:
            q.append((t, P_of[mid]))
    while True:
        with lock:
            if not q:
                break
        time.sleep(0.001)
    paced = srv.stats()
    paced_wall = time.perf_counter() - t0
    # saturation: keep the server full for a short burst
    srv.reset_stats()
    t1 = time.perf_counter()
    n_sat = 0
    while time.perf_counter() - t1 < min(3.0, seconds):
        for k in range(3):
            mid = ids[k]
            p, sc = encoded[k][n_sat % 2]
            t = srv.submit(mid, p, sc)
            with lock:
                q.append((t, P_of[mid]))
            n_sat += 1
    while True:
        with lock:
            if not q:
                break
        time.sleep(0.001)
    sat = srv.stats()
    done.set()
    th.join()
    srv.close()
    keys = ("frames_done", "frames_per_s", "gathers_per_s", "latency_p50_us", "latency_p99_us", "latency_max_us",
            "mean_batch_frames", "batches", "builds", "evictions", "frames_refused")
    return {"variant": variant, "rate_hz": rate_hz, "seconds": seconds, "initial_build_s": build_s,
            "paced": {k: paced[k] for k in keys}, "paced_wall_s": paced_wall, "new_maps": len(new_ids),
            "saturated": {k: sat[k] for k in keys}, "errors": errors[:3]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--config", default="paper")
    ap.add_argument("--frames", type=int, default=8, help="distinct resident frames cycled through")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-variants", action="store_true", help="skip the reduced-precision and batched variants")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 1024^2 workload's HBM-streamed gather block (paper config only)")
    ap.add_argument("--serve", type=float, default=5.0, help="seconds of the serving mix per variant (0 = skip)")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="MB",
                    help="only run a plain device copy of MB megabytes 10 times (HBM counter calibration)")
    ap.add_argument("--table", choices=("auto", "x4", "plain"), default="auto",
                    help="headline table form: auto = four sensors interleaved (pat_table_to_x4) while the table "
                         "stays in the Infinity Cache, the plain [S][P] table when it streams from HBM")
    ap.add_argument("--only", choices=("tables", "headline", "rotated", "batch64"), default=None,
                    help="profiling runs: only the two table builds, or the table builds followed by only the "
                         "headline single-frame launches, only the gather on rotated table copies (the table "
                         "streamed from HBM), or only 64-frame launches; prints no JSON line")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              f"(frame-parallel sharding across GPUs needs no exchange and is described in the design notes).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1501_03869_amd import inputs, pat

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration > 0:
        # a plain copy of known size: the scale of the HBM byte counters
        n = int(args.copy_calibration * 1e6) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 10}), flush=True)
        return
    dev = torch.device("cuda:0")
    ctx = pat.Context(0)
    vol = args.config in VOLUME_CONFIGS
    geo = inputs.config3(args.config) if vol else inputs.config(args.config)
    grid = f"{geo.nx}x{geo.ny}x{geo.nz}" if vol else f"{geo.nx}x{geo.ny}"
    print(f"[bench] {geo.name}: grid {grid} S={geo.S} P={geo.P} N={geo.n_samples}", file=sys.stderr, flush=True)

    if vol:
        # ROI in 4x4x2-voxel tiles: 32 neighbouring voxels per gather tile
        geo.pix = pat.tile_order_3d(geo.nx, geo.ny, geo.nz, geo.pix, 4, 4, 2)
    else:
        # ROI in 32x32-tile, Z-order-inside order: compact pixel blocks for the gather
        geo.pix = pat.tile_order(geo.nx, geo.ny, geo.pix, 32, 32)
    speed = torch.from_numpy(geo.speed).to(dev)
    pix = torch.from_numpy(geo.pix).to(dev)
    build = ctx.eikonal_tables_3d if vol else ctx.eikonal_tables
    build(speed, geo.h, geo.sensors, pix)  # first call: allocations and code loading
    torch.cuda.synchronize()
    t = time.perf_counter()
    table = build(speed, geo.h, geo.sensors, pix)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t
    est = ctx.eikonal_stats()
    n_nodes = geo.nx * geo.ny * (geo.nz if vol else 1)
    print(f"[bench] tables built in {build_s:.3f} s ({est['rounds']} rounds)", file=sys.stderr, flush=True)
    if args.only == "tables":
        return
    build_o2_s = None
    if not vol and geo.nx * geo.ny <= 512 * 512:
        # the paper's second-order scheme (heap-ordered marching, one map per wave)
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx.eikonal_tables_o2(speed, geo.h, geo.sensors, pix)
        torch.cuda.synchronize()
        build_o2_s = time.perf_counter() - t
        print(f"[bench] second-order tables built in {build_o2_s:.3f} s", file=sys.stderr, flush=True)

    table_h = table.cpu().numpy()
    # The resident table in the form pat_backproject gathers fastest from (the
    # same float32 delays, laid out once offline): while it stays in the
    # Infinity Cache, four sensors per 16-byte entry (pat_table_to_x4), which
    # the split-sensor kernel reads; when it streams from HBM and has at least
    # 131072 columns, the plain [S][P] table, which goes to the wave-window
    # kernel.
    streamed = 4 * geo.S * geo.P > (128 << 20) and geo.P >= 131072
    form = args.table if args.table != "auto" else ("plain" if streamed else "x4")
    table_head = ctx.table_to_x4(table) if form == "x4" else table
    win = form == "plain" and streamed
    torch.cuda.synchronize()
    if vol:
        frames_h = [inputs.frame_for3(geo, table_h, f) for f in range(args.frames)]
    else:
        # the large grid's vascular phantom has tens of thousands of nodes: point
        # absorbers keep its frame synthesis short (the content does not change the work)
        phantom = "points" if geo.nx * geo.ny > 512 * 512 else "segments"
        frames_h = [inputs.frame_for(geo, table_h, f, phantom=phantom) for f in range(args.frames)]
    frames = torch.from_numpy(np.stack(frames_h)).to(dev)
    img = torch.empty((args.frames, geo.P), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def timed(fn, steps, warmup):
        """Run fn(i) warmup + steps times on the current stream; per-call device
        times from HIP events on that stream, wall time of the timed steps."""
        for i in range(warmup):
            fn(i)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for i in range(steps):
            ev[i][0].record(stream)
            fn(i)
            ev[i][1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, [a.elapsed_time(b) for a, b in ev]

    def step(i, st=None):
        r = i % args.frames
        ctx.backproject(table_head, frames[r], geo.dt, geo.t0, filtered=False, out=img[r], stream=st or stream)

    S, P, N = geo.S, geo.P, geo.n_samples
    bytes_per_frame = 4 * S * P + 4 * S * N + 4 * P
    if args.only == "headline":
        for i in range(args.warmup + args.steps):
            step(i)
        torch.cuda.synchronize()
        print("[bench] headline launches done", file=sys.stderr, flush=True)
        return
    if args.only == "rotated":
        rotated_tables(ctx, geo, table, frames, img, stream, max(args.steps, 1))
        print("[bench] rotated-table launches done", file=sys.stderr, flush=True)
        return
    if args.only == "batch64":
        run_batch64(ctx, geo, table, frames, frames_h, stream, timed, args, names=("batch64_v0_f32", "batch64_v3_q16_f16"),
                    table_h=None if vol else table_h)
        print("[bench] 64-frame launches done", file=sys.stderr, flush=True)
        return

    # (a) per-launch device time: HIP events around every launch on its
    # stream (p50/p99), and two events around the whole run of back-to-back
    # launches (the mean launch duration the roofline uses)
    _, dev_ms = timed(step, args.steps, args.warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(args.steps):
        step(i)
    e1.record(stream)
    torch.cuda.synchronize()
    avg_kernel_s = e0.elapsed_time(e1) * 1e-3 / args.steps
    achieved = bytes_per_frame / avg_kernel_s / 1e9

    # (b) throughput: the same single-frame launches, captured back to back in
    # a HIP graph so that host-side call overhead does not starve the GPU;
    # exactly args.steps frames are timed
    glen = min(64, args.steps)
    ctx.reserve(S, P, 1)
    graph = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(stream)
    with torch.cuda.stream(cap):
        for i in range(glen):
            step(i, cap)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=cap):
        for i in range(glen):
            step(i, cap)
    for _ in range(max(1, args.warmup // glen)):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done + glen <= args.steps:
        graph.replay()
        done += glen
    for i in range(args.steps - done):
        step(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gathers = args.steps * S * P
    value = gathers / wall

    # end-to-end latency: host frame -> H2D -> back projection -> D2H image
    pinned_in = [torch.from_numpy(f).pin_memory() for f in frames_h[:4]]
    pinned_out = torch.empty((P,), dtype=torch.float32).pin_memory()
    dframe = torch.empty_like(frames[0])
    lat = []
    for i in range(max(50, min(args.steps, 200))):
        t1 = time.perf_counter()
        dframe.copy_(pinned_in[i % 4], non_blocking=True)
        ctx.backproject(table_head, dframe, geo.dt, geo.t0, filtered=False, out=img[0], stream=stream)
        pinned_out.copy_(img[0], non_blocking=True)
        stream.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "gathers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{geo.name}: {grid} grid h={geo.h * 1e3:g} mm, {S} sensors, {P} ROI "
                               f"{'voxels' if vol else 'pixels'}, {N} samples at {1e-6 / geo.dt:g} MHz, "
                               f"FP32 table{' (four sensors interleaved)' if form == 'x4' else ''} + FP32 "
                               f"signals, fused filter+gather, one frame per step",
                   "sensors": S, "pixels": P, "samples": N, "frames_per_step": 1,
                   "table_format": ("f32 seconds, four sensors interleaved per pixel (pat_table_to_x4)" if form == "x4"
                                    else "f32 seconds, [S][P]")},
        "frames_per_s": args.steps / wall,
        "timing_note": "value/frames_per_s: single-frame launches replayed from a HIP graph of up to 64 launches; "
                       "device_ms_*: HIP events around each eager launch; roofline: HIP events around the run of "
                       "back-to-back eager launches (mean launch duration)",
        "device_ms_per_frame_mean": avg_kernel_s * 1e3,
        "device_ms_per_frame_p50": percentile(dev_ms, 50),
        "device_ms_per_frame_p99": percentile(dev_ms, 99),
        "latency_ms_p50": percentile(lat, 50),
        "latency_ms_p99": percentile(lat, 99),
        "latency_note": "host frame -> H2D -> fused filter+gather -> D2H image, synchronous, pinned buffers",
        "table_build_s": build_s,
        "table_build_rounds": est["rounds"],
        "table_build_nodes_per_s": S * n_nodes / build_s,
        "table_build_tile_node_sweeps": est["sweeps"] * (512 if vol else 1024),
        "table_build_note": "pat_eikonal_tables" + ("_3d" if vol else "") + " wall time for all sensors (second "
                            "call), host validation and seeding included; nodes_per_s = sensors x grid nodes solved "
                            "per second; tile_node_sweeps = in-tile relaxation sweeps x nodes per tile (32 x 32, or "
                            "8^3 for 3-D bricks), a work counter",
        "table_build_o2_s": build_o2_s,
        "table_build_o2_note": "pat_eikonal_tables_o2 (the paper's second-order scheme) wall time for all sensors; "
                               "null for 3-D and grids above 512^2",
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.config if args.table == "auto" else ""),
                     "table_residency": ("infinity_cache" if 4 * S * P < (256 << 20) else "hbm"),
                     "residency_note": "a table below the 256 MB Infinity Cache is re-read from it between "
                                       "launches, so achieved is algorithmic bytes per second, not HBM "
                                       "bandwidth; roofline_hbm streams copies of it from HBM",
                     "kernel": ("pat_backproject, one launch per frame (k_bp_win at these shapes: fused UBP filter "
                                "+ delay-and-sum gather, one wave per 256 table columns, the filtered signal read "
                                "from a per-wave LDS window)" if win else
                                "pat_backproject, one launch per frame (k_bp_px at these shapes: fused UBP filter "
                                "+ delay-and-sum gather, sensors split inside 32-pixel-tile workgroups" +
                                (", table interleaved by four sensors)" if form == "x4" else ")")),
                     "algorithmic_bytes_per_launch": bytes_per_frame,
                     "traffic_note": "bytes per launch from FETCH_SIZE + WRITE_SIZE scaled by a plain copy's "
                                     "counters; null when not measured for this config or kernel source"},
        "paper_context": "123.79 ms for 512 sensors x 21323 pixels on an NVIDIA Tesla C2075, transfers included",
    }
    rh = rotated_tables(ctx, geo, table, frames, img, stream, args.steps)
    if rh is not None:
        out["roofline_hbm"] = rh
    if args.config == "paper" and not args.no_large:
        # the same gather on the 1024^2 workload, whose table streams from HBM
        out["roofline_large_hbm"] = large_hbm(ctx, stream)
    if not args.no_variants:
        out["variants"] = run_variants(ctx, geo, table, frames, frames_h, stream, timed, args,
                                       table_h=None if vol else table_h)
    if args.serve > 0 and not vol:
        out["serving"] = [run_serving(ctx, args.serve, v) for v in ("v0", "v3")]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(geo, vol)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
