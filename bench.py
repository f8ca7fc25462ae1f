"""Throughput benchmark of the haemoglobin-estimation hot path on one MI355X.

One step = one hb_estimate_frames call over a batch of synthetic 1920x1080
frames (log-attenuation + 2-level Haar + Tikhonov, posterior over a 256x256
THb x SO2 grid, inverse Haar and maps), frames already resident in HBM.

Prints one JSON line with frames/s (value), Mpixel/s, the roofline of the
dominant kernel (the posterior) from per-kernel HIP events recorded on the
launch stream, and the FP64 CPU oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/s + Mpixel/s at 1920x1080 on 1 GPU; p99 frame latency, 16 streams"
FP32_VECTOR_PEAK_TFLOPS = 157.3
# Algorithmic operations per (LL pixel, grid node) pair of the posterior:
# 3 sub + 3 mul + 2 add (squared distance), 1 mul (-1/(2 sigma^2)), 1 sub (max
# offset), 1 add + 2 mul + 2 add (three moments) = 15 flops, plus one exp.
FLOPS_PER_PAIR = 15
EXPS_PER_PAIR = 1
# HBM bytes per posterior launch of the default workload (16 frames), from the
# rocprofv3 FETCH_SIZE/WRITE_SIZE runs summarised in
# profiles/hot_path_1080p_L2_G256_b16.md, valid for the device sources whose
# combined sha256 (kernel_source_sha) starts with PROFILED_KERNEL_SHA; reported
# as null for any other source or workload.
PROFILED_KERNEL_SHA = "bd2ead1ae8648636"
PROFILED_POSTERIOR_TRAFFIC = 1236.93e6
KERNEL_SOURCES = ("hb_kernels.hip", "hb_internal.h", "hb_df.h")


def kernel_source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1706_07263_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--levels", type=int, default=2)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--split", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample (0 = skip)")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=8.0,
                    help="duration of the 16-stream serving run (0 = skip)")
    ap.add_argument("--serve-warmup", type=float, default=2.0)
    ap.add_argument("--serve-budget-gib", type=float, default=48.0)
    ap.add_argument("--no-table1", action="store_true", help="skip the Table 1 speed-ratio analogue")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--sequence", type=int, default=0,
                    help="only time the first N frames of the video, all resident in HBM, "
                         "at batch 1, 4 and 16 (one JSON line)")
    return ap.parse_args()


def log(msg, quiet=False):
    if not quiet:
        print(msg, file=sys.stderr, flush=True)


def _render_frame(job):
    from paper_1706_07263_amd import synth
    i, dtype = job
    return synth.config3((i,), dtype=dtype).frames


def render_video(idx, dtype: str, workers: int = 8) -> np.ndarray:
    """Frames idx of the 1920x1080 video, rendered in fresh worker processes."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    ctx = multiprocessing.get_context("spawn")
    with ProcessPoolExecutor(max_workers=max(1, min(workers, len(idx))), mp_context=ctx) as pool:
        return np.concatenate(list(pool.map(_render_frame, [(i, dtype) for i in idx])))


def cpu_baseline(target_s: float, levels: int, grid: int, quiet: bool):
    """Time the FP64 oracle on the benchmark's video frames: a whole-width row
    band of frame 0 sized for about target_s, or whole frames 0, 1, ... when
    one frame takes less than that."""
    from oracle import hb_oracle as orc
    from paper_1706_07263_amd import synth
    from tests import hbtest
    w = synth.config3((0,))
    s = dict(w.plan)
    s["levels"], s["grid_thb"], s["grid_so2"] = levels, grid, grid
    b = 1 << levels
    fr = w.frames.astype(np.float64)
    model = hbtest.oracle_model(synth.spectra())
    # calibration on a small band, then a band sized for the target time
    rows = 4 * b
    t0 = time.perf_counter()
    orc.estimate(hbtest.oracle_params(1920, rows, s), model, fr[:, :rows])
    dt = time.perf_counter() - t0
    rows = int(min(1080, max(b, rows * target_s / max(dt, 1e-3)))) // b * b
    rows = max(rows, b)
    t0 = time.perf_counter()
    orc.estimate(hbtest.oracle_params(1920, rows, s), model, fr[:, :rows])
    dt = time.perf_counter() - t0
    if rows == 1080 and dt < 0.5 * target_s:
        # a whole frame is quick: time frames 0 .. n-1 together instead
        n = int(min(8, max(2, round(target_s / dt))))
        fr = render_video(list(range(n)), "f32").astype(np.float64)
        t0 = time.perf_counter()
        orc.estimate(hbtest.oracle_params(1920, 1080, s), model, fr)
        dt = time.perf_counter() - t0
        log(f"cpu oracle: {n} frames of 1920x1080 in {dt:.2f} s on {orc.threads()} threads", quiet)
        return {"value": n / dt, "unit": "frames/s", "cores": orc.threads(), "kind": "oracle",
                "sample": f"frames 0..{n - 1} (1920x1080, {(1080 // b) * (1920 // b)} low-pass pixels x "
                          f"{grid * grid} nodes each), {dt:.2f} s"}
    frac = rows / 1080.0
    log(f"cpu oracle: {rows} rows x 1920 in {dt:.2f} s on {orc.threads()} threads", quiet)
    return {"value": frac / dt, "unit": "frames/s", "cores": orc.threads(), "kind": "oracle",
            "sample": f"rows 0..{rows - 1} of frame 0 (1920x{rows} px, "
                      f"{(rows // b) * (1920 // b)} low-pass pixels x {grid * grid} nodes), "
                      f"{dt:.2f} s, scaled by {rows}/1080"}


PAPER_TABLE1_HZ = {"bayes_full_resolution": 3.54, "proposed_w1": 12.7, "proposed_w3": 14.4, "tikhonov": 43.5}


def host_serial(torch, plan, host, dev, maps, stream, steps, warmup) -> float:
    """Calls per second: copy the batch from pinned memory, then estimate,
    one after the other on one stream."""
    def step():
        dev.copy_(host, non_blocking=True)
        plan.estimate(dev, maps, stream)
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(steps):
            step()
    torch.cuda.synchronize()
    return steps / (time.perf_counter() - t0)


def host_overlapped(torch, plan, host, dev, maps, stream, steps, warmup) -> float:
    """Calls per second with two device slots: a copy stream (default
    priority) fills one slot while the compute stream estimates the other."""
    slots = [dev, torch.empty_like(dev)]
    copy_s = torch.cuda.Stream(dev.device)
    copied = [torch.cuda.Event(), torch.cuda.Event()]
    done = [torch.cuda.Event(), torch.cuda.Event()]

    def run(n):
        for i in range(n):
            k = i & 1
            copy_s.wait_event(done[k])
            with torch.cuda.stream(copy_s):
                slots[k].copy_(host, non_blocking=True)
            copied[k].record(copy_s)
            stream.wait_event(copied[k])
            plan.estimate(slots[k], maps, stream)
            done[k].record(stream)
    run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    return steps / (time.perf_counter() - t0)


def time_plan(hb, torch, desc, spectra, frames, maps, stream, steps, warmup):
    with hb.Plan(desc, 0) as plan:
        plan.set_forward_model(spectra)
        with torch.cuda.stream(stream):
            for _ in range(warmup):
                plan.estimate(frames, maps, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with torch.cuda.stream(stream):
            for _ in range(steps):
                plan.estimate(frames, maps, stream)
        torch.cuda.synchronize()
        return steps * frames.shape[0] / (time.perf_counter() - t0)


def table1_analogue(a, hb, torch, synth, frames, maps, stream, settings):
    """The paper's speed comparison in kind, on the same frames and grid:
    posterior on every pixel (levels 0), the proposed method with 1 and 3 Haar
    levels, and Tikhonov on every coefficient."""
    H, W = frames.shape[1], frames.shape[2]
    modes = {"bayes_full_resolution": dict(levels=0), "proposed_w1": dict(levels=1),
             "proposed_w3": dict(levels=3), "tikhonov": dict(levels=1, lowpass=hb.HB_LOWPASS_TIKHONOV)}
    out = {}
    for name, m in modes.items():
        desc = hb.make_desc(W, H, levels=m["levels"], dtype=a.dtype, max_batch=frames.shape[0], grid_thb=a.grid,
                            grid_so2=a.grid, lam=settings["lam"], sigma=settings["sigma"],
                            lowpass=m.get("lowpass", hb.HB_LOWPASS_BAYES))
        steps = 3 if m["levels"] == 0 else 10
        out[name] = round(time_plan(hb, torch, desc, synth.spectra(), frames, maps, stream, steps, 1), 2)
        log(f"table 1 analogue: {name} {out[name]} frames/s", a.quiet)
    base = out["bayes_full_resolution"]
    pbase = PAPER_TABLE1_HZ["bayes_full_resolution"]
    return {"frames_per_s": out, "speedup_vs_full_resolution": {k: round(v / base, 2) for k, v in out.items()},
            "paper_hz": PAPER_TABLE1_HZ,
            "paper_speedup_vs_full_resolution": {k: round(v / pbase, 2) for k, v in PAPER_TABLE1_HZ.items()},
            "grid": f"{a.grid}x{a.grid}", "frames": "the benchmark's 1920x1080 frames"}


SERVE_MAX_BATCH = {(480, 640): 8, (1024, 1280): 6, (1080, 1920): 4, (2160, 3840): 2}


def serving(a):
    """16 Poisson camera streams of mixed resolution at 30 fps, FP16 frames."""
    import torch
    from paper_1706_07263_amd import synth
    from paper_1706_07263_amd.serve import GpuExecutor, Server, render_sources, workload_requests
    reqs, offered = workload_requests(a.serve_warmup + a.serve_seconds)
    classes = sorted(offered, key=lambda c: c.pixels)
    log(f"serving: rendering {len(classes)} source frames", a.quiet)
    raw = render_sources(classes, n_sources=1, workers=8)
    sources = {c: torch.from_numpy(v).pin_memory() for c, v in raw.items()}
    ex = GpuExecutor(synth.spectra(), sources)
    srv = Server(ex, {c: SERVE_MAX_BATCH[(c.height, c.width)] for c in classes},
                 hbm_budget=int(a.serve_budget_gib * (1 << 30)), offered=offered, max_lanes=2)
    log(f"serving: {len(srv.lanes)} lanes, {srv.used / 2**30:.2f} GiB; {len(reqs)} frames over "
        f"{a.serve_warmup + a.serve_seconds:.1f} s", a.quiet)
    rep = srv.run(reqs, warmup_s=a.serve_warmup)
    srv.close()
    out = rep.summary()
    out["streams"] = 16
    out["offered_pairs_per_s"] = sum(offered.values())
    out["offered_mpixel_per_s"] = round(sum(r.cls.pixels for r in reqs) / (a.serve_warmup + a.serve_seconds) / 1e6, 1)
    out["window_s"] = a.serve_seconds
    log(f"serving: p50 {out['p50_ms']} ms, p99 {out['p99_ms']} ms, {out['mpixel_per_s']} Mpixel/s", a.quiet)
    return out


def sequence(a, torch, hb, synth, hbtest):
    """Frames 0..N-1 of the 1920x1080 video rendered once and kept in HBM,
    then estimated in order at batch 1, 4 and 16 (the last call of a pass
    takes what is left), each pass timed on the host clock between device
    synchronisations after one untimed call."""
    H, W, n = 1080, 1920, a.sequence
    dev = torch.device("cuda:0")
    parts = []
    for s0 in range(0, n, 32):
        idx = list(range(s0, min(n, s0 + 32)))
        parts.append(hbtest.to_device(render_video(idx, a.dtype, workers=16), a.dtype))
        log(f"rendered frames {idx[0]}..{idx[-1]}", a.quiet)
    frames = torch.cat(parts)
    del parts
    settings = dict(synth.config3((0,), dtype=a.dtype).plan)
    fps, mpx = {}, {}
    for B in (1, 4, 16):
        maps = [torch.empty((B, H, W), device=dev, dtype=torch.float32) for _ in range(4)]
        desc = hb.make_desc(W, H, levels=a.levels, dtype=a.dtype, max_batch=B, grid_thb=a.grid,
                            grid_so2=a.grid, lam=settings["lam"], sigma=settings["sigma"], grid_split=a.split)
        with hb.Plan(desc, 0) as plan:
            plan.set_forward_model(synth.spectra())
            stream = torch.cuda.Stream(dev)
            with torch.cuda.stream(stream):
                plan.estimate(frames[:B], maps, stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with torch.cuda.stream(stream):
                for s0 in range(0, n, B):
                    plan.estimate(frames[s0:s0 + B], maps, stream)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        fps[str(B)] = round(n / dt, 2)
        mpx[str(B)] = round(n * H * W / dt / 1e6, 2)
        log(f"batch {B}: {n} frames in {dt:.3f} s", a.quiet)
    print(json.dumps({"metric": "frames/s and Mpixel/s over the whole video sequence", "frames": n,
                      "frames_per_s": fps, "mpixel_per_s": mpx, "dtype": a.dtype, "data": "synthetic",
                      "config": {"workload": f"1920x1080 video frames 0..{n - 1}, {a.levels} Haar levels, "
                                             f"{a.grid}x{a.grid} THb x SO2 posterior grid, {a.dtype} frames",
                                 "frames_resident_in_hbm": True}}), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported "
              "(each frame and each stream is independent: see the sharding notes)", file=sys.stderr)
        sys.exit(2)
    import torch
    if a.copy_calib_mib:
        n = a.copy_calib_mib * (1 << 20) // 4
        src = torch.arange(n, device="cuda:0", dtype=torch.float32)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes": n * 4, "launches": 3}), flush=True)
        return
    from paper_1706_07263_amd import build as hb_build
    if not os.path.exists(hb_build.LIB):
        import __graft_entry__
        __graft_entry__.build()
    from paper_1706_07263_amd import hb, synth
    from tests import hbtest
    if a.sequence:
        sequence(a, torch, hb, synth, hbtest)
        return

    B = a.batch
    H, W = 1080, 1920
    log(f"generating {B} synthetic 1080p frames", a.quiet)
    idx = [int(i * 300 / B) for i in range(B)]
    wl = synth.config3((0,), dtype=a.dtype)
    wl.frames = render_video(idx, a.dtype)
    settings = dict(wl.plan)
    settings["levels"], settings["grid_thb"], settings["grid_so2"] = a.levels, a.grid, a.grid

    dev = torch.device("cuda:0")
    frames = hbtest.to_device(wl.frames, a.dtype)
    maps = [torch.empty((B, H, W), device=dev, dtype=torch.float32) for _ in range(4)]
    desc = hb.make_desc(W, H, levels=a.levels, dtype=a.dtype, max_batch=B, grid_thb=a.grid,
                        grid_so2=a.grid, lam=settings["lam"], sigma=settings["sigma"], grid_split=a.split)
    plan = hb.Plan(desc, 0).set_forward_model(synth.spectra())
    info = plan.info()
    stream = torch.cuda.Stream(dev)

    log(f"warmup {a.warmup}", a.quiet)
    with torch.cuda.stream(stream):
        for _ in range(a.warmup):
            plan.estimate(frames, maps, stream)
    torch.cuda.synchronize()

    hb.hb_plan_set_timing(plan.handle, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for _ in range(a.steps):
            plan.estimate(frames, maps, stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms, launches = hb.hb_plan_get_timing(plan.handle)
    evaluated, full = hb.hb_plan_get_work(plan.handle)
    hb.hb_plan_set_timing(plan.handle, False)
    log(f"timed {a.steps} steps in {elapsed:.3f} s; stage ms {ms / np.maximum(launches, 1)}", a.quiet)

    fps = a.steps * B / elapsed
    LL = (H >> a.levels) * (W >> a.levels)
    pairs_per_launch = B * LL * a.grid * a.grid
    k2_s = ms[1] / max(launches[1], 1) / 1e3
    # Evaluated pairs per launch (chunks whose weights are exactly zero are
    # skipped; the flops of the roofline are those actually executed).
    eval_per_launch = evaluated / max(launches[1], 1) if evaluated else pairs_per_launch
    achieved = eval_per_launch * FLOPS_PER_PAIR / k2_s / 1e12
    sha = kernel_source_sha()
    default_workload = (B, a.levels, a.grid, a.dtype, a.split) == (16, 2, 256, "f32", 0)
    traffic = PROFILED_POSTERIOR_TRAFFIC if (sha == PROFILED_KERNEL_SHA and default_workload) else None
    roofline = {"bound": "alu", "kernel": "k_posterior", "achieved": round(achieved, 3),
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": traffic, "traffic_unit": "bytes per launch", "avg_launch_ms": round(k2_s * 1e3, 4),
                "evaluated_pairs_per_launch": int(eval_per_launch), "full_grid_pairs_per_launch": pairs_per_launch,
                "evaluated_pairs_per_s": eval_per_launch / k2_s,
                "full_grid_pairs_per_s": pairs_per_launch / k2_s,
                "flops_per_pair": FLOPS_PER_PAIR, "exps_per_pair": EXPS_PER_PAIR}
    stage = {"log_haar_ms": ms[0] / max(launches[0], 1), "posterior_ms": ms[1] / max(launches[1], 1),
             "recompose_ms": ms[2] / max(launches[2], 1), "call_ms": ms[3] / max(launches[3], 1)}
    # K1 algorithmic bytes: frames read; detail part (8 B/px) and the
    # double-float low-pass observation (24 B per low-pass pixel) written.
    k1_bytes = B * H * W * ((12 if a.dtype == "f32" else 6) + 8) + B * LL * 24
    stage["log_haar_GBps"] = k1_bytes / (stage["log_haar_ms"] * 1e-3) / 1e9
    # With one grid split, the MFMA kernel and <= 2 levels the posterior kernel
    # writes the maps itself and the recomposition kernel is not launched.
    stage["recompose_fused"] = bool(info["grid_split"] == 1 and info["posterior_kernel"] == "mfma"
                                    and a.levels <= 2)

    plan.close()

    table1 = None if a.no_table1 else table1_analogue(a, hb, torch, synth, frames, maps, stream, settings)

    # The same frames stored in FP16 (device-side RNE cast), same plan settings.
    half = None
    if a.dtype == "f32":
        frames16 = frames.half()
        desc16 = hb.make_desc(W, H, levels=a.levels, dtype="f16", max_batch=B, grid_thb=a.grid,
                              grid_so2=a.grid, lam=settings["lam"], sigma=settings["sigma"], grid_split=a.split)
        with hb.Plan(desc16, 0) as plan16:
            plan16.set_forward_model(synth.spectra())
            with torch.cuda.stream(stream):
                for _ in range(a.warmup):
                    plan16.estimate(frames16, maps, stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            with torch.cuda.stream(stream):
                for _ in range(a.steps):
                    plan16.estimate(frames16, maps, stream)
            torch.cuda.synchronize()
            fps16 = a.steps * B / (time.perf_counter() - t1)
        half = {"frames_per_s": round(fps16, 3), "vs_fp32": round(fps16 / fps, 4)}
        log(f"fp16 storage: {fps16:.1f} frames/s", a.quiet)
        del frames16
    # End to end with the frames copied from pinned host memory every step
    # (the library takes device pointers, so this is context, not the value):
    # serially on one stream, and overlapped (a copy stream fills one of two
    # device slots while the other is estimated), for FP32 and FP16 storage.
    pcie = None
    if not a.no_table1 and a.dtype == "f32":
        pcie = {"host_bytes_per_frame_f32": H * W * 12, "host_bytes_per_frame_f16": H * W * 6}
        for tag, dev_frames, dt in (("f32", frames, "f32"), ("f16", frames.half(), "f16")):
            host = dev_frames.cpu().pin_memory()
            d_h = hb.make_desc(W, H, levels=a.levels, dtype=dt, max_batch=B, grid_thb=a.grid, grid_so2=a.grid,
                               lam=settings["lam"], sigma=settings["sigma"], grid_split=a.split)
            with hb.Plan(d_h, 0) as plan_h:
                plan_h.set_forward_model(synth.spectra())
                if tag == "f32":
                    pcie["serial_frames_per_s_f32"] = round(
                        host_serial(torch, plan_h, host, dev_frames, maps, stream, a.steps, a.warmup) * B, 2)
                pcie[f"overlapped_frames_per_s_{tag}"] = round(
                    host_overlapped(torch, plan_h, host, dev_frames, maps, stream, a.steps, a.warmup) * B, 2)
            del host
        log(f"frames from pinned host memory (frames/s): {pcie}", a.quiet)

    # Throughput at the batch sizes of the video workload (the first b of the
    # frames above, one plan per batch size).
    sweep = {}
    if not a.no_table1:
        for b in (1, 4, 8, 16):
            if b > B:
                continue
            d = hb.make_desc(W, H, levels=a.levels, dtype=a.dtype, max_batch=b, grid_thb=a.grid,
                             grid_so2=a.grid, lam=settings["lam"], sigma=settings["sigma"])
            sub = frames[:b]
            subm = [m[:b] for m in maps]
            sweep[str(b)] = round(time_plan(hb, torch, d, synth.spectra(), sub, subm, stream, a.steps, a.warmup), 2)
        log(f"batch sweep (frames/s): {sweep}", a.quiet)
    del frames, maps
    torch.cuda.empty_cache()
    serve = serving(a) if a.serve_seconds > 0 else None

    cpu = None
    if a.cpu_seconds > 0:
        cpu = cpu_baseline(a.cpu_seconds, a.levels, a.grid, a.quiet)

    out = {
        "metric": METRIC, "value": round(fps, 3), "unit": "frames/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(elapsed / a.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": a.dtype,
        "data": "synthetic",
        "config": {"workload": f"1920x1080 video frames, {a.levels} Haar levels, {a.grid}x{a.grid} "
                               f"THb x SO2 posterior grid, {a.dtype} frames",
                   "global_batch": B, "frame": "1920x1080", "levels": a.levels,
                   "grid": f"{a.grid}x{a.grid}", "grid_split": info["grid_split"],
                   "posterior_kernel": info["posterior_kernel"], "parallelism": "1 GPU"},
        "mpixel_per_s": round(fps * H * W / 1e6, 2),
        "stages_ms_per_call": {k: round(v, 4) for k, v in stage.items()},
        "roofline": roofline,
        "batch_sweep_frames_per_s": sweep or None,
        "pinned_host_input": pcie,
        "fp16_storage": half,
        "table1_analogue": table1,
        "cpu_baseline": cpu,
        "p99_latency_ms_16_streams": serve["p99_ms"] if serve else None,
        "serving": serve,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
