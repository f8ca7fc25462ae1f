"""Throughput benchmark of the haemoglobin-estimation hot path on one MI355X.

One step = one hb_estimate_frames call over a batch of synthetic 1920x1080
frames (log-attenuation + 2-level Haar + Tikhonov, posterior over a 256x256
THb x SO2 grid, inverse Haar and maps), frames already resident in HBM.

Prints one JSON line with frames/s (value), Mpixel/s, the roofline of the
dominant kernel (the posterior) from per-kernel HIP events recorded on the
launch stream, and the FP64 CPU oracle timed on a bounded sample of the same
workload.  Further legs (``--legs``) add the posterior without skipping and
with exact skipping, half-precision storage,
the stereo 1280x1024 pair with a 512x512 grid, a batch sweep, the Table 1
analogue, frames from host memory and the 16-stream serving runs.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/s + Mpixel/s at 1920x1080 on 1 GPU; p99 frame latency, 16 streams"
LEGS = ("main", "modes", "fp16", "config4", "sweep", "table1", "pcie", "serve", "cpu")

# Algorithmic operations per (LL pixel, grid node) pair of the posterior:
# 3 sub + 3 mul + 2 add (squared distance), 1 mul (-1/(2 sigma^2)), 1 sub (the
# reference), 1 add + 2 mul + 2 add (three moments) = 15 flops, plus one exp.
# The MFMA kernel forms the first 10 (the logit) on the matrix cores from
# exact bf16 splits and the 5 moment flops on the VALU.
FLOPS_PER_PAIR = 15
FLOPS_PER_PAIR_MFMA = 10
FLOPS_PER_PAIR_VALU = 5
EXPS_PER_PAIR = 1
FP32_VECTOR_PEAK_TFLOPS = 157.3        # MI355X FP32 vector peak (context; the measured mix ceiling is the peak)
# Roofline of the posterior: its chunk evaluation (one 16-node chunk against
# one 16-pixel block = 256 pairs: one bf16 16x16x32 MFMA, four v_exp_f32 and
# nine FP32 VALU instructions) measured with no memory traffic by the `mix`
# microbenchmark (paper_1706_07263_amd/ceiling.py, csrc/hb_ceiling.hip) at
# the kernel's six waves per SIMD, on every run: that rate x 15 flops is the
# roofline's peak.  For context, a nominal ceiling from unit counts at
# 2.4 GHz: 16 cycles per MFMA, 8 per v_exp_f32, 4 per FP32 VALU instruction
# (16 lanes per SIMD) = 84 cycles per chunk-block; on the box the FP32 FMA
# issues faster than that (the `fma` microbenchmark), so the measured mix
# ceiling is the higher, and binding, one.
MFMA_CYCLES, FMA_CYCLES, EXP_CYCLES = 16, 4, 8
CHUNK_BLOCK_CYCLES = MFMA_CYCLES + 4 * EXP_CYCLES + 9 * FMA_CYCLES      # 84
N_SIMD, CLOCK_HZ = 1024, 2.4e9
NOMINAL_CEILING_PAIRS_PER_S = 256 * N_SIMD * CLOCK_HZ / CHUNK_BLOCK_CYCLES      # 7.49e12
# HBM bytes per posterior launch of the default workload (16 frames), from the
# rocprofv3 FETCH_SIZE/WRITE_SIZE runs summarised in profiles/, valid for the
# device sources whose combined sha256 (kernel_source_sha) starts with
# PROFILED_KERNEL_SHA; reported as null for any other source or workload.
PROFILED_KERNEL_SHA = "53f13351ed65cd57"
PROFILED_POSTERIOR_TRAFFIC = 1186.5e6
KERNEL_SOURCES = ("hb_kernels.hip", "hb_internal.h", "hb_df.h")


def kernel_source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1706_07263_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # The GPU's clocks take some 50 ms of continuous work to settle after an
    # idle spell (per-call times fall by 10% over that span): the default
    # warm-up covers it.
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--levels", type=int, default=2)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--split", type=int, default=0)
    ap.add_argument("--legs", default="all",
                    help="comma-separated legs to run besides the timed workload: " + ",".join(LEGS[1:]) +
                         " ('all' = every leg, 'main' = only the timed workload)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample on all host threads (0 = skip)")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=8.0,
                    help="duration of each 16-stream serving run (0 = skip)")
    ap.add_argument("--serve-warmup", type=float, default=2.0)
    ap.add_argument("--serve-budget-gib", type=float, default=48.0)
    ap.add_argument("--serve-sources", type=int, default=4, help="distinct pre-rendered frames per class")
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="offered load of the loaded serving run as a fraction of the measured "
                         "saturated throughput of the same stream mix")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--sequence", type=int, default=0,
                    help="only time the first N frames of the video, all resident in HBM, "
                         "at batch 1, 4 and 16 (one JSON line)")
    ap.add_argument("--cpu-probe-rows", type=int, default=0, help=argparse.SUPPRESS)
    a = ap.parse_args(argv)
    a.leg_set = set(LEGS) if a.legs == "all" else ({"main"} | set(x for x in a.legs.split(",") if x))
    unknown = a.leg_set - set(LEGS)
    if unknown:
        ap.error(f"unknown legs {sorted(unknown)}")
    return a


def log(msg, quiet=False):
    if not quiet:
        print(msg, file=sys.stderr, flush=True)


def frames_to_device(frames: np.ndarray, dtype: str):
    """[n][H][W][3] storage-dtype array -> contiguous device tensor (bf16 as int16 bits)."""
    import torch
    if dtype == "bf16":
        return torch.from_numpy(np.ascontiguousarray(frames).view(np.int16)).cuda()
    return torch.from_numpy(np.ascontiguousarray(frames)).cuda()


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


def _render_config4(dtype):
    from paper_1706_07263_amd import synth
    return synth.config4(dtype).frames


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle
# ---------------------------------------------------------------------------

def _oracle_inputs(levels: int, grid: int, rows: int):
    from oracle import hb_oracle as orc
    from paper_1706_07263_amd import synth
    sp = synth.spectra()
    s = synth.plan_settings(levels=levels, grid=grid)
    params = orc.Params(width=1920, height=rows, levels=levels, grid_thb=grid, grid_so2=grid,
                        thb_min=s["thb_min"], thb_max=s["thb_max"], so2_min=s["so2_min"], so2_max=s["so2_max"],
                        lambda_rel=s["lam"], sigma=s["sigma"])
    model = orc.Model(sp.eps_hb, sp.eps_hbo2, sp.response, sp.path_length_cm)
    return orc, params, model


def cpu_probe(rows: int, levels: int, grid: int) -> None:
    """Child process: time the oracle on rows 0..rows-1 of video frame 0 with
    the threads OpenMP gives it (OMP_NUM_THREADS), print one JSON line."""
    from paper_1706_07263_amd import synth
    fr = synth.config3((0,)).frames[:, :rows].astype(np.float64)
    orc, params, model = _oracle_inputs(levels, grid, rows)
    t0 = time.perf_counter()
    orc.estimate(params, model, fr)
    dt = time.perf_counter() - t0
    print(json.dumps({"rows": rows, "seconds": dt, "threads": orc.threads()}), flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(target_s: float, levels: int, grid: int, quiet: bool):
    """Time the FP64 oracle on the benchmark's video frames on all host
    threads (a whole-width row band of frame 0 sized for about target_s, or
    whole frames 0, 1, ... when one frame takes less), and on one thread in a
    child process (a 16-row band)."""
    from paper_1706_07263_amd import synth
    orc, _, model = _oracle_inputs(levels, grid, 8)
    b = 1 << levels
    fr = synth.config3((0,)).frames.astype(np.float64)

    def timed(rows, frames):
        _, params, _ = _oracle_inputs(levels, grid, rows)
        t0 = time.perf_counter()
        orc.estimate(params, model, frames[:, :rows])
        return time.perf_counter() - t0

    rows = 4 * b
    dt = timed(rows, fr)
    rows = int(min(1080, max(b, rows * target_s / max(dt, 1e-3)))) // b * b
    rows = max(rows, b)
    dt = timed(rows, fr)
    lp = (rows // b) * (1920 // b)
    if rows == 1080 and dt < 0.5 * target_s:
        # whole video frames 0, 150, 299 (more, spread over the sequence, if
        # they take less than the target), each timed alone; the median
        idx = [0, 150, 299] if dt * 3 >= 0.5 * target_s else \
            [int(i * 299 / (n - 1)) for n in [int(min(9, round(target_s / dt)))] for i in range(n)]
        frs = render_video(idx, "f32").astype(np.float64)
        times = [timed(1080, frs[i:i + 1]) for i in range(len(idx))]
        dt = float(np.median(times))
        out = {"value": 1.0 / dt, "unit": "frames/s", "cores": orc.threads(), "kind": "oracle",
               "sample": f"video frames {', '.join(map(str, idx))} (1920x1080, {(1080 // b) * (1920 // b)} "
                         f"low-pass pixels x {grid * grid} nodes each), each timed alone: median {dt:.2f} s "
                         f"of {', '.join(f'{t:.2f}' for t in times)} s"}
    else:
        out = {"value": (rows / 1080.0) / dt, "unit": "frames/s", "cores": orc.threads(), "kind": "oracle",
               "sample": f"rows 0..{rows - 1} of frame 0 (1920x{rows} px, {lp} low-pass pixels x "
                         f"{grid * grid} nodes), {dt:.2f} s, scaled by {rows}/1080"}
    log(f"cpu oracle: {out['sample']} on {orc.threads()} threads", quiet)
    # one thread, in a child process (OpenMP's thread count is fixed at start-up)
    rows1 = 4 * b
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-probe-rows", str(rows1),
                        "--levels", str(levels), "--grid", str(grid)], env=env, capture_output=True,
                       text=True, timeout=600)
    one = None
    if r.returncode == 0 and r.stdout.strip():
        p = json.loads(r.stdout.strip().splitlines()[-1])
        pairs = (rows1 // b) * (1920 // b) * grid * grid
        one = {"frames_per_s": (rows1 / 1080.0) / p["seconds"], "threads": p["threads"],
               "pairs_per_s": pairs / p["seconds"],
               "sample": f"rows 0..{rows1 - 1} of frame 0, {p['seconds']:.2f} s, scaled by {rows1}/1080"}
        log(f"cpu oracle, one thread: {one}", quiet)
    out["cpu_model"] = cpu_model()
    out["one_thread"] = one
    return out


# ---------------------------------------------------------------------------
# GPU legs
# ---------------------------------------------------------------------------

PAPER_TABLE1_HZ = {"bayes_full_resolution": 3.54, "proposed_w1": 12.7, "proposed_w3": 14.4, "tikhonov": 43.5}


def make_desc(hb, a, W, H, B, dtype=None, **kw):
    from paper_1706_07263_amd import synth
    s = synth.plan_settings(levels=kw.pop("levels", a.levels), grid=kw.pop("grid", a.grid))
    return hb.make_desc(W, H, levels=s["levels"], dtype=dtype or a.dtype, max_batch=B, grid_thb=s["grid_thb"],
                        grid_so2=s["grid_so2"], lam=s["lam"], sigma=s["sigma"],
                        grid_split=kw.pop("grid_split", a.split), **kw)


def run_timed(hb, torch, plan, frames, maps, stream, steps, warmup, call_ms=None):
    """Warm-up calls, then `steps` calls timed on the host clock between device
    synchronisations, with the plan's per-kernel HIP events and pair counter.
    Returns (seconds, stage ms per call, evaluated pairs per posterior launch,
    full-grid pairs per launch, pixels per launch whose posterior sums took
    double-float logits for lying far from the grid's nodes).  With a list `call_ms`, HIP events on the
    launch stream around every timed call append each call's milliseconds."""
    with torch.cuda.stream(stream):
        for _ in range(warmup):
            plan.estimate(frames, maps, stream)
    torch.cuda.synchronize()
    hb.hb_plan_set_timing(plan.handle, True)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)] if call_ms is not None else None
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for i in range(steps):
            if ev:
                ev[i][0].record(stream)
            plan.estimate(frames, maps, stream)
            if ev:
                ev[i][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if ev:
        call_ms.extend(e0.elapsed_time(e1) for e0, e1 in ev)
    ms, launches = hb.hb_plan_get_timing(plan.handle)
    evaluated, full = hb.hb_plan_get_work(plan.handle)
    far = hb.hb_plan_get_far_pixels(plan.handle)
    hb.hb_plan_set_timing(plan.handle, False)
    per = ms / np.maximum(launches, 1)
    n = max(launches[1], 1)
    return elapsed, per, evaluated / n, full / n, far / n


def time_plan(hb, torch, desc, spectra, frames, maps, stream, steps, warmup):
    with hb.Plan(desc, 0) as plan:
        plan.set_forward_model(spectra)
        elapsed, *_ = run_timed(hb, torch, plan, frames, maps, stream, steps, warmup)
        return steps * frames.shape[0] / elapsed


def posterior_modes(a, hb, torch, synth, frames, maps, stream, mix_rate):
    """The same frames with exact skipping (tolerance 0: only chunks whose
    float32 weights are all zero; bit-identical to no skipping) and with no
    skipping at all (every pair of the grid evaluated)."""
    B, H, W = frames.shape[0], frames.shape[1], frames.shape[2]
    out = {}
    for name, tol, steps in (("exact_skip", 0.0, 6), ("full_grid", -1.0, 3)):
        with hb.Plan(make_desc(hb, a, W, H, B, posterior_tolerance=tol), 0) as plan:
            plan.set_forward_model(synth.spectra())
            elapsed, per, ev, full, _ = run_timed(hb, torch, plan, frames, maps, stream, steps, 1)
        k2 = per[1] * 1e-3
        out[name] = {"posterior_tolerance_um": tol, "skip_log2": "none" if tol < 0 else 160,
                     "frames_per_s": round(steps * B / elapsed, 2), "call_ms": round(per[3], 4),
                     "posterior_ms": round(per[1], 4), "evaluated_fraction": round(ev / full, 5),
                     "evaluated_pairs_per_s": ev / k2,
                     "achieved_tflops": round(ev * FLOPS_PER_PAIR / k2 / 1e12, 3),
                     "frac_of_ceiling": round(ev / k2 / mix_rate, 4)}
        log(f"posterior {name}: {out[name]}", a.quiet)
    return out


def table1_analogue(a, hb, torch, synth, frames, maps, stream):
    """The paper's speed comparison in kind, on the same frames and grid:
    posterior on every pixel (levels 0), the proposed method with 1 and 3 Haar
    levels, and Tikhonov on every coefficient."""
    B, H, W = frames.shape[0], frames.shape[1], frames.shape[2]
    modes = {"bayes_full_resolution": dict(levels=0), "proposed_w1": dict(levels=1),
             "proposed_w3": dict(levels=3), "tikhonov": dict(levels=1, lowpass=hb.HB_LOWPASS_TIKHONOV)}
    out = {}
    for name, m in modes.items():
        desc = make_desc(hb, a, W, H, B, levels=m["levels"], lowpass=m.get("lowpass", hb.HB_LOWPASS_BAYES))
        steps = 3 if m["levels"] == 0 else 10
        out[name] = round(time_plan(hb, torch, desc, synth.spectra(), frames, maps, stream, steps, 1), 2)
        log(f"table 1 analogue: {name} {out[name]} frames/s", a.quiet)
    base = out["bayes_full_resolution"]
    pbase = PAPER_TABLE1_HZ["bayes_full_resolution"]
    return {"frames_per_s": out, "speedup_vs_full_resolution": {k: round(v / base, 2) for k, v in out.items()},
            "paper_hz": PAPER_TABLE1_HZ,
            "paper_speedup_vs_full_resolution": {k: round(v / pbase, 2) for k, v in PAPER_TABLE1_HZ.items()},
            "grid": f"{a.grid}x{a.grid}", "frames": "the benchmark's 1920x1080 frames"}


def config4_storage(a, hb, torch, synth, stream):
    """The stereo 1280x1024 pair with a 512x512 grid and one Haar level, the
    frames stored in FP32, FP16 and BF16 (each rendered from FP64 with one
    rounding); both views in one call."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    ctx = multiprocessing.get_context("spawn")
    dtypes = ("f32", "f16", "bf16")
    with ProcessPoolExecutor(max_workers=3, mp_context=ctx) as pool:
        host = dict(zip(dtypes, pool.map(_render_config4, dtypes)))
    H, W = 1024, 1280
    maps = [torch.empty((2, H, W), device="cuda", dtype=torch.float32) for _ in range(4)]
    out = {}
    for dt in dtypes:
        fr = frames_to_device(host[dt], dt)
        with hb.Plan(make_desc(hb, a, W, H, 2, dtype=dt, levels=1, grid=512, grid_split=0), 0) as plan:
            plan.set_forward_model(synth.spectra())
            elapsed, per, ev, full, _ = run_timed(hb, torch, plan, fr, maps, stream, 10, 2)
        out[dt] = {"frames_per_s": round(20 / elapsed, 2), "call_ms": round(per[3], 4),
                   "log_haar_ms": round(per[0], 4), "posterior_ms": round(per[1], 4),
                   "evaluated_fraction": round(ev / full, 5)}
        del fr
    for dt in ("f16", "bf16"):
        out[dt]["vs_f32"] = round(out[dt]["frames_per_s"] / out["f32"]["frames_per_s"], 4)
    out["workload"] = "stereo pair 1280x1024 (2 frames per call), 1 Haar level, 512x512 grid"
    log(f"config 4 storage: {out}", a.quiet)
    return out


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


SERVE_MAX_BATCH = {(480, 640): 8, (1024, 1280): 6, (1080, 1920): 4, (2160, 3840): 2}


def serving(a):
    """16 Poisson camera streams of mixed resolution, with a.serve_sources
    distinct frames per class: FP16 frames at 30 frames/s per stream; the
    plain FP32 path on the same streams (FP32 frames, twice the bytes per
    frame); then the FP16 mix offered far above capacity for a short run,
    whose served rate is the saturated throughput (every lane busy, full
    batches); then a run offered a.serve_load of that throughput (rho),
    stepped down to 0.5 if the queues do not keep up."""
    import torch
    from paper_1706_07263_amd import synth
    from paper_1706_07263_amd.serve import GpuExecutor, Server, render_sources, workload_requests
    dur = a.serve_warmup + a.serve_seconds
    n_streams = sum(cnt for cnt, *_ in synth.SERVE_CLASSES)

    def server(dtype):
        _, offered = workload_requests(dur, n_sources=a.serve_sources, dtype=dtype)
        classes = sorted(offered, key=lambda c: c.pixels)
        log(f"serving: rendering {len(classes)} x {a.serve_sources} {dtype} source frames", a.quiet)
        raw = render_sources(classes, n_sources=a.serve_sources, workers=8)
        sources = {c: torch.from_numpy(v).pin_memory() for c, v in raw.items()}
        srv = Server(GpuExecutor(synth.spectra(), sources), {c: SERVE_MAX_BATCH[(c.height, c.width)] for c in classes},
                     hbm_budget=int(a.serve_budget_gib * (1 << 30)), offered=offered, max_lanes=2)
        log(f"serving {dtype}: {len(srv.lanes)} lanes, {srv.used / 2**30:.2f} GiB", a.quiet)
        return srv

    def point(srv, fps, duration, warmup, dtype="f16"):
        reqs, off = workload_requests(duration, fps=fps, n_sources=a.serve_sources, dtype=dtype)
        rep = srv.run(reqs, warmup_s=warmup)
        out = rep.summary()
        out["fps_per_stream"] = round(fps, 2)
        out["offered_frames_per_s"] = round(len([r for r in reqs if r.arrival >= warmup]) / (duration - warmup), 2)
        out["offered_pairs_per_s"] = sum(off.values())
        out["offered_mpixel_per_s"] = round(sum(r.cls.pixels for r in reqs) / duration / 1e6, 1)
        out["window_s"] = round(duration - warmup, 3)
        out["sources_per_class"] = a.serve_sources
        out["frame_dtype"] = dtype
        log(f"serving {dtype} at {fps:.1f} frames/s per stream: p50 {out['p50_ms']} ms, p99 {out['p99_ms']} ms, "
            f"{out['frames_per_s']} frames/s served, {out['mpixel_per_s']} Mpixel/s, "
            f"mean batch {out['mean_batch']}, max queue {out['max_queue']}", a.quiet)
        return out

    srv32 = server("f32")
    plain = point(srv32, 30.0, dur, a.serve_warmup, "f32")
    srv32.close()
    del srv32
    torch.cuda.empty_cache()
    srv = server("f16")
    base = point(srv, 30.0, dur, a.serve_warmup)
    base["streams"] = n_streams
    base["fp32_path"] = {k: plain[k] for k in ("frames", "p50_ms", "p99_ms", "max_ms", "frames_per_s",
                                               "mpixel_per_s", "hbm_bytes", "mean_batch", "per_class")}
    # Saturated throughput: the mix offered far above what the lanes can
    # serve (1000 frames/s per stream, several times the capacity) for one
    # second; every frame served over the whole run (arrivals end long before
    # the queues drain, so every lane stays busy) over the run's length is
    # the capacity.
    hi = 1000.0
    sat = point(srv, hi, 1.0, 0.0)
    cap = sat["frames_per_s"] / n_streams          # frames/s per stream at saturation
    loaded = None
    for rho in (a.serve_load, 0.5):
        loaded = point(srv, rho * cap, dur, a.serve_warmup)
        loaded["rho"] = rho
        # kept up: served what was offered, and no queue beyond a few batches
        if loaded["frames_per_s"] >= 0.95 * loaded["offered_frames_per_s"] and loaded["p99_ms"] < 100.0:
            break
    loaded["saturated"] = {"fps_per_stream_offered": round(hi, 1), "frames_per_s": sat["frames_per_s"],
                           "mpixel_per_s": sat["mpixel_per_s"], "mean_batch": sat["mean_batch"]}
    srv.close()
    return base, loaded


def sequence(a, torch, hb, synth):
    """Frames 0..N-1 of the 1920x1080 video rendered once and kept in HBM,
    then estimated in order at batch 1, 4 and 16 (the last call of a pass
    takes what is left), each pass timed on the host clock between device
    synchronisations after an untimed pass over the same frames (the clocks
    settle during it)."""
    H, W, n = 1080, 1920, a.sequence
    dev = torch.device("cuda:0")
    parts = []
    for s0 in range(0, n, 32):
        idx = list(range(s0, min(n, s0 + 32)))
        parts.append(frames_to_device(render_video(idx, a.dtype, workers=16), a.dtype))
        log(f"rendered frames {idx[0]}..{idx[-1]}", a.quiet)
    frames = torch.cat(parts)
    del parts
    fps, mpx = {}, {}
    for B in (1, 4, 16):
        maps = [torch.empty((B, H, W), device=dev, dtype=torch.float32) for _ in range(4)]
        with hb.Plan(make_desc(hb, a, W, H, B), 0) as plan:
            plan.set_forward_model(synth.spectra())
            stream = torch.cuda.Stream(dev)
            with torch.cuda.stream(stream):
                for s0 in range(0, n, B):
                    plan.estimate(frames[s0:s0 + B], maps, stream)
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
    if a.cpu_probe_rows:
        cpu_probe(a.cpu_probe_rows, a.levels, a.grid)
        return
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
    if a.sequence:
        sequence(a, torch, hb, synth)
        return
    legs = a.leg_set

    B = a.batch
    H, W = 1080, 1920
    log(f"generating {B} synthetic 1080p frames", a.quiet)
    idx = [int(i * 300 / B) for i in range(B)]
    dev = torch.device("cuda:0")
    frames = frames_to_device(render_video(idx, a.dtype), a.dtype)
    maps = [torch.empty((B, H, W), device=dev, dtype=torch.float32) for _ in range(4)]
    plan = hb.Plan(make_desc(hb, a, W, H, B), 0).set_forward_model(synth.spectra())
    info = plan.info()
    stream = torch.cuda.Stream(dev)

    log(f"warmup {a.warmup}, timed {a.steps}", a.quiet)
    call_ms = []
    elapsed, per, eval_per_launch, full_per_launch, far_per_launch = run_timed(hb, torch, plan, frames, maps,
                                                                               stream, a.steps, a.warmup, call_ms)
    plan.close()
    log(f"timed {a.steps} steps in {elapsed:.3f} s; stage ms {per}", a.quiet)

    fps = a.steps * B / elapsed
    LL = (H >> a.levels) * (W >> a.levels)
    k2_s = per[1] / 1e3
    eval_rate = eval_per_launch / k2_s
    achieved = eval_per_launch * FLOPS_PER_PAIR / k2_s / 1e12
    sha = kernel_source_sha()
    default_workload = (B, a.levels, a.grid, a.dtype, a.split) == (16, 2, 256, "f32", 0)
    traffic = PROFILED_POSTERIOR_TRAFFIC if (sha == PROFILED_KERNEL_SHA and default_workload) else None
    from paper_1706_07263_amd import ceiling
    ceil = ceiling.ceilings(6)
    log(f"ceilings: {ceil}", a.quiet)
    mix_rate = ceil["mix_pairs_per_s"]
    peak = mix_rate * FLOPS_PER_PAIR / 1e12
    roofline = {
        "bound": "alu", "kernel": "k_posterior", "achieved": round(achieved, 3), "peak": round(peak, 2),
        "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": traffic,
        "traffic_unit": "bytes per launch",
        "peak_basis": f"measured issue ceiling of the posterior's chunk evaluation (1 bf16 16x16x32 MFMA, "
                      f"4 v_exp_f32, 9 FP32 VALU per 256 pairs, no memory, 6 waves per SIMD): "
                      f"{mix_rate:.3e} pairs/s ({ceil['mix_cycles_per_chunk_block']:.1f} SIMD cycles per "
                      f"chunk-block at 2.4 GHz) x {FLOPS_PER_PAIR} flops",
        "unit_of_work": "evaluated (low-pass pixel, grid node) pair; skipped chunks are not counted",
        "avg_launch_ms": round(per[1], 4), "launches_timed": a.steps,
        "evaluated_pairs_per_launch": int(eval_per_launch), "full_grid_pairs_per_launch": int(full_per_launch),
        "evaluated_fraction": round(eval_per_launch / max(full_per_launch, 1), 5),
        "far_pixels_per_launch": far_per_launch,
        "evaluated_pairs_per_s": eval_rate, "ceiling_pairs_per_s": mix_rate,
        "nominal_ceiling_pairs_per_s": NOMINAL_CEILING_PAIRS_PER_S,
        "frac_of_nominal_ceiling": round(eval_rate / NOMINAL_CEILING_PAIRS_PER_S, 4),
        "full_grid_pairs_per_s_equivalent": full_per_launch / k2_s,
        "flops_per_pair": FLOPS_PER_PAIR, "flops_per_pair_on_mfma": FLOPS_PER_PAIR_MFMA,
        "flops_per_pair_on_valu": FLOPS_PER_PAIR_VALU, "exps_per_pair": EXPS_PER_PAIR,
        "frac_of_fp32_vector_peak": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
    }
    stage = {"log_haar_ms": per[0], "posterior_ms": per[1], "recompose_ms": per[2], "call_ms": per[3],
             "call_ms_median": float(np.median(call_ms)), "call_ms_min": float(np.min(call_ms)),
             "call_ms_max": float(np.max(call_ms))}
    # K1 algorithmic bytes: frames read; detail part (8 B/px) and the
    # double-float low-pass observation (24 B per low-pass pixel) written.
    k1_bytes = B * H * W * ((12 if a.dtype == "f32" else 6) + 8) + B * LL * 24
    stage["log_haar_GBps"] = k1_bytes / (stage["log_haar_ms"] * 1e-3) / 1e9
    # With one grid split, the MFMA kernel and <= 2 levels the posterior kernel
    # writes the maps itself and the recomposition kernel is not launched.
    stage["recompose_fused"] = bool(info["grid_split"] == 1 and info["posterior_kernel"] == "mfma"
                                    and a.levels <= 2)

    modes = None
    if "modes" in legs:
        modes = posterior_modes(a, hb, torch, synth, frames, maps, stream, mix_rate)
        modes["default"] = {"posterior_tolerance_um": 1e-6, "skip_log2": info["skip_log2"],
                            "band_log2": info["band_log2"], "band_chunks_per_wave": info["band_chunks"],
                            "skip_bound_um": info["skip_bound"], "frames_per_s": round(fps, 2),
                            "call_ms": round(per[3], 4), "posterior_ms": round(per[1], 4),
                            "evaluated_fraction": roofline["evaluated_fraction"],
                            "evaluated_pairs_per_s": eval_rate, "achieved_tflops": round(achieved, 3),
                            "frac_of_ceiling": round(eval_rate / mix_rate, 4)}

    table1 = table1_analogue(a, hb, torch, synth, frames, maps, stream) if "table1" in legs else None

    half = None
    if "fp16" in legs and a.dtype == "f32":
        frames16 = frames.half()
        with hb.Plan(make_desc(hb, a, W, H, B, dtype="f16"), 0) as plan16:
            plan16.set_forward_model(synth.spectra())
            e16, *_ = run_timed(hb, torch, plan16, frames16, maps, stream, a.steps, a.warmup)
        fps16 = a.steps * B / e16
        half = {"frames_per_s": round(fps16, 3), "vs_fp32": round(fps16 / fps, 4)}
        log(f"fp16 storage: {fps16:.1f} frames/s", a.quiet)
        del frames16

    # End to end with the frames copied from pinned host memory every step
    # (the library takes device pointers, so this is context, not the value).
    pcie = None
    if "pcie" in legs and a.dtype == "f32":
        pcie = {"host_bytes_per_frame_f32": H * W * 12, "host_bytes_per_frame_f16": H * W * 6}
        for tag, dev_frames, dt in (("f32", frames, "f32"), ("f16", frames.half(), "f16")):
            host = dev_frames.cpu().pin_memory()
            with hb.Plan(make_desc(hb, a, W, H, B, dtype=dt), 0) as plan_h:
                plan_h.set_forward_model(synth.spectra())
                if tag == "f32":
                    pcie["serial_frames_per_s_f32"] = round(
                        host_serial(torch, plan_h, host, dev_frames, maps, stream, a.steps, a.warmup) * B, 2)
                pcie[f"overlapped_frames_per_s_{tag}"] = round(
                    host_overlapped(torch, plan_h, host, dev_frames, maps, stream, a.steps, a.warmup) * B, 2)
            del host
        log(f"frames from pinned host memory (frames/s): {pcie}", a.quiet)

    sweep = None
    if "sweep" in legs:
        sweep = {}
        for b in (1, 4, 8, 16):
            if b > B:
                continue
            sub = frames[:b]
            subm = [m[:b] for m in maps]
            sweep[str(b)] = round(time_plan(hb, torch, make_desc(hb, a, W, H, b), synth.spectra(), sub, subm,
                                            stream, a.steps, a.warmup), 2)
        log(f"batch sweep (frames/s): {sweep}", a.quiet)
    del frames, maps
    torch.cuda.empty_cache()

    c4 = config4_storage(a, hb, torch, synth, stream) if "config4" in legs else None
    torch.cuda.empty_cache()

    serve = serve_load = None
    if "serve" in legs and a.serve_seconds > 0:
        serve, serve_load = serving(a)

    cpu = None
    if "cpu" in legs and a.cpu_seconds > 0:
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
                   "posterior_kernel": info["posterior_kernel"],
                   "posterior_tolerance_um": 1e-6, "skip_log2": info["skip_log2"],
                   "band_log2": info["band_log2"], "band_chunks_per_wave": info["band_chunks"],
                   "parallelism": "1 GPU"},
        "mpixel_per_s": round(fps * H * W / 1e6, 2),
        "stages_ms_per_call": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in stage.items()},
        "roofline": roofline,
        "hbm_roofline": {"bound": "hbm", "kernel": "k_log_haar_reg", "achieved": round(stage["log_haar_GBps"], 1),
                         "peak": 8000.0, "unit": "GB/s", "frac": round(stage["log_haar_GBps"] / 8000.0, 4),
                         "algorithmic_bytes_per_launch": int(k1_bytes),
                         "note": "log-attenuation, Haar, Tikhonov and the detail part: frames read, detail part "
                                 "and double-float observation written"},
        "posterior_modes": modes,
        "ceiling": ceil,
        "batch_sweep_frames_per_s": sweep,
        "pinned_host_input": pcie,
        "fp16_storage": half,
        "config4_storage": c4,
        "table1_analogue": table1,
        "cpu_baseline": cpu,
        "p99_latency_ms_16_streams": serve["p99_ms"] if serve else None,
        "serving": serve,
        "serving_loaded": serve_load,
        "kernel_source_sha": sha,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
