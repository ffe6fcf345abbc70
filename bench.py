#!/usr/bin/env python3
"""Throughput of the ridge-directed circle Hough transform on one MI355X.

Headline (the timed step): one full detection of a 1024x1024 uint16 (12-bit) synthetic frame
with 200 rings (radii 8-60 px, profile sigma 1-2.5 px, amplitude 400-1200 counts, background
ramp 300-600 counts, Poisson shot noise plus read noise sigma 10), radius bins 5-70: ridges,
votes, smoothing, peaks, circle fits, ring list back on the host.  The frame is resident in
HBM before the timed region.  Kernel durations come from HIP events recorded on the
library's stream around each launch inside the timed region.

Also reported, on the same GPU:
  - the same plain step replayed from the captured HIP graph;
  - batched: 64 frames of the headline kind in one launch sequence (graph replay);
  - uneven batch: 64 uint16 frames of sizes from {512^2, 1024x768, 1280x1024, 2048x1088}
    with 50-800 rings each;
  - differentiable: 16 float32 1024^2 frames with 300 rings each: detection, soft
    accumulator + ring-profile loss forward and backward, 20 Levenberg-Marquardt steps per
    detected ring, and the accuracy of refined vs algebraic-fit rings against the truth;
  - stream: the whole 2000-frame 2048^2 uint16 sequence with 1000 moving rings (rendered on
    the GPU before the timed region and resident in HBM), 32 frames per launch, refinement of
    all detections, linking of the refined rings into tracks with depths, link accuracy
    against the generator's truth over the whole sequence;
  - edges: the plain step with directed edges (gradient magnitude) on the headline frame;
  - the dominant kernel's roofline figures, against the LDS datapath and against the LDS
    atomic rate measured on the same GPU;
  - the CPU oracle timed on a bounded sample of the headline workload (one process, and a
    pool of processes over frames, the paper's scaling model), and its agreement with the
    GPU on the headline frame.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing
import os
import re
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# The fused vote / smoothing / peak kernel runs out of LDS (the accumulator never reaches HBM):
# its ceiling is the LDS datapath, 256 CUs x 32 banks x 4 bytes per clock at 2.4 GHz (GB/s)
LDS_PEAK_GBS = 256 * 32 * 4 * 2.4
POOL_MAX = 16        # worker processes at most (the host share of one GPU)
LM_TOL = 1e-6       # refinement convergence in the stream leg (pixels)
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "vote_c2_1024_traffic.md")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--batch", type=int, default=64, help="frames of the batched measurement (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--uneven", type=int, default=64, help="frames of the uneven batch (0: skip)")
    ap.add_argument("--edge-steps", type=int, default=100, help="plain steps with directed edges (0: skip)")
    ap.add_argument("--step-steps", type=int, default=100,
                    help="plain steps per radius step s = 1, 2, 3 (0: skip)")
    ap.add_argument("--diff-frames", type=int, default=16, help="frames of the differentiable step (0: skip)")
    ap.add_argument("--diff-steps", type=int, default=3)
    ap.add_argument("--stream-frames", type=int, default=2000, help="frames of the stream, 32 per launch (0: skip)")
    ap.add_argument("--coded-launches", type=int, default=4,
                    help="32-frame calls of the stream through encoded ridge streams (0: skip)")
    ap.add_argument("--cpu-frames", type=int, default=8, help="frames of the single-process oracle sample")
    ap.add_argument("--cpu-pool-frames", type=int, default=32, help="frames of the frame-parallel oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only copy a BYTES-sized device buffer 10 times (reference for HBM byte counters)")
    ap.add_argument("--lds-calibration", action="store_true",
                    help="only measure the LDS atomic-add rate (the vote step's ceiling)")
    ap.add_argument("--vote-phases", action="store_true",
                    help="only time the vote kernel's phases on the headline frame and a 2048^2 stream frame")
    return ap.parse_args()


def list_schedule(durations, workers):
    """Makespan when each of `workers` takes the next duration of the list as it becomes free."""
    import heapq
    free = [0.0] * workers
    for d in durations:
        heapq.heapreplace(free, free[0] + float(d))
    return max(free)


def vote_phases():
    """Where the vote kernel's time goes: shader clocks per phase (summed over workgroups,
    shares of their summed lifetimes, clocks per tile) on the headline c2 frame and on the first
    2048^2 stream frame, from the library's phase-timed instance of the kernel (best of 3
    calls by lifetime), and the tiles' own durations from one more such call, with the
    makespans their queue order and a longest-first order would give."""
    import numpy as np
    import torch

    from paper_1310_1371_amd import synth
    from paper_1310_1371_amd.detector import Detector
    det = Detector(max_width=2048, max_height=2048, max_peaks=16384)
    cus = torch.cuda.get_device_properties(0).multi_processor_count      # one vote workgroup per CU
    st = synth.Stream(seed=4)
    xs, ys, zs = st.trajectories(1)
    f5 = torch.empty((2048, 2048), dtype=torch.int16, device="cuda")
    st.render_device(xs[0], ys[0], zs[0], f5, torch.Generator(device="cuda").manual_seed(4))
    f2 = synth.config2()
    out = {}
    for name, img, p in (("c2_1024_u16", torch.from_numpy(f2.image).cuda(), f2.params),
                         ("c5_2048_u16_frame0", f5.view(torch.uint16), dict(synth.PARAMS_C5))):
        det.detect(img, p)
        best = min((det.profile_vote_phases(img, p) for _ in range(3)), key=lambda r: r["lifetime_sum"])
        life = best["lifetime_sum"]
        rec = det.profile_vote_tiles(img, p)
        dur = (rec[:, 3] - rec[:, 2]).astype(float)
        by_queue = dur[np.argsort(rec[:, 1])]
        out_tiles = {"mean_clocks": float(dur.mean()), "max_clocks": float(dur.max()),
                     "median_clocks": float(np.median(dur)), "mean_work_per_cu": float(dur.sum() / cus),
                     # each workgroup takes the next tile when it is free: the makespan of the
                     # launch's queue order with the measured tile times, and of longest first
                     "queue_order_makespan": list_schedule(by_queue, cus),
                     "longest_first_makespan": list_schedule(np.sort(dur)[::-1], cus)}
        out[name] = {"tiles": best["tiles"], "per_tile": out_tiles,
                     "clocks_per_tile": {k: v / best["tiles"] for k, v in best["phases"].items()},
                     "share_of_lifetimes": {k: v / life for k, v in best["phases"].items()},
                     "mean_tile_clocks": sum(best["phases"].values()) / best["tiles"],
                     "workgroup_lifetime_clocks": {"max": best["lifetime_max"], "min": best["lifetime_min"],
                                                   "mean": life / min(cus, best["tiles"])}}
    det.close()
    return out


def lds_ceiling():
    """LDS atomic adds per second at random addresses, with and without the returned value,
    measured by the library's calibration kernel on device 0."""
    import ctypes

    from paper_1310_1371_amd import native as N
    out = {}
    for rtn, name in ((1, "with_return"), (0, "no_return")):
        rate, ms = ctypes.c_double(), ctypes.c_double()
        N.check(N.lib().rd_measure_lds_atomics(0, rtn, ctypes.byref(rate), ctypes.byref(ms)),
                "rd_measure_lds_atomics")
        out[name] = {"atomics_per_s": rate.value, "launch_ms": ms.value}
    return out


def copy_calibration(nbytes: int):
    """A plain device-to-device copy of known size, the reference the HBM byte counters are
    scaled by."""
    import torch
    a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 10}), flush=True)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pool_size():
    return max(1, min(POOL_MAX, len(os.sched_getaffinity(0))))


def pool_map(fn, items):
    """fn over items in worker processes started fresh (spawn): this process may hold a GPU
    context, which a forked child must not inherit."""
    with ProcessPoolExecutor(max_workers=pool_size(), mp_context=multiprocessing.get_context("spawn")) as ex:
        return list(ex.map(fn, items))


def _oracle_timed(args):
    """Worker: the oracle on one frame in one thread; (seconds, rings)."""
    from threadpoolctl import threadpool_limits

    from oracle import ridge_hough as O
    img, params = args
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        rings = O.detect(img, params)
        return time.perf_counter() - t0, rings


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, headline, batch_frames, uneven_frames):
    """The FP64 oracle on bounded samples of the workloads: one process (one thread) on
    `args.cpu_frames` headline-kind frames, the headline frame first, and a pool of processes
    over frames (the paper's scaling model: one process per core) on the c2 batch and on part
    of the uneven batch.  Returns (cpu_baseline, the oracle's rings of the headline frame)."""
    from threadpoolctl import threadpool_limits

    from oracle import ridge_hough as O

    single = [headline] + batch_frames[:max(args.cpu_frames - 1, 0)]
    head_rings = None
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for i, f in enumerate(single):
            r = O.detect(f.image, f.params)
            if i == 0:
                head_rings = r
        dt1 = time.perf_counter() - t0
    px1 = sum(f.image.size for f in single)
    P = pool_size()
    legs = {}
    with ProcessPoolExecutor(max_workers=P, mp_context=multiprocessing.get_context("spawn")) as ex:
        list(ex.map(_oracle_timed, [(f.image[:32, :32].copy(), f.params) for f in batch_frames[:P]]))   # start-up
        for name, frames in (("c2_batch", batch_frames[:args.cpu_pool_frames]),
                             ("uneven_batch", uneven_frames[:max(args.cpu_pool_frames // 2, 1)])):
            if not frames:
                continue
            t0 = time.perf_counter()
            res = list(ex.map(_oracle_timed, [(f.image, f.params) for f in frames]))
            dt = time.perf_counter() - t0
            px = sum(f.image.size for f in frames)
            legs[name] = {"value": px / dt / 1e6, "unit": "Mpixel/s", "frames_per_s": len(frames) / dt,
                          "frames": len(frames), "wall_s": dt, "cpu_s": sum(r[0] for r in res)}
    main = legs.get("c2_batch")
    out = {"value": main["value"] if main else px1 / dt1 / 1e6, "unit": "Mpixel/s", "cores": P if main else 1,
           "kind": "oracle", "cpu_model": _cpu_model(), "host_cpus": len(os.sched_getaffinity(0)),
           "frames_per_s": main["frames_per_s"] if main else len(single) / dt1,
           "sample": (f"{main['frames']} frames of 1024x1024 u16 with 200 rings (seeds 1000..) over a pool of "
                      f"{P} single-thread processes, {main['wall_s']:.1f} s wall, {main['cpu_s']:.1f} s of CPU"
                      if main else f"{len(single)} frames on one thread"),
           "frame_parallel": legs,
           "single_process": {"value": px1 / dt1 / 1e6, "unit": "Mpixel/s", "cores": 1,
                              "frames_per_s": len(single) / dt1, "frames": len(single), "wall_s": dt1,
                              "sample": f"the headline frame and {len(single) - 1} more of its kind, one thread"}}
    return out, head_rings


def parity_block(det, headline, head_rings, frame_dev):
    """The GPU against the oracle on the headline frame: ridge sets (symmetric difference over
    the oracle's ridge count) and ring lists (matched by Hough voxel; unmatched both ways; the
    largest centre / radius difference of the matched rings)."""
    import numpy as np

    from oracle import ridge_hough as O
    p = headline.params
    xs, ys, _, _, _ = O.ridges(headline.image, p)
    xy, _, _ = det.ridges(frame_dev, p)
    so = set(zip(xs.tolist(), ys.tolist()))
    sg = set(map(tuple, xy.cpu().numpy().tolist()))
    gpu = det.detect(frame_dev, p)
    kr = {(int(r["a"]), int(r["b"]), int(r["r_bin"])): r for r in head_rings}
    kg = {(int(r["a"]), int(r["b"]), int(r["r_bin"])): r for r in gpu}
    common = set(kr) & set(kg)
    dmax = max((max(abs(float(kr[k][f]) - float(kg[k][f])) for f in ("cx", "cy", "r")) for k in common),
               default=0.0)
    return {"frame": "the headline frame (1024x1024 u16, seed 1)",
            "ridges_oracle": len(so), "ridges_gpu": len(sg), "ridge_symmetric_difference": len(so ^ sg),
            "ridge_mismatch_pct": 100.0 * len(so ^ sg) / max(len(so), 1),
            "rings_oracle": len(kr), "rings_gpu": len(kg), "rings_matched": len(common),
            "unmatched_oracle_rings": len(set(kr) - set(kg)), "unmatched_gpu_rings": len(set(kg) - set(kr)),
            "max_abs_diff_px": dmax, "tolerance_px": 0.05}


def traffic_from_profile(kernel_src: str):
    """HBM bytes per launch of the vote kernel from the committed PMC summary, if it was taken
    on this exact kernel source; None otherwise."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    text = open(PROFILE_TRAFFIC).read()
    m = re.search(r"source sha256: ([0-9a-f]{64})", text)
    b = re.search(r"bytes per launch: ([0-9.eE+]+)", text)
    if not m or not b:
        return None
    digest = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    return float(b.group(1)) if m.group(1) == digest else None


def match(truth_xy_r, found_xy_r, tol=2.0):
    """Nearest-truth matching of found rings: per found ring the truth index or -1."""
    import numpy as np
    t = np.asarray(truth_xy_r)
    out = []
    for cx, cy, r in found_xy_r:
        d = np.hypot(t[:, 0] - cx, t[:, 1] - cy)
        j = int(np.argmin(d))
        out.append(j if d[j] <= tol and abs(t[j, 2] - r) <= tol else -1)
    return out


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.lds_calibration:
        print(json.dumps({"lds_atomic_rate": lds_ceiling()}), flush=True)
        return
    if args.vote_phases:
        print(json.dumps({"vote_phases": vote_phases()}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: frames are independent, so a batch would shard by frames "
              "across GPUs with no collective; multi-GPU runs are not part of this build.", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    from paper_1310_1371_amd import synth

    # host frames first (worker processes are spawned, never forked from a GPU process)
    log("[bench] host frames")
    f = synth.config2()
    batch_host = pool_map(synth.config2, [1000 + i for i in range(max(args.batch, args.cpu_pool_frames,
                                                                      args.cpu_frames))])
    uneven_host = pool_map(synth.config3_frame, synth.config3_plan(2, args.uneven)) if args.uneven > 0 else []

    import torch

    from paper_1310_1371_amd.detector import Detector

    log("[bench] headline frame")
    H, W = f.image.shape
    p = f.params
    frame = torch.from_numpy(f.image).cuda()
    det = Detector(max_width=2048, max_height=2048, max_peaks=16384, max_frames=max(args.batch, args.uneven, 32, 1),
                   max_batch_pixels=max(args.batch * W * H, 64 * 2048 * 1088, 32 * 2048 * 2048))
    for _ in range(args.warmup):
        rings = det.detect(frame, p)
    st = det.stats()
    n_ridges = st["ridges"]

    # ---- the timed region: plain detections, kernel times from HIP events on the stream
    log("[bench] timed plain steps")
    det.enable_timing(True)
    det.read_timing(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rings = det.detect(frame, p)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timing = det.read_timing(reset=True)
    det.enable_timing(False)
    ms_step = dt / args.steps * 1e3
    px = W * H
    value = px * args.steps / dt / 1e6
    kernel_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in timing.items()}

    # plain detections replayed from the captured graph (no per-kernel events)
    for _ in range(5):
        det.detect(frame, p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        det.detect(frame, p)
    torch.cuda.synchronize()
    dt_graph = time.perf_counter() - t0

    # ---- roofline of the dominant kernel (the vote / smoothing / peak kernel).  Its algorithmic
    # work is the 2 L N_ridge votes, one 4-byte LDS atomic add each; the accumulator's cells and
    # the smoothing taps at hotspots are not counted.  Ceilings: the LDS datapath, and the LDS
    # atomic-add rate at random addresses measured on this GPU by the calibration kernel.
    dom = max(kernel_ms, key=kernel_ms.get)
    L = p["r_max"] - p["r_min"] + 3
    votes = 2 * L * n_ridges
    lds_bytes = 4 * votes
    launch_s = kernel_ms["vote"] * 1e-3
    ceiling = lds_ceiling()
    best_rate = max(v["atomics_per_s"] for v in ceiling.values())
    roof = {"bound": "lds", "kernel": "k_vote (votes, hotspot smoothing, 3x3x3 peaks)" if dom == "vote" else dom,
            "achieved": lds_bytes / launch_s / 1e9,
            "peak": LDS_PEAK_GBS, "unit": "GB/s",
            "work": f"2 x {L} levels x {n_ridges} ridges = {votes} votes per launch, one 4-byte LDS atomic add "
                    f"each ({lds_bytes} B); peak = LDS datapath, 256 CUs x 128 B/clock x 2.4 GHz",
            "votes_per_s": votes / launch_s,
            "launch_ms": kernel_ms["vote"],
            "traffic": traffic_from_profile(os.path.join(ROOT, "paper_1310_1371_amd", "csrc", "vote.hip")),
            "lds_atomic_ceiling": {"atomics_per_s": best_rate, "frac": votes / launch_s / best_rate,
                                   "measured": ceiling,
                                   "how": "rd_measure_lds_atomics: 1024-thread workgroups, 64 KiB of counters "
                                          "each, random 16-bit halves, best of 3 launches"}}
    roof["frac"] = roof["achieved"] / roof["peak"]

    out = {
        "metric": "Mpixel/s + frames/s, ridge-directed Hough at 1024^2; batched vs plain",
        "value": value,
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp64 stencil, int32 votes, int64 fit moments",
        "data": "synthetic",
        "config": {"workload": "plain rd_detect, one 1024x1024 u16 12-bit frame, 200 rings, radii 5-70",
                   "frame": [W, H], "rings_truth": int(len(f.R)), "ridges": n_ridges,
                   "rings_found": int(len(rings))},
        "frames_per_s": args.steps / dt,
        "plain_graph_replay": {"value": px * args.steps / dt_graph / 1e6, "unit": "Mpixel/s",
                               "frames_per_s": args.steps / dt_graph},
        "kernel_ms": kernel_ms,
        "roofline": roof,
        "paper": {"frames_per_s": 6.28, "hardware": "one process on an Intel i7-3820 CPU",
                  "workload": "968x728 frames with about 50 rings (context only)"},
    }

    # ---- batched: 64 frames of the same workload in one launch sequence (graph replay)
    if args.batch > 0:
        log(f"[bench] batched {args.batch} frames")
        frames = [torch.from_numpy(fr.image).cuda() for fr in batch_host[:args.batch]]
        for _ in range(2):
            det.detect_batch(frames, p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            det.detect_batch(frames, p)
        torch.cuda.synchronize()
        dtb = (time.perf_counter() - t0) / args.batch_steps
        # per-kernel times of the batch (timing events in the replayed graph), after the
        # timed batches; every kernel is read on the first call after a reset
        det.enable_timing(True)
        kb = {}
        for _ in range(2):
            det.read_timing(reset=True)
            det.detect_batch(frames, p)
            for k, (ms, n) in det.read_timing(reset=True).items():
                kb.setdefault(k, []).append(ms / max(n, 1))
        det.enable_timing(False)
        kb = {k: min(v) for k, v in kb.items()}
        nr_b = det.stats()["ridges"]
        # the ridge kernel's own figures: 86 fp64 flops per pixel (two 17-tap passes, the
        # Sobel responses, the eigenvalue), and HBM bytes 2 per u16 pixel read + 12 per ridge
        st_s = kb["ridge"] * 1e-3
        out["batched"] = {"frames": args.batch, "value": args.batch * px / dtb / 1e6, "unit": "Mpixel/s",
                          "frames_per_s": args.batch / dtb, "ms_per_batch": dtb * 1e3,
                          "vs_plain": (args.batch * px / dtb / 1e6) / value,
                          "kernel_ms_per_batch": kb,
                          "ridge_kernel": {"bound": "alu", "achieved": 86.0 * args.batch * px / st_s / 1e12,
                                           "peak": 78.6, "unit": "TFLOP/s (fp64)",
                                           "frac": 86.0 * args.batch * px / st_s / 1e12 / 78.6,
                                           "hbm_GBs": (2.0 * args.batch * px + 12.0 * nr_b) / st_s / 1e9,
                                           "hbm_frac": (2.0 * args.batch * px + 12.0 * nr_b) / st_s / 8e12},
                          "workload": f"{args.batch} frames of 1024x1024 u16, 200 rings each (seeds 1000..)"}
        # the same batch with steps 1-2 in float32 (rd_params.curvature_fp32)
        p32 = dict(p, curvature_fp32=1)
        for _ in range(2):
            det.detect_batch(frames, p32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            det.detect_batch(frames, p32)
        torch.cuda.synchronize()
        dt32 = (time.perf_counter() - t0) / args.batch_steps
        det.enable_timing(True)
        det.read_timing(reset=True)
        det.detect_batch(frames, p32)
        ms32 = det.read_timing(reset=True)["ridge"]
        det.enable_timing(False)
        out["batched"]["curvature_fp32"] = {"value": args.batch * px / dt32 / 1e6, "unit": "Mpixel/s",
                                            "ms_per_batch": dt32 * 1e3, "ridge_kernel_ms": ms32[0] / max(ms32[1], 1),
                                            "vs_plain": (args.batch * px / dt32 / 1e6) / value}
        del frames

    # ---- uneven batch, with the launch shapes the autotuner picks for it
    if args.uneven > 0:
        log(f"[bench] uneven batch of {args.uneven}")
        uframes = [torch.from_numpy(fr.image).cuda() for fr in uneven_host]
        upx = sum(fr.image.size for fr in uneven_host)
        pu = uneven_host[0].params
        default_tuning = det.get_tuning()
        tuned = det.autotune(uframes, pu, reps=2)
        for _ in range(2):
            det.detect_batch(uframes, pu)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_steps):
            res = det.detect_batch(uframes, pu)
        torch.cuda.synchronize()
        dtu = (time.perf_counter() - t0) / args.batch_steps
        t0 = time.perf_counter()
        for fr in uframes:
            det.detect(fr, pu)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t0
        det.set_tuning(**default_tuning)
        out["uneven_batch"] = {"frames": args.uneven, "mpixels": upx / 1e6, "value": upx / dtu / 1e6,
                               "unit": "Mpixel/s", "frames_per_s": args.uneven / dtu, "ms_per_batch": dtu * 1e3,
                               "plain_per_frame_frames_per_s": args.uneven / dtp,
                               "rings_found": int(sum(len(r) for r in res)),
                               "rings_placed": int(sum(len(fr.R) for fr in uneven_host)),
                               "autotuned": tuned, "default_tuning": default_tuning,
                               "workload": "64 u16 frames, sizes from {512^2, 1024x768, 1280x1024, 2048x1088}, "
                                           "50-800 rings each (seed 2), launch shapes from rd_autotune"}
        del uframes

    if args.edge_steps > 0:
        log(f"[bench] directed edges, {args.edge_steps} plain steps")
        out["edges"] = edges(det, frame, p, W, H, args, torch)

    if args.step_steps > 0:
        log(f"[bench] radius steps 1-3, {args.step_steps} plain steps each")
        out["radius_step"] = radius_step(det, frame, f, args, np, torch)

    # ---- differentiable step
    if args.diff_frames > 0:
        log(f"[bench] differentiable step on {args.diff_frames} frames")
        out["differentiable"] = differentiable(det, args, np, torch, synth)

    # ---- stream
    if args.stream_frames > 0:
        log(f"[bench] stream of {args.stream_frames} frames")
        out["stream"] = stream(det, args, np, torch, synth)

    if not args.no_cpu_baseline:
        log("[bench] cpu baseline")
        out["cpu_baseline"], head_rings = cpu_baseline(args, f, batch_host, uneven_host)
        out["parity"] = parity_block(det, f, head_rings, frame)
    print(json.dumps(out), flush=True)
    det.close()


def edges(det, frame, p, W, H, args, torch):
    """The plain path with directed edges (gradient magnitude as the measure) on the same
    frame: T = -12 counts / px, a quarter of the weakest ring's smoothed gradient."""
    pe = dict(p, measure=1, k_threshold=-12.0)
    for _ in range(5):
        rings = det.detect(frame, pe)
    n_edge = det.stats()["ridges"]
    det.enable_timing(True)
    det.read_timing(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.edge_steps):
        rings = det.detect(frame, pe)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    timing = det.read_timing(reset=True)
    det.enable_timing(False)
    kms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in timing.items()}
    L = p["r_max"] - p["r_min"] + 3
    lds_bytes = 4 * 2 * L * n_edge          # the votes' LDS bytes, as in the roofline above
    return {"value": W * H * args.edge_steps / dt / 1e6, "unit": "Mpixel/s", "frames_per_s": args.edge_steps / dt,
            "ms_per_step": dt / args.edge_steps * 1e3, "kernel_ms": kms, "edge_pixels": int(n_edge),
            "rings_found": int(len(rings)),
            "vote_roofline_frac": lds_bytes / (kms["vote"] * 1e-3) / 1e9 / LDS_PEAK_GBS,
            "workload": "plain rd_detect with directed edges (measure 1, T = -12 counts/px) on the same "
                        "1024x1024 u16 frame"}


def radius_step(det, frame, f, args, np, torch):
    """The plain path on the headline frame with the radius levels in steps of s = 1, 2, 3
    (levels r_min - s + s l): throughput, the vote kernel's time, and the rings against the
    generator's truth (a ring is found when a detection lies within 2 px of its centre and
    2 px + s/2 of its radius; errors are means over the found rings)."""
    out = {}
    truth = np.stack([f.cx, f.cy, f.R], 1)
    H, W = f.image.shape
    for s in (1, 2, 3):
        ps = dict(f.params, r_step=s, annulus_halfwidth=max(2, (s + 1) // 2 + 1))
        for _ in range(5):
            rings = det.detect(frame, ps)
        det.enable_timing(True)
        det.read_timing(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.step_steps):
            rings = det.detect(frame, ps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        timing = det.read_timing(reset=True)
        det.enable_timing(False)
        found = np.stack([rings["cx"], rings["cy"], rings["r"]], 1).astype(np.float64)
        err = []
        hit = set()
        for j in range(len(truth)):
            d = np.hypot(found[:, 0] - truth[j, 0], found[:, 1] - truth[j, 1])
            k = int(np.argmin(d)) if len(d) else -1
            if k >= 0 and d[k] <= 2.0 and abs(found[k, 2] - truth[j, 2]) <= 2.0 + s / 2:
                hit.add(j)
                err.append(np.abs(found[k] - truth[j]))
        err = np.array(err)
        out[f"s{s}"] = {"value": W * H * args.step_steps / dt / 1e6, "unit": "Mpixel/s",
                        "frames_per_s": args.step_steps / dt,
                        "vote_ms": timing["vote"][0] / max(timing["vote"][1], 1),
                        "levels": (ps["r_max"] - ps["r_min"]) // s + 3, "annulus_halfwidth": ps["annulus_halfwidth"],
                        "rings_found": int(len(rings)), "truth_found": len(hit), "truth": int(len(truth)),
                        "mean_abs_err_px": {"cx": float(err[:, 0].mean()), "cy": float(err[:, 1].mean()),
                                            "r": float(err[:, 2].mean())} if len(err) else None}
    out["workload"] = ("plain rd_detect on the headline 1024x1024 u16 frame with radius levels in steps of s "
                       "(r_step), annulus half-width max(2, ceil(s/2) + 1); accuracy against the generator's rings")
    return out


def differentiable(det, args, np, torch, synth):
    from paper_1310_1371_amd.autograd import ring_fit_loss_batch, soft_accumulator_batch

    fs = synth.config4(seed=3, n_frames=args.diff_frames)
    p = fs[0].params
    s = 1.5
    imgs = [torch.from_numpy(fr.image).cuda() for fr in fs]
    X = torch.stack(imgs)                       # the frames as one [F, H, W] tensor in HBM
    L = p["r_max"] - p["r_min"] + 3
    G = torch.randn((L, 1024, 1024), device="cuda", generator=torch.Generator(device="cuda").manual_seed(0))
    Gb = G.expand(len(fs), -1, -1, -1).contiguous()     # the upstream gradient of every frame's accumulator

    def step():
        # detection, then the soft accumulator and the ring losses of all frames with their
        # gradients (one library call per stage for the whole batch), then 20 LM steps per ring
        res = det.detect_batch(imgs, p)
        th0_all = torch.from_numpy(np.concatenate([np.stack([r["cx"], r["cy"], r["r"]], 1) for r in res])
                                   .astype(np.float64)).cuda()
        fo = torch.from_numpy(np.concatenate([np.full(len(r), i) for i, r in enumerate(res)]).astype(np.int32)).cuda()
        x = X.clone().requires_grad_(True)
        acc = soft_accumulator_batch(x, det, p)
        theta = th0_all.clone().requires_grad_(True)
        loss = ring_fit_loss_batch(x, theta, th0_all, fo, det, s)
        torch.autograd.backward([loss.sum(), acc], [None, Gb])
        theta_ref, lm_loss = det.refine(imgs, th0_all, s, iters=20, frame_of=fo)
        return res, th0_all, theta_ref, (x.grad, theta.grad)

    res, th0_all, theta, _ = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.diff_steps):
        res, th0_all, theta, _ = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.diff_steps
    # refinement alone, all rings of all frames in one launch
    fo = torch.cat([torch.full((len(r),), i, dtype=torch.int32, device="cuda") for i, r in enumerate(res)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.diff_steps):
        det.refine(imgs, th0_all, s, iters=20, frame_of=fo)
    torch.cuda.synchronize()
    dt_lm = (time.perf_counter() - t0) / args.diff_steps

    # accuracy against the generator's rings: algebraic (Kasa) fit vs refined profile fit
    kasa = th0_all.cpu().numpy()
    ref = theta.cpu().numpy()
    err_k, err_r = [], []
    k = 0
    for fr, rings in zip(fs, res):
        n = len(rings)
        truth = np.stack([fr.cx, fr.cy, fr.R], 1)
        idx = match(truth, kasa[k:k + n])
        for j, t in enumerate(idx):
            if t >= 0:
                err_k.append(np.abs(kasa[k + j] - truth[t]))
                err_r.append(np.abs(ref[k + j] - truth[t]))
        k += n
    err_k, err_r = np.array(err_k), np.array(err_r)
    npx = sum(fr.image.size for fr in fs)
    return {"frames": len(fs), "value": npx / dt / 1e6, "unit": "Mpixel/s", "frames_per_s": len(fs) / dt,
            "ms_per_step": dt * 1e3, "ms_refine_20_steps": dt_lm * 1e3, "rings_refined": int(th0_all.shape[0]),
            "rings_truth": int(sum(len(fr.R) for fr in fs)), "rings_matched": int(len(err_k)),
            "mean_abs_err_px": {"kasa": {"cx": float(err_k[:, 0].mean()), "cy": float(err_k[:, 1].mean()),
                                         "r": float(err_k[:, 2].mean())},
                                "refined": {"cx": float(err_r[:, 0].mean()), "cy": float(err_r[:, 1].mean()),
                                            "r": float(err_r[:, 2].mean())}},
            "workload": "16 f32 1024^2 frames, 300 rings each: batched detection, soft accumulator + ring loss "
                        "forward/backward over the batch (one library call per stage), 20 LM steps per detected ring"}


def stream(det, args, np, torch, synth):
    """The whole sequence, 32 frames per launch, frames resident in HBM: rendered on the GPU
    (the stream's model, the device's noise) before the timed region.  Each launch: detection,
    LM refinement of every ring to convergence (a step whose update is within 1e-6 px in every
    component is the last; at most 20), then the refined rings linked into tracks with depths
    on the GPU.
    One untimed warm-up launch on the first 32 frames; then every launch is timed.  Link
    accuracy is scored against the generator's truth afterwards."""
    from paper_1310_1371_amd.tracking import Linker
    st = synth.Stream(seed=4)
    n = args.stream_frames
    p = dict(synth.PARAMS_C5)
    xs, ys, zs = st.trajectories(n)
    t0 = time.perf_counter()
    store = torch.empty((n, st.H, st.W), dtype=torch.int16, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(4)
    for t in range(n):
        st.render_device(xs[t], ys[t], zs[t], store[t], gen)
        if t % 500 == 499:
            log(f"[bench]   rendered {t + 1} frames")
    torch.cuda.synchronize()
    t_render = time.perf_counter() - t0
    frames = store.view(torch.uint16)
    launches = [(k, min(k + 32, n)) for k in range(0, n, 32)]

    steps = []

    def run(linker, k0, k1, keep):
        fb = [frames[i] for i in range(k0, k1)]
        res = det.detect_batch(fb, p)
        th0 = torch.from_numpy(np.concatenate([np.stack([r["cx"], r["cy"], r["r"]], 1) for r in res])
                               .astype(np.float64)).cuda()
        fo = torch.cat([torch.full((len(r),), i, dtype=torch.int32, device="cuda") for i, r in enumerate(res)])
        theta, _, nst = det.refine(fb, th0, 1.5, iters=20, frame_of=fo, tol=LM_TOL, return_steps=True)
        offs = np.zeros(len(res) + 1, dtype=np.int32)
        offs[1:] = np.cumsum([len(r) for r in res])
        dets = theta.float().contiguous()
        ids, z = linker.link(dets, offs)
        if keep is not None:
            keep.append((dets, ids, z, offs))
            steps.append(nst)
        return int(th0.shape[0])

    warm = Linker(gate=8.0, memory=2, depth=(8.0, 0.0, 72.0), max_frames=32, stream=det.stream)
    run(warm, 0, min(32, n), None)
    warm.close()
    linker = Linker(gate=8.0, memory=2, depth=(8.0, 0.0, 72.0), max_frames=32, stream=det.stream)
    linked = []
    n_rings = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (k0, k1) in enumerate(launches):
        n_rings += run(linker, k0, k1, linked)
        if i % 16 == 15:
            log(f"[bench]   launch {i + 1} of {len(launches)}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tracks = linker.info()["tracks"]
    linker.close()
    st_all = torch.cat(steps).double()
    coded = ridge_streams(det, frames, p, np, torch, args.coded_launches) if args.coded_launches > 0 else None
    del store, frames
    truth = np.stack([xs, ys, st.radius(zs)], 2)
    z_truth = np.sqrt((st.radius(zs) - 8.0) / 72.0)
    acc = link_accuracy(np, linked, truth, z_truth)
    # the same refined rings linked with the acceleration model (untimed above; timed here alone)
    acc_lk = Linker(gate=8.0, memory=2, depth=(8.0, 0.0, 72.0), max_frames=32, stream=det.stream,
                    model="acceleration")
    relinked = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for dets, _, _, offs in linked:
        ids, z = acc_lk.link(dets, offs)
        relinked.append((dets, ids, z, offs))
    torch.cuda.synchronize()
    t_acc = time.perf_counter() - t0
    acc_lk.close()
    acc["acceleration_model"] = dict(link_accuracy(np, relinked, truth, z_truth),
                                     ms_per_launch=t_acc / len(linked) * 1e3)
    return {"frames": n, "launches_timed": len(launches), "frames_per_s": n / dt,
            "value": n * st.W * st.H / dt / 1e6, "unit": "Mpixel/s", "ms_per_launch": dt / len(launches) * 1e3,
            "s_total": dt, "rings_detected_and_refined": n_rings, "tracks": tracks, "linking": acc,
            "linking_model": "constant velocity (the acceleration model's figures under linking)",
            "lm_steps": {"tol_px": LM_TOL, "max_steps": 20, "mean": float(st_all.mean()),
                         "max": int(st_all.max()), "at_max": int((st_all >= 20).sum())},
            "s_render_untimed": t_render, "encoded_ridge_streams": coded,
            "workload": f"the whole {n}-frame 2048^2 u16 stream (1000 rings on random walks, radii 8-80), rendered "
                        f"on the GPU and resident in HBM, {len(launches)} launches of up to 32 frames, each: "
                        "batched detection, LM refinement of every detection to convergence (update <= 1e-6 px, "
                        "at most 20 steps), linking (gate 8 px, memory 2) and depth"}


def ridge_streams(det, frames, p, np, torch, launches=4):
    """The stream's frames as encoded ridge streams, 32 frames per call: steps 1-2 and the
    encoding on the GPU (rd_encode_ridges), the streams copied to pinned host memory (the
    transfer the format is for), then steps 3-5 from the host copy (rd_detect_encoded, which
    stages it back).  The rings must equal rd_detect_batch's on the same frames."""
    n = min(launches * 32, frames.shape[0])
    batches = [[frames[i] for i in range(k, min(k + 32, n))] for k in range(0, n, 32)]
    buf = torch.empty(32 * 2 * 2048 * 2048 // 4, dtype=torch.uint8, device="cuda")
    pinned = torch.empty(buf.numel(), dtype=torch.uint8).pin_memory()
    host = pinned.numpy()
    enc, offs = det.encode_ridges(batches[0], p, out=buf)           # warm-up
    same = all(a.tobytes() == b.tobytes() for a, b in
               zip(det.detect_encoded(enc, offs, p), det.detect_batch(batches[0], p)))
    t_enc = t_copy = t_det = 0.0
    nbytes = 0
    for fb in batches:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        enc, offs = det.encode_ridges(fb, p, out=buf)
        t1 = time.perf_counter()
        total = int(offs[-1])
        pinned[:total].copy_(enc[:total])
        t2 = time.perf_counter()
        det.detect_encoded(host[:total], offs, p)
        t3 = time.perf_counter()
        t_enc += t1 - t0
        t_copy += t2 - t1
        t_det += t3 - t2
        nbytes += total
    nf = sum(len(b) for b in batches)
    raw = 2 * 2048 * 2048
    return {"frames": nf, "bytes_per_frame": nbytes / nf, "raw_bytes_per_frame": raw,
            "compression": raw * nf / nbytes, "rings_equal_rd_detect_batch": bool(same),
            "encode_frames_per_s": nf / t_enc, "copy_to_host_GBs": nbytes / t_copy / 1e9,
            "detect_from_host_streams_frames_per_s": nf / t_det,
            "workload": f"{nf} frames of the 2048^2 stream, 32 per call: rd_encode_ridges on the resident frames, "
                        "the streams copied to pinned host memory, rd_detect_encoded from that copy"}


def link_accuracy(np, linked, truth, z_truth):
    """Each detection is given the truth ring whose centre is nearest (within 3 px, radius
    within 3 px); a link (consecutive detections of one track) is right when both ends have
    the same truth ring.  truth: (frames, rings, 3) centre and radius; z_truth: (frames, rings)."""
    from scipy.spatial import cKDTree
    xs, ids, zs, frame = [], [], [], []
    f0 = 0
    for th, i, z, offs in linked:
        xs.append(th.cpu().numpy())
        ids.append(i.cpu().numpy())
        zs.append(z.cpu().numpy())
        frame.append(f0 + np.repeat(np.arange(len(offs) - 1), np.diff(offs)))
        f0 += len(offs) - 1
    x, ids, z, frame = np.concatenate(xs), np.concatenate(ids), np.concatenate(zs), np.concatenate(frame)
    match = np.full(len(x), -1)
    z_true = np.full(len(x), np.nan)
    bounds = np.searchsorted(frame, np.arange(f0 + 1))
    for f in range(f0):
        sel = np.arange(bounds[f], bounds[f + 1])
        if len(sel) == 0:
            continue
        d, j = cKDTree(truth[f, :, :2]).query(x[sel, :2])
        ok = (d < 3.0) & (np.abs(truth[f, j, 2] - x[sel, 2]) < 3.0)
        match[sel[ok]] = j[ok]
        z_true[sel[ok]] = z_truth[f, j[ok]]
    order = np.lexsort((frame, ids))
    same = ids[order][1:] == ids[order][:-1]
    a, b = match[order][:-1][same], match[order][1:][same]
    right = (a == b) & (a >= 0)
    return {"links": int(same.sum()), "links_right": float(right.mean()) if same.any() else None,
            "detections_matched_to_truth": float((match >= 0).mean()),
            "depth_mean_abs_err": float(np.nanmean(np.abs(z - z_true))),
            "tracks_per_truth_ring": float(len(np.unique(ids[ids >= 0])) / truth.shape[1])}


if __name__ == "__main__":
    main()
