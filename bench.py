#!/usr/bin/env python3
"""Tracked frames/s of the per-frame Gauss-Newton tracking step on one MI355X.

Workload (synthetic, seeded): the human-scale body, 50,000 vertices / 99,904
triangles, 24 links, 75 joint parameters, up to 4 influences per vertex,
640x480 float32 depth with 2 mm noise and 25 % zero pixels, a 30-frame
trajectory; 5 Gauss-Newton iterations (pose + per-vertex offsets) per frame.
A step is one frame: every pass of the hot path over one depth image.  All
depth frames are on the GPU before timing starts; the tracker state is reset
to the initial pose at the start of each pass over the 30-frame sequence.

Prints one JSON line with frames/s, per-frame latency percentiles, the
roofline of the dominant kernel (HIP-event timed inside the timed region) and
the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
FP32_VECTOR_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0


def algorithmic_bytes(kernel, V, F, N_px, N_valid, K=4, temporal=False):
    """Minimum HBM bytes of one launch of each timed pass (float32 SoA): the
    method's own traffic, excluding the never-materialised dense J and any
    exhaustive search."""
    return {
        # template, offsets, weights, links in; vertices out
        "skin": V * (36 + 5 * K),
        # vertices, incident faces in; normals out
        "normals": 12 * F + 24 * V,
        # (no launch of its own: the producing kernels count into the
        # buckets, the association lays them out)
        "bucket": 0,
        # depth in, association out, cell records read and the next layout
        # written (16 B per 16 pixels each), the bucketed vertices read once,
        # per-pixel sums; in the same launch the normals (vertices and fans
        # in, normals out)
        "assoc": 10 * N_px + 16 * V + 28 * N_valid + 12 * F + 28 * V,
        # vertices, normals, offsets, template, weights, links, sums in
        "normal_eq": V * (52 + 5 * K),
        "solve": 0,
        "shape": V * (92 + 5 * K + (12 if temporal else 0)),
    }[kernel]


def frame_bytes(V, F, N_px, N_valid, n_iters, K=4, temporal=False, depth_upload=True):
    """Algorithmic bytes of one frame of (pose + offset) iterations: per
    iteration the association (with the normals and the bucket layout),
    normal equations, re-skin at the new pose and the offset step (which
    skins the next surface into the buckets), plus the frame-start skin and
    the depth image."""
    b = lambda k: algorithmic_bytes(k, V, F, N_px, N_valid, K, temporal)  # noqa: E731
    per_iter = b("assoc") + b("normal_eq") + b("skin") + b("shape")
    return n_iters * per_iter + b("skin") + (4 * N_px if depth_upload else 0)


REPEATABLE = ("skin", "assoc", "normal_eq", "solve")

# sources whose change invalidates a kernel's committed counter reading
KERNEL_SOURCES = {
    "assoc": ["association.hip", "common.h", "surface.h"],
    "normal_eq": ["normal_eq.hip", "common.h"],
    "solve": ["solve.hip", "common.h", "fk.h"],
    "shape": ["solve.hip", "common.h", "surface.h"],
    "skin": ["kinematics.hip", "common.h", "surface.h"],
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_human-50k-640x480.md")


def sources_digest(kernel):
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES.get(kernel, []):
        with open(os.path.join(ROOT, "paper_1711_07999_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` read from the committed hardware
    counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the same counters'
    reading for a copy of known size), or None when there is no reading or the
    kernel's sources changed since it was taken."""
    if kernel not in KERNEL_SOURCES or not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if not line.startswith("traffic:"):
                continue
            kv = dict(item.split("=", 1) for item in line.split()[1:])
            if kv.get("kernel") == kernel:
                return float(kv["bytes"]) if kv.get("sources") == sources_digest(kernel) else None
    return None


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(w, threads, budget_s, max_frames, fp32=False):
    """Frames/s of the oracle (float64, or its float32 instantiation) on the
    first frames of the sequence (at least two), until the time budget is
    spent."""
    import oracle

    used = oracle.set_threads(threads)
    m = oracle.Model(w.body.model)
    th = w.theta0.copy()
    phi = np.zeros((m.V, 3))
    prev = np.zeros((m.V, 3))
    t0 = time.perf_counter()
    n = 0
    while n < max_frames and (n < 2 or time.perf_counter() - t0 < budget_s):
        oracle.track_frame(m, w.body.camera, w.params, th, phi, prev, depth=w.frames[n % len(w.frames)], fp32=fp32)
        n += 1
    dt = time.perf_counter() - t0
    return used, n, dt


def cpu_baseline(w, budget_s=12.0, max_frames=30):
    """The oracle (float64 C++, OpenMP over the pixel and vertex loops) on
    the same frames: all of the host's cores available to this process,
    then one core; and its float32 instantiation on all cores."""
    cores = len(os.sched_getaffinity(0))
    used, n, dt = _oracle_rate(w, cores, budget_s, max_frames)
    used1, n1, dt1 = _oracle_rate(w, 1, budget_s, max_frames)
    used32, n32, dt32 = _oracle_rate(w, cores, budget_s / 2, max_frames, fp32=True)
    return {"value": n / dt, "unit": "frames/s", "cores": used, "kind": "oracle",
            "sample": f"first {n} frames of the same 30-frame sequence, float64 oracle, "
                      f"{used} OpenMP threads, {dt:.1f} s",
            "nproc": os.cpu_count(), "affinity_cores": cores, "cpu_model": _cpu_model(),
            "one_core": {"value": n1 / dt1, "unit": "frames/s", "cores": used1,
                         "sample": f"first {n1} frames, 1 thread, {dt1:.1f} s"},
            "fp32": {"value": n32 / dt32, "unit": "frames/s", "cores": used32,
                     "sample": f"first {n32} frames, float32 instantiation of the oracle, "
                               f"{used32} OpenMP threads, {dt32:.1f} s"}}


def _gram_params(base, gram):
    prm = dict(base)
    prm["gram_mode"] = 1 if gram == "bf16x3" else 0
    if prm["gram_mode"]:
        prm["pose_solve_fp64"] = 1
        prm["shape_solve_fp64"] = 1
    return prm


def _run_frames(T, trk, frames, theta0, nsteps, lat=None):
    """Track `nsteps` frames of the sequence (reset to the initial pose at
    the start of each pass over it); per-frame host latency into `lat`."""
    nseq = len(frames)
    for s in range(nsteps):
        if s % nseq == 0:
            trk.reset(theta0)
        t0 = time.perf_counter()
        rc = trk.frame(frames[s % nseq])
        t1 = time.perf_counter()
        if rc != 0:
            raise RuntimeError(f"frame {s}: {T.track_last_error()}")
        if lat is not None:
            lat.append(t1 - t0)


def _timed_frames(T, trk, frames, theta0, warmup, steps):
    import torch

    _run_frames(T, trk, frames, theta0, max(warmup, 1))
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    _run_frames(T, trk, frames, theta0, steps, lat)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lat_ms = np.array(lat) * 1e3
    return elapsed, lat_ms


def _roof(kind, dom, ms, V, F, N_px, N_valid, P, V_obs, gram_mode, temporal):
    """Roofline of one launch of pass `dom` lasting `ms`."""
    if dom == "solve":
        # dense-equivalent factorisation and two triangular solves, float32
        # vector arithmetic, against the chip's fp32 vector peak
        flops = P ** 3 / 3 + 2 * P * P
        achieved = flops / (ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_VECTOR_PEAK_TFLOPS}
    if dom == "normal_eq" and kind == "mfma":
        flops = P * (P + 1) * V_obs
        peak = BF16_MFMA_PEAK_TFLOPS if gram_mode else FP32_MFMA_PEAK_TFLOPS
        achieved = flops / (ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak}
    b = algorithmic_bytes(dom, V, F, N_px, N_valid, temporal=temporal)
    achieved = b / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS}


def batched_copies(T, w, frames_dev, prm, B, nsat):
    """B streams of the same workload in one server (each its own state,
    started from a slightly different pose and frame), every stream always
    with frames waiting: aggregate frames/s and algorithmic HBM bytes/s of
    the batched launches."""
    import torch

    m, cam = w.body.model, w.body.camera
    V, F, N_px = m["rest_xyz"].shape[0], m["faces"].shape[0], cam["width"] * cam["height"]
    sv = T.track_server_create(dict(prm, active=None), 1 << 38, B)
    try:
        ids = []
        for s in range(B):
            rng = np.random.default_rng(7000 + s)
            th0 = w.theta0 + np.where(w.body.angular, rng.uniform(-0.005, 0.005, len(w.theta0)), 0.0)
            ids.append(T.track_server_open(sv, m, cam, th0))
        nseq = len(frames_dev)
        for s in range(B):   # one frame each to build the launch graphs
            T.track_server_submit(sv, ids[s], frames_dev[s % nseq], tag=-1)
        while T.track_server_info(sv)["frames_pending"]:
            T.track_server_step(sv)
        T.track_server_poll(sv, 4 * B)
        for s in range(B):
            for k in range(1, nsat + 1):
                T.track_server_submit(sv, ids[s], frames_dev[(s + k) % nseq], tag=k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = 0
        while n < B * nsat:
            n += T.track_server_step(sv)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        cs = T.track_server_poll(sv, B * nsat + 16)
        nvalid = float(np.mean([c["n_valid_px"] for c in cs]))
        failed = sum(c["status"] != 0 for c in cs)
    finally:
        T.track_server_destroy(sv)
    fps = n / dt
    fb = frame_bytes(V, F, N_px, nvalid, int(prm["n_iters"]), temporal=prm["lambda_t"] > 0)
    gbs = fps * fb / 1e9
    return {"streams": B, "frames": n, "seconds": dt, "fps": fps, "failed_frames": failed,
            "bytes_per_frame": fb, "achieved_GBs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}


def batched_only(args):
    import torch

    import synth
    from paper_1711_07999_amd import track as T

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = synth.workload_human(n_frames=30)
    frames = [torch.from_numpy(f).to("cuda:0") for f in w.frames]
    prm = _gram_params(w.params, args.gram)
    out = batched_copies(T, w, frames, prm, args.batched, args.batch_frames)
    print(json.dumps({"metric": "batched copies of the human-50k-640x480 workload", "gram": args.gram, **out}),
          flush=True)


def highres(T, stream, args):
    """The high-resolution configuration on its own: 200,000 vertices,
    512x424, 60 frames, offsets under Laplacian and temporal regularisation,
    float64 pose solve; frames/s and per-frame latency of whole frames."""
    import torch

    import synth

    w = synth.workload_highres()
    m, cam = w.body.model, w.body.camera
    frames = [torch.from_numpy(f).to(torch.device("cuda:0")) for f in w.frames]
    trk = T.Tracker(m, cam, w.params, w.theta0, stream=stream.cuda_stream)
    el, lat = _timed_frames(T, trk, frames, w.theta0, max(args.warmup, 1), args.steps)
    trk.close()
    return {"workload": w.name, "value": args.steps / el, "unit": "frames/s",
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "vertices": int(m["rest_xyz"].shape[0]), "triangles": int(m["faces"].shape[0]),
            "depth": f"{cam['width']}x{cam['height']}", "gn_iters_per_frame": int(w.params["n_iters"]),
            "sequence_frames": len(frames), "lambda_t": float(w.params["lambda_t"]),
            "pose_solve": "float64" if w.params.get("pose_solve_fp64") else "float32"}


def highres_only(args):
    import torch

    from paper_1711_07999_amd import track as T

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    stream = torch.cuda.current_stream(torch.device("cuda:0"))
    out = highres(T, stream, args)
    print(json.dumps({"metric": "tracked frames/s + p99 frame latency (high-resolution configuration)", **out}),
          flush=True)


def single_stream(args):
    import torch

    import synth
    from paper_1711_07999_amd import track as T

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    w = synth.workload_human(n_frames=30)
    m, cam = w.body.model, w.body.camera
    V, F, P = m["rest_xyz"].shape[0], m["faces"].shape[0], len(w.theta0)
    N_px = cam["width"] * cam["height"]
    prm = _gram_params(w.params, args.gram)
    temporal = prm["lambda_t"] > 0
    frames = [torch.from_numpy(f).to(dev) for f in w.frames]
    stream = torch.cuda.current_stream(dev)
    trk = T.Tracker(m, cam, prm, w.theta0, stream=stream.cuda_stream)
    nseq = len(frames)

    # warmup: first with every pass timed (per-pass durations inside frames,
    # and the dominant pass), then plain, so the frame graphs are captured
    # before timing
    for k in range(len(T.KERNEL_NAMES)):
        T.track_kernel_timing(trk.ctx, k, True)
    nw = max(args.warmup, 1)
    _run_frames(T, trk, frames, w.theta0, nw)
    per_kernel = {}
    for k, name in enumerate(T.KERNEL_NAMES):
        n, ms = T.track_kernel_time(trk.ctx, k)
        per_kernel[name] = (n, ms)
        T.track_kernel_timing(trk.ctx, k, False)
    # the dominant pass among those a single kernel carries (its launch
    # duration is that kernel's; bucket and shape are two-kernel passes or
    # consume their inputs)
    dom = max(REPEATABLE, key=lambda k: per_kernel[k][1])
    dom_id = T.KERNEL_NAMES.index(dom)

    # timed region: whole frames replayed from their graphs
    elapsed, lat_ms = _timed_frames(T, trk, frames, w.theta0, nw, args.steps)
    stats = trk.state(want_verts=False)[3]
    V_obs, N_valid = stats["n_obs_verts"], stats["n_valid_px"]
    fps = args.steps / elapsed

    # the dominant kernel inside frames: the same frames with that pass's
    # launches bracketed by HIP events stamped by its own dispatch packet
    T.track_kernel_timing(trk.ctx, dom_id, True)
    _run_frames(T, trk, frames, w.theta0, args.inframe_frames)
    n_in, ms_in = T.track_kernel_time(trk.ctx, dom_id)
    T.track_kernel_timing(trk.ctx, dom_id, False)
    avg_in = ms_in / max(n_in, 1)
    # and launched back to back on the state the last frame left (same
    # inputs and launch configuration), one pair of HIP events around them
    last = frames[(args.inframe_frames - 1) % nseq]
    avg_rep = T.track_kernel_bench(trk.ctx, dom_id, last, args.kernel_reps)
    # and from cold caches: before each launch a 512 MiB write evicts the
    # L2s and the 256 MB last-level cache; each launch is timed alone between
    # its own pair of events (so it includes their dispatch, as the in-frame
    # figure does), the same single-launch timing without the eviction beside
    flush = torch.empty(1 << 29, dtype=torch.uint8, device=dev)
    cold, warm1 = [], []
    for _ in range(20):
        flush.zero_()
        cold.append(T.track_kernel_bench(trk.ctx, dom_id, last, 1))
        warm1.append(T.track_kernel_bench(trk.ctx, dom_id, last, 1))
    del flush
    trk.close()

    # The roofline takes the back-to-back figure: a pair of events around a
    # single launch adds the events' own dispatch to the span (several us
    # against the profiler's trace of the same launches), while 200 launches
    # between one pair agree with the trace to within 1 %.  The in-frame
    # event figure stands beside it as an upper bound of the in-frame time.
    kind = "mfma" if dom == "normal_eq" else "hbm"
    roof = _roof(kind, dom, avg_rep, V, F, N_px, N_valid, P, V_obs, prm["gram_mode"], temporal)
    inf = _roof(kind, dom, avg_in, V, F, N_px, N_valid, P, V_obs, prm["gram_mode"], temporal)
    roof.update({"traffic": measured_traffic(dom), "kernel": dom, "avg_launch_ms": avg_rep,
                 "launches": args.kernel_reps,
                 "timing": "back-to-back launches on the last timed frame's inputs, one pair of HIP events",
                 "in_frame_upper_bound": {"avg_launch_ms": avg_in, "launches": n_in, "achieved": inf["achieved"],
                                          "frac": inf["frac"],
                                          "timing": "each in-frame launch between its own pair of HIP events "
                                                    "(includes the events' dispatch)"}})
    cold_ms = float(np.mean(cold))
    cr = _roof(kind, dom, cold_ms, V, F, N_px, N_valid, P, V_obs, prm["gram_mode"], temporal)
    roof["cold_upper_bound"] = {"avg_launch_ms": cold_ms, "launches": len(cold), "achieved": cr["achieved"],
                                "frac": cr["frac"], "single_launch_warm_ms": float(np.mean(warm1)),
                                "timing": "each launch alone between its own pair of HIP events after a 512 MiB "
                                          "write that evicts the caches (includes the events' dispatch); "
                                          "single_launch_warm_ms: the same without the eviction"}

    # every pass inside frames (from the timed warm-up): microseconds per
    # launch and its algorithmic bytes (flops for the Gram) against peak
    passes = {}
    for name, (n, ms) in per_kernel.items():
        if n == 0:
            continue
        us = ms / n * 1e3
        e = {"launches_per_frame": n / nw, "us_per_launch": us}
        if name != "solve":
            b = algorithmic_bytes(name, V, F, N_px, N_valid, temporal=temporal)
            e.update({"bytes_per_launch": b, "GBs": b / (us * 1e-6) / 1e9,
                      "frac_of_hbm_peak": b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS})
        if name == "normal_eq":
            r = _roof("mfma", name, us * 1e-3, V, F, N_px, N_valid, P, V_obs, prm["gram_mode"], temporal)
            e.update({"gram_TFLOPs": r["achieved"], "frac_of_mfma_peak": r["frac"]})
        passes[name] = e

    out = {
        "metric": "tracked frames/s + p99 frame latency (50k-vert body, 640x480 depth)",
        "value": fps,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if not prm["gram_mode"] else "bf16x3+f32",
        "data": "synthetic",
        "config": {"workload": w.name, "vertices": V, "triangles": F, "links": 24, "dof": P,
                   "max_influences": 4, "depth": f"{cam['width']}x{cam['height']}",
                   "gn_iters_per_frame": int(prm["n_iters"]), "sequence_frames": nseq,
                   "gram": args.gram},
        "roofline": roof,
        "passes_in_frame": passes,
        "frame_bytes": frame_bytes(V, F, N_px, N_valid, int(prm["n_iters"]), temporal=temporal),
    }
    out["frame_GBs"] = out["frame_bytes"] * fps / 1e9
    if not args.no_extra:
        # the precision form on the same workload
        other = "bf16x3" if args.gram == "fp32" else "fp32"
        prm2 = _gram_params(w.params, other)
        trk2 = T.Tracker(m, cam, prm2, w.theta0, stream=stream.cuda_stream)
        el2, lat2 = _timed_frames(T, trk2, frames, w.theta0, nw, args.steps)
        trk2.close()
        out[f"{other}_form"] = {"value": args.steps / el2, "unit": "frames/s",
                                "p50_ms": float(np.percentile(lat2, 50)), "p99_ms": float(np.percentile(lat2, 99)),
                                "speedup_vs_main": (args.steps / el2) / fps,
                                "solves": "float64" if other == "bf16x3" else "float32"}
        # the high-resolution configuration
        out["highres"] = highres(T, stream, args)
        # B copies of the workload batched through one server
        out["batched_copies"] = [batched_copies(T, w, frames, prm, B, args.batch_frames) for B in (16, 32)]
        # the serving mix, shortened: 64 streams of six sizes, 45 frames each
        # at 30 frames/s (Poisson), then saturation
        lite = argparse.Namespace(**vars(args))
        lite.streams, lite.frames, lite.sat_frames, lite.seq_frames = 64, 45, 10, 10
        out["serving_mix"] = serve(lite, lite=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------------
# serving: 64 streams of mixed sizes through one server
# ---------------------------------------------------------------------------
SERVE_COMBOS = [(V, W, H, f) for V in (10000, 50000, 200000)
                for (W, H, f) in ((320, 240, 262.5), (640, 480, 525.0))]


def _pingpong(k, n):
    """Frame k of an endless forward-backward walk over n frames."""
    q = k % (2 * n - 2)
    return q if q < n else 2 * n - 2 - q


def serve(args, lite=False):
    """The serving mix: configured load (Poisson arrivals), saturation, and
    unless `lite` the admission run under a 1 GiB budget and the alone-vs-mix
    check.  Prints the JSON line, or with `lite` returns it."""
    import torch

    import synth
    from paper_1711_07999_amd import track as T

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    log = lambda msg: print(f"[serve] {msg}", file=sys.stderr, flush=True)  # noqa: E731
    seqs = []
    for ci, (V, W, H, f) in enumerate(SERVE_COMBOS):
        w = synth.workload_human(seed=20 + ci, n_frames=args.seq_frames, n_verts=V, width=W, height=H, focal=f)
        seqs.append((w, [torch.from_numpy(x).to(dev) for x in w.frames]))
        log(f"workload {w.name} ready")
    prm = dict(seqs[0][0].params, active=None)
    streams = []
    for s in range(args.streams):
        rng = np.random.default_rng(5000 + s)
        ci = int(rng.integers(len(SERVE_COMBOS)))
        w = seqs[ci][0]
        th0 = w.theta0 + np.where(w.body.angular, rng.uniform(-0.005, 0.005, len(w.theta0)), 0.0)
        gaps = rng.exponential(1.0 / 30.0, args.frames)
        streams.append(dict(ci=ci, th0=th0, arrive=np.cumsum(gaps)))

    def open_all(sv):
        return [T.track_server_open(sv, seqs[st["ci"]][0].body.model, seqs[st["ci"]][0].body.camera, st["th0"])
                for st in streams]

    def frame_of(s, k):
        return seqs[streams[s]["ci"]][1][_pingpong(k, args.seq_frames)]

    budget = int(args.budget_gb * (1 << 30))
    # (i) configured load: Poisson arrivals at 30 frames/s per stream
    sv = T.track_server_create(prm, budget, args.streams)
    ids = open_all(sv)
    for s in range(len(streams)):  # warm the graphs of the batch shapes with one frame each
        T.track_server_submit(sv, ids[s], frame_of(s, 0), tag=-1)
    while T.track_server_info(sv)["frames_pending"]:
        T.track_server_step(sv)
    T.track_server_poll(sv, 100000)
    log("configured load")
    nxt = [1] * len(streams)
    total = len(streams) * args.frames
    lat, done, steps = [], 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while done < total - len(streams):
        now = time.perf_counter() - t0
        for s, st in enumerate(streams):
            while nxt[s] < args.frames and st["arrive"][nxt[s]] <= now:
                T.track_server_submit(sv, ids[s], frame_of(s, nxt[s]), tag=s * 100000 + nxt[s])
                nxt[s] += 1
        info = T.track_server_info(sv)
        if info["frames_pending"] == 0:
            future = [st["arrive"][nxt[s]] for s, st in enumerate(streams) if nxt[s] < args.frames]
            if future:
                time.sleep(max(0.0, min(future) - (time.perf_counter() - t0)))
            continue
        T.track_server_step(sv)
        steps += 1
        t_now = time.perf_counter() - t0
        for c in T.track_server_poll(sv, 100000):
            s, k = divmod(c["tag"], 100000)
            lat.append(t_now - streams[s]["arrive"][k])
            done += 1
    t_load = time.perf_counter() - t0
    T.track_server_destroy(sv)
    lat_ms = np.array(lat) * 1e3
    log(f"configured load done: {done} frames in {t_load:.2f} s, {steps} steps")

    # (ii) saturation: every stream always has frames waiting
    sv = T.track_server_create(prm, budget, args.streams)
    ids = open_all(sv)
    nsat = args.sat_frames
    for s in range(len(streams)):
        T.track_server_submit(sv, ids[s], frame_of(s, 0), tag=-1)
    while T.track_server_info(sv)["frames_pending"]:
        T.track_server_step(sv)
    T.track_server_poll(sv, 100000)
    for s in range(len(streams)):
        for k in range(1, nsat + 1):
            T.track_server_submit(sv, ids[s], frame_of(s, k), tag=s * 100000 + k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_sat = 0
    while n_sat < len(streams) * nsat:
        n_sat += T.track_server_step(sv)
    torch.cuda.synchronize()
    t_sat = time.perf_counter() - t0
    T.track_server_poll(sv, 1000000)
    chosen = list(range(0, len(streams), max(1, len(streams) // 8)))[:8]
    mix_state = {s: T.track_server_state(sv, ids[s], len(streams[s]["th0"]),
                                         seqs[streams[s]["ci"]][0].body.model["rest_xyz"].shape[0])
                 for s in chosen}
    T.track_server_destroy(sv)
    log(f"saturation: {n_sat} frames in {t_sat:.2f} s")
    mix = {}
    for st in streams:
        name = seqs[st["ci"]][0].name
        mix[name] = mix.get(name, 0) + 1
    if lite:
        return {"streams": len(streams), "mix": mix, "sequence_frames_per_size": args.seq_frames,
                "configured_load": {"offered_fps": 30.0 * len(streams), "achieved_fps": done / t_load,
                                    "p50_ms": float(np.percentile(lat_ms, 50)),
                                    "p99_ms": float(np.percentile(lat_ms, 99)), "frames": done},
                "saturation_fps": n_sat / t_sat, "saturation_frames": n_sat}

    # (iv) eight streams rerun alone must end bit-identical
    same = []
    for s in chosen:
        sv = T.track_server_create(prm, budget, 1)
        sid = T.track_server_open(sv, seqs[streams[s]["ci"]][0].body.model, seqs[streams[s]["ci"]][0].body.camera,
                                  streams[s]["th0"])
        for k in range(0, nsat + 1):
            T.track_server_submit(sv, sid, frame_of(s, k), tag=k)
        while T.track_server_info(sv)["frames_pending"]:
            T.track_server_step(sv)
        th, phi = T.track_server_state(sv, sid, len(streams[s]["th0"]),
                                       seqs[streams[s]["ci"]][0].body.model["rest_xyz"].shape[0])
        T.track_server_destroy(sv)
        same.append(bool(np.array_equal(th, mix_state[s][0]) and np.array_equal(phi, mix_state[s][1])))
    log(f"alone vs mix: {same}")

    # (iii) admission under a 1 GiB budget: streams queue instead of failing
    sv = T.track_server_create(prm, 1 << 30, args.streams)
    ids = open_all(sv)
    info0 = T.track_server_info(sv)
    for s in range(len(streams)):
        for k in range(args.admit_frames):
            T.track_server_submit(sv, ids[s], frame_of(s, k), tag=s * 100000 + k)
    finished, max_res, n_adm, failed = set(), 0, 0, 0
    t0 = time.perf_counter()
    while len(finished) < len(streams):
        T.track_server_step(sv)
        for c in T.track_server_poll(sv, 100000):
            n_adm += 1
            failed += c["status"] != 0
            s, k = divmod(c["tag"], 100000)
            if k == args.admit_frames - 1:
                finished.add(s)
                T.track_server_close(sv, ids[s])
        max_res = max(max_res, T.track_server_info(sv)["resident"])
    t_adm = time.perf_counter() - t0
    T.track_server_destroy(sv)
    log(f"admission: {n_adm} frames, max resident {max_res}")

    out = {
        "metric": "aggregate tracked frames/s + p99 latency (64 streams, 10k-200k-vert bodies, 320x240/640x480)",
        "value": n_sat / t_sat,
        "unit": "frames/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serving-mix", "streams": len(streams), "mix": mix,
                   "frames_per_stream_load": args.frames, "frames_per_stream_saturation": nsat,
                   "arrivals": "Poisson, 30 frames/s per stream", "gn_iters_per_frame": int(prm["n_iters"]),
                   "sequence": f"{args.seq_frames} rendered frames per size, walked forward and back"},
        "configured_load": {"offered_fps": 30.0 * len(streams), "achieved_fps": done / t_load,
                            "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
                            "frames": done, "steps": steps},
        "saturation": {"frames": n_sat, "seconds": t_sat, "fps": n_sat / t_sat},
        "admission_1GiB": {"frames": n_adm, "failed_frames": failed, "max_resident": max_res,
                           "waiting_at_open": info0["waiting"], "resident_at_open": info0["resident"],
                           "seconds": t_adm},
        "alone_vs_mix_bit_identical": {"streams": chosen, "identical": same},
    }
    print(json.dumps(out), flush=True)


def modes(args):
    """Tracking modes and schedules of Section 5.1 on the 30-frame human
    workload against its synthetic ground truth: joint-position accuracy
    against the threshold (AUC over 0-10 cm), reconstruction error of the
    visible surface (Section 5.3), GPU time per frame."""
    import torch

    import synth
    from paper_1711_07999_amd import metrics as M
    from paper_1711_07999_amd import track as T

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    w = synth.workload_human(n_frames=args.seq_frames)
    m, cam = w.body.model, w.body.camera
    frames = [torch.from_numpy(f).to(dev) for f in w.frames]
    links = np.unique(m["link_joint"])
    truth = [synth.joint_matrices(m, w.theta_true[f])[links, :3, 3] for f in range(len(frames))]
    thr = np.linspace(0.0, 0.10, 101)
    n_it = int(w.params["n_iters"])
    out = {"metric": "tracking modes (joint accuracy AUC 0-10 cm, reconstruction error, GPU ms/frame)",
           "config": {"workload": w.name, "frames": len(frames), "joints_scored": int(links.size),
                      "ground_truth": "synthetic: matrix linear-blend posed surface with 5 mm folds"},
           "modes": {}}
    for mode in M.MODES:
        model = M.model_for(mode, m)
        dp, ds = M.mode_schedule(mode, 0, n_it)
        prm = dict(w.params, n_iters=len(dp), do_pose=dp, do_shape=ds)
        trk = T.Tracker(model, cam, prm, w.theta0)
        errs, rec, ms = [], [], []
        try:
            for f, depth in enumerate(frames):
                dp, ds = M.mode_schedule(mode, f, n_it)
                if not (np.array_equal(dp, prm["do_pose"]) and np.array_equal(ds, prm["do_shape"])):
                    prm = dict(prm, n_iters=len(dp), do_pose=dp, do_shape=ds)
                    trk.set_params(prm)
                rc = trk.frame(depth)
                if rc != 0:
                    raise RuntimeError(f"{mode} frame {f}: {T.track_last_error()}")
                _, _, v, st = trk.state()
                ms.append(st["ms_total"])
                errs.append(M.joint_errors(trk.joint_positions()[links], truth[f]))
                rec.append(M.reconstruction_errors(v, M.vertex_normals(v, m["faces"]), w.frames[f], cam))
        finally:
            trk.close()
        e = np.stack(errs)
        r = np.concatenate(rec)
        curve = M.accuracy_curve(e, thr)
        out["modes"][mode] = {
            "iterations": {"pose": int(np.sum(M.mode_schedule(mode, 1, n_it)[0])),
                           "offsets_first_frame": int(np.sum(M.mode_schedule(mode, 0, n_it)[1])),
                           "offsets_later_frames": int(np.sum(M.mode_schedule(mode, 1, n_it)[1]))},
            "joint_error_mean_m": float(e.mean()), "joint_error_max_m": float(e.max()),
            "within_2cm": float(M.accuracy_curve(e, [0.02])[0]), "within_5cm": float(M.accuracy_curve(e, [0.05])[0]),
            "auc_0_10cm": M.curve_auc(thr, curve),
            "reconstruction_mm": {"mean": float(r.mean() * 1e3), "median": float(np.median(r) * 1e3),
                                  "p90": float(np.percentile(r, 90) * 1e3), "vertices": int(r.size)},
            "gpu_ms_per_frame": float(np.mean(ms[1:])),
        }
        print(f"[modes] {mode}: {json.dumps(out['modes'][mode])}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def copy_calibration(args):
    """A plain device copy of known size, for scaling hardware byte counters
    (FETCH_SIZE / WRITE_SIZE) to bytes: 64 MiB read and 64 MiB written per
    launch, 10 launches."""
    import torch

    n = 16 << 20
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(10):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_kernel_bytes_read": 4 * n, "copy_kernel_bytes_written": 4 * n, "launches": 10}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--gram", choices=["fp32", "bf16x3"], default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=200,
                    help="back-to-back launches of the dominant kernel (an extra figure of its roofline)")
    ap.add_argument("--inframe-frames", type=int, default=30,
                    help="frames tracked with the dominant kernel's launches timed (its roofline)")
    ap.add_argument("--batch-frames", type=int, default=20,
                    help="frames per stream of the batched copies at saturation")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other operand form and the batched copies")
    ap.add_argument("--serve", action="store_true", help="serving mix instead of the single-stream step")
    ap.add_argument("--modes", action="store_true",
                    help="tracking modes and schedules against the synthetic ground truth")
    ap.add_argument("--highres", action="store_true",
                    help="only the high-resolution configuration (200,000 vertices, 512x424)")
    ap.add_argument("--batched", type=int, default=0,
                    help="only B copies of the workload batched through one server")
    ap.add_argument("--streams", type=int, default=64)
    ap.add_argument("--frames", type=int, default=300, help="frames per stream at the configured load")
    ap.add_argument("--sat-frames", type=int, default=30, help="frames per stream at saturation")
    ap.add_argument("--admit-frames", type=int, default=10)
    ap.add_argument("--seq-frames", type=int, default=30)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only a plain copy of known size (for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): tracking streams are independent "
              "and would be spread over GPUs by a front end, with no communication between them",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args)
    elif args.serve:
        serve(args)
    elif args.modes:
        modes(args)
    elif args.batched:
        batched_only(args)
    elif args.highres:
        highres_only(args)
    else:
        single_stream(args)


if __name__ == "__main__":
    main()
