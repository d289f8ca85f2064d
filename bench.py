"""Benchmark: pixel-frames/s of the whole per-frame path on one MI355X.

Workload: 640x512 FP32 frames, 16x16x8 analysis window, 17x17 candidate
velocities on a 0.5 px/frame grid over [-4, 4]; smooth non-uniform clutter
flow with an occluding band, 20 point targets and sigma = 1 noise (seeded
synthetic frames, generated before timing and resident in HBM).

One step = one frame pushed through the whole path (row sliding DFT with the
frame's copy into the delay ring, per-pixel kernel).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, GB/s

# HBM bytes per launch of the per-pixel kernel, measured with rocprofv3 PMC
# counters (FETCH_SIZE and WRITE_SIZE, each scaled by what the same counter
# reads for a plain copy of known size).  The figure only stands for the
# kernel source it was taken on: a change to any of these files voids it.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_pixel16_{workload}.txt")
# the same for the temporal-ring and direct-spectrum forms
TRAFFIC_FILE_FORM = os.path.join(ROOT, "profiles", "traffic_pixel16_{form}_{workload}.txt")
# seeded 640x512 scenes for the learned leg's accuracy figures: the first three
# of the network's evaluation seeds (none of them used in its training)
LEARNED_EVAL_SEEDS = (2000, 2001, 2002)

# pixel-kernel launches timed with HIP events inside the timed region: one in
# this many (the events' own cost stays out of the step time)
TIMING_EVERY = 8

KERNEL_SOURCES = ["paper_1408_3526_amd/csrc/rmdf_pixel16.h", "paper_1408_3526_amd/csrc/rmdf_pixel16.hip",
                  "paper_1408_3526_amd/csrc/rmdf_kernels.h", "paper_1408_3526_amd/csrc/rmdf_wave.h"]

WORKLOADS = {
    "640x512": dict(H=512, W=640, M=(16, 16, 8), grid=(-4.0, 4.0, 0.5), frames=200, seed=1, targets=20),
    "1280x1024": dict(H=1024, W=1280, M=(16, 16, 8), grid=(-4.0, 4.0, 0.5), frames=100, seed=2, targets=50),
    "64x64": dict(H=64, W=64, M=(8, 8, 4), grid=(-4.0, 4.0, 1.0), frames=32, seed=0, targets=3),
    # the paper's own configuration (Sec. 3): 64x64 frames, K = (4, 4, 2) i.e. a 9x9x5 window,
    # B = 3, m' = K, 17x17 grid at 0.25 px/frame, on its simulated scene (Sec. 4)
    "paper64": dict(H=64, W=64, M=(9, 9, 5), grid=(-2.0, 2.0, 0.25), frames=64, seed=7, targets=1, scene="paper"),
}

# The paper's fastest full-pipeline rate on its own configuration: 43.7 frames/s of
# 64x64 pixels (row-parallel C++ on the 8 threads of an i7-4810MQ, Sec. 5).  Only
# the paper64 workload is the same workload, so only its line carries vs_baseline.
PAPER_RATE = {"paper64": {"value": 43.7 * 64 * 64, "unit": "pixel-frames/s",
                          "what": "paper Sec. 5: C++ parallel_for over rows, 8 threads, Intel i7-4810MQ"}}


def algorithmic_bytes_per_pixel_frame(M, nv):
    """Bytes the method itself must move per pixel and frame: observer state
    read + write (Mx*My*Mz reals of a Hermitian spectrum, FP32), smoothed
    autocorrelation read + write (nv FP32), frame in, delayed frame in,
    output out, velocity (2 FP32) and its grid index (int32) out."""
    Mx, My, Mz = M
    return 2 * 4 * Mx * My * Mz + 2 * 4 * nv + 4 + 4 + 4 + 8 + 4


def kernel_source_digest():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kname, workload, form=None):
    """HBM bytes per launch from the committed counter summary, or None when
    it is absent or was taken on another kernel, workload or source."""
    path = TRAFFIC_FILE.format(workload=workload) if form is None else TRAFFIC_FILE_FORM.format(form=form,
                                                                                                workload=workload)
    try:
        with open(path) as f:
            kv = dict(line.split("=", 1) for line in (ln.strip() for ln in f) if "=" in line and not line.startswith("#"))
    except OSError:
        return None
    if (kv.get("kernel") != kname or kv.get("workload") != workload
            or kv.get("source_sha256") != kernel_source_digest()):
        return None
    return float(kv["hbm_bytes_per_launch"])


def copy_calibration(nbytes=1 << 30, reps=10):
    """A plain device copy of known size, for scaling the PMC byte counters:
    each launch reads and writes nbytes."""
    import torch
    torch.cuda.set_device(0)
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps({"copy_bytes_read_per_launch": nbytes, "copy_bytes_written_per_launch": nbytes,
                      "launches": 2 * reps, "ms_per_copy": ms,
                      "read_plus_write_GBps": 2 * nbytes / (ms / 1e3) / 1e9}), flush=True)


def hbm_ceiling(nbytes=1 << 31, reps=5):
    """Practical HBM ceilings on this GPU from the library's streaming probe
    (rmdf_hbm_probe): best GB/s over grid sizes and cached / non-temporal
    access, for read, write and copy (read + write bytes).  The per-pixel
    kernel reads and writes about equally (the observer state), so its
    practical ceiling is the copy rate."""
    import torch

    from paper_1408_3526_amd import binding
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.empty(1 << 16, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    best = {}
    for kind, name, moved in ((0, "read", nbytes), (1, "write", nbytes), (2, "copy", 2 * nbytes)):
        for nt in (False, True):
            for blocks in (1024, 2048, 4096, 8192, 16384):
                run = lambda: binding.hbm_probe(kind, src if kind != 1 else None,  # noqa: E731
                                                sink if kind == 0 else dst, nbytes, blocks, nt)
                run()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(reps):
                    run()
                e1.record(stream)
                torch.cuda.synchronize()
                gbs = moved * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
                if gbs > best.get(name, {}).get("GBps", 0.0):
                    best[name] = {"GBps": gbs, "workgroups": blocks, "nontemporal": nt}
    del src, dst, sink
    torch.cuda.empty_cache()
    return best


# Batched streams: (count, H, W, window, velocity grid (lo, hi, step), targets)
BATCH24 = [(8, 256, 320, (8, 8, 4), (-4.0, 4.0, 1.0), 5),
           (8, 512, 640, (16, 16, 8), (-4.0, 4.0, 0.5), 20),
           (8, 1024, 1280, (16, 16, 8), (-4.0, 4.0, 0.5), 50)]


def _batch_stream_frames(job):
    seed, H, W, nfr, nt = job
    from paper_1408_3526_amd import scenes
    return scenes.flow_scene(seed, H=H, W=W, T=nfr, n_targets=nt, varying_noise=(H >= 1024)).frames


def batch_inputs(nfr):
    """Seeded frames of the 24 streams (own seed, velocity field, band and
    targets per stream), generated in worker processes; call before the GPU
    is touched (the workers are forked)."""
    import concurrent.futures as cf

    from paper_1408_3526_amd import scenes
    jobs, specs = [], []
    seed = 300
    for count, H, W, M, gr, nt in BATCH24:
        g = scenes.grid(*gr)
        for _ in range(count):
            seed += 1
            jobs.append((seed, H, W, nfr, nt))
            specs.append(dict(H=H, W=W, M=M, gx=g, gy=g))
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        frames = list(ex.map(_batch_stream_frames, jobs))
    print("generated 24 streams x %d frames (%.0f s)" % (nfr, time.perf_counter() - t0), file=sys.stderr, flush=True)
    return frames, specs


def batch_leg(frames_np, specs, steps, warmup, tune_iters=5):
    """24 streams of three sizes advanced together, one hipGraph launch per
    step (frames copied into the streams' input slots inside the timed
    region); tiles and schedule chosen by the autotuner first.  Aggregate
    pixel-frames/s, p50/p99 step latency, algorithmic bytes and the share of
    each tile family in them."""
    import torch

    from paper_1408_3526_amd import binding
    torch.cuda.set_device(0)
    frames = [torch.from_numpy(f).cuda() for f in frames_np]
    nfr = frames[0].shape[0]
    b = binding.Batch(specs)
    for i in range(warmup):
        b.push([f[i % nfr] for f in frames])
    report = b.autotune(iters=tune_iters)
    print(report, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    b.set_timing(True)
    w0 = time.perf_counter()
    for i in range(steps):
        b.push([f[(warmup + i) % nfr] for f in frames])
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    lat = b.latency()
    b.close()
    del frames
    torch.cuda.empty_cache()
    px = sum(sp["H"] * sp["W"] for sp in specs)
    fam = {}
    for sp in specs:
        key = "%dx%d @%dx%dx%d" % (sp["W"], sp["H"], *sp["M"])
        fam[key] = fam.get(key, 0) + sp["H"] * sp["W"] * algorithmic_bytes_per_pixel_frame(sp["M"], len(sp["gx"]) ** 2)
    byt = sum(fam.values())
    return {"value": steps * px / wall, "unit": "pixel-frames/s", "steps": steps, "warmup": warmup,
            "ms_per_step": 1e3 * wall / steps,
            "config": {"workload": "24 streams: 8 x 320x256 (8x8x4, 9x9 grid), 8 x 640x512 and 8 x 1280x1024 "
                                   "(16x16x8, 17x17 grid at 0.5 px/frame)", "frames_distinct": nfr,
                       "pixels_per_step": px},
            "latency_ms": {"p50": lat["p50_ms"], "p99": lat["p99_ms"], "mean": lat["mean_ms"]},
            "algorithmic_GBps": byt * steps / wall / 1e9,
            "hbm_frac": byt * steps / wall / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes_share": {k: v / byt for k, v in fam.items()},
            "autotune": report.strip().splitlines()}


def cpu_baseline_batch(frames_np, specs, strip_rows=32, n_frames=4):
    """The FP64 oracle on the batched workload: one full-width strip
    (strip_rows rows plus the My - 1 rows above) of the first stream of each
    size class over its first n_frames frames, all host cores; the aggregate
    rate is the step's pixel count over the time the oracle would take for
    every stream of the step at its class's rate.  A few seconds of CPU work."""
    import numpy as np

    import oracle
    oracle.lib()
    cores = oracle.threads()
    per_class, seen = [], set()
    for f, sp in zip(frames_np, specs):
        key = (sp["H"], sp["W"], sp["M"])
        if key in seen:
            continue
        seen.add(key)
        H, W, M = sp["H"], sp["W"], sp["M"]
        y0 = H // 2 - strip_rows // 2
        ya = max(0, y0 - (M[1] - 1))
        sub = np.ascontiguousarray(f[:n_frames, ya:y0 + strip_rows, :])
        cfg = oracle.Cfg(H=sub.shape[1], W=W, Mx=M[0], My=M[1], Mz=M[2], gx=sp["gx"], gy=sp["gy"])
        t0 = time.perf_counter()
        oracle.run(cfg, sub)
        dt = time.perf_counter() - t0
        per_class.append({"stream": "%dx%d @%dx%dx%d" % (W, H, *M), "rate": n_frames * strip_rows * W / dt,
                          "seconds": dt})
    rate = {c["stream"]: c["rate"] for c in per_class}
    step_s = sum(sp["H"] * sp["W"] / rate["%dx%d @%dx%dx%d" % (sp["W"], sp["H"], *sp["M"])] for sp in specs)
    px = sum(sp["H"] * sp["W"] for sp in specs)
    return {"value": px / step_s, "unit": "pixel-frames/s", "cores": cores, "kind": "oracle",
            "sample": "one full-width %d-row strip (+My-1 rows above, centred) of one stream per size class, "
                      "first %d frames; aggregate over the step's %d streams" % (strip_rows, n_frames, len(specs)),
            "per_class": per_class}


def batch_bench(args):
    """The batched-streams workload on its own (--batch24): one JSON line."""
    frames_np, specs = batch_inputs(args.frames or 12)
    r = batch_leg(frames_np, specs, args.steps, args.warmup)
    res = {"metric": "batched streams: aggregate pixel-frames/s, per-step latency", "mode": "batch24",
           "n_gpus": 1, "higher_is_better": True, "dtype": "f32", "data": "synthetic"}
    res.update(r)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_batch(frames_np, specs)
    print(json.dumps(res), flush=True)


def make_scene(wl):
    from paper_1408_3526_amd import scenes
    H, W = wl["H"], wl["W"]
    if wl.get("scene") == "paper":
        return scenes.paper_scene(wl["seed"], H=H, W=W, T=wl["frames"])
    if wl["M"] == (8, 8, 4):
        return scenes.translate_scene(wl["seed"], H=H, W=W, T=wl["frames"], v=(1, -2), n_targets=wl["targets"])
    return scenes.flow_scene(wl["seed"], H=H, W=W, T=wl["frames"], n_targets=wl["targets"],
                             varying_noise=(H >= 1024))


def learned_leg(dev, sc, M, g, steps, warmup):
    """Learned velocity mode (trained weights shipped with the package):
    pixel-frames/s on the benchmark's frames; and, for both modes, the PEF
    residual RMS and the velocity RMSE against the scene's true field (over
    the last 10 of 40 frames, anchors away from the targets and the frame
    border) and the learned mode's fallback rate, averaged over three seeded
    640x512 scenes that the network was not trained on (the first three of its
    evaluation seeds).  None when no weights are present."""
    import numpy as np
    import torch

    from paper_1408_3526_amd import binding, learned
    if M != (16, 16, 8) or not os.path.exists(learned.DEFAULT_WEIGHTS):
        return None
    w = np.load(learned.DEFAULT_WEIGHTS)
    T, H, W = dev.shape
    acc = learned.evaluate(w, LEARNED_EVAL_SEEDS, H=H, W=W, T=40)
    resid = {"plain": acc["search"]["residual_rms"], "learned": acc["learned"]["residual_rms"]}
    rmse = {"plain": acc["search"]["velocity_rmse"], "learned": acc["learned"]["velocity_rmse"]}
    fallback = {"learned": acc["learned"]["fallback_rate"]}

    f = binding.Filter(H, W, *M, g, g, velocity_mode=binding.VEL_LEARNED, conf_threshold=0.9)
    f.set_weights(w)
    for i in range(warmup):
        f.push_frame(dev[i % T])
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(steps):
        f.push_frame(dev[(warmup + i) % T])
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    # kernel split (HIP events around each launch, in a separate loop so the
    # events stay out of the timed one): first pass (spectrum, search,
    # features), network (count reset + the one network kernel), finish
    f.set_timing(kernels=[0, 3, 4])
    for k in (0, 3, 4):
        f.kernel_time(k)
    n_split = min(steps, 50)
    for i in range(n_split):
        f.push_frame(dev[i % T])
    split = {name: f.kernel_time(k)[0] / n_split for name, k in (("first_pass", 0), ("network", 3), ("finish", 4))}
    f.close()
    # the network reads 1152 BF16 features and writes 3 FP32 outputs per anchor
    net_bytes = H * W * (1152 * 2 + 3 * 4)
    return {"value": steps * H * W / (ms / 1e3), "unit": "pixel-frames/s", "ms_per_step": ms / steps,
            "kernel_ms": split, "network_GBps": net_bytes / (split["network"] / 1e3) / 1e9,
            "residual_rms": resid["learned"], "plain_residual_rms": resid["plain"],
            "residual_ratio": resid["learned"] / resid["plain"],
            "equal_residual_within_5pct": bool(resid["learned"] <= 1.05 * resid["plain"]),
            "velocity_rmse": rmse["learned"], "plain_velocity_rmse": rmse["plain"],
            "fallback_rate": fallback["learned"], "conf_threshold": 0.9,
            "accuracy_seeds": list(LEARNED_EVAL_SEEDS)}


def refined_leg(dev, sc, M, g, steps, warmup):
    """Velocity mode 3 (peak refined between grid points, coefficients at the
    refined velocity) on the same frames: pixel-frames/s and pixel-kernel time,
    PEF residual RMS and velocity RMSE against the true field for both modes
    over the last 10 of the first 40 frames (away from targets and border)."""
    import numpy as np
    import torch

    from paper_1408_3526_amd import binding, learned
    T, H, W = dev.shape
    dx, dy, dt = M[0] // 2, M[1] // 2, M[2] // 2
    tv = sc.velocity[np.clip(np.arange(H) - dy, 0, H - 1)][:, np.clip(np.arange(W) - dx, 0, W - 1)]
    stats = {}
    n_eval = min(40, T)
    for mode in (binding.VEL_SEARCH, binding.VEL_REFINED):
        f = binding.Filter(H, W, *M, g, g, velocity_mode=mode)
        resid, rmse = [], []
        for t in range(n_eval):
            f.push_frame(dev[t])
            if t >= n_eval - 10:
                out = f.output().cpu().numpy()
                vxy, _ = f.velocity()
                vxy = vxy.cpu().numpy()
                m = learned.valid_mask(H, W, sc.targets, t - dt, dx=dx, dy=dy)
                resid.append(float(np.sqrt(np.mean(out[m].astype(np.float64) ** 2))))
                rmse.append(float(np.sqrt(np.mean(np.sum((vxy[m] - tv[m]) ** 2, -1)))))
        f.close()
        stats[mode] = (float(np.mean(resid)), float(np.mean(rmse)))
    f = binding.Filter(H, W, *M, g, g, velocity_mode=binding.VEL_REFINED)
    for i in range(warmup):
        f.push_frame(dev[i % T])
    torch.cuda.synchronize()
    f.set_timing(kernels=[0])
    f.kernel_time(0)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(steps):
        f.push_frame(dev[(warmup + i) % T])
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    k = f.kernel_time(0)
    f.set_timing(False)
    f.close()
    ps, pr = stats[binding.VEL_SEARCH], stats[binding.VEL_REFINED]
    return {"value": steps * H * W / (ms / 1e3), "unit": "pixel-frames/s", "ms_per_step": ms / steps,
            "kernel_ms": k[0] / max(k[1], 1),
            "residual_rms": pr[0], "plain_residual_rms": ps[0], "residual_ratio": pr[0] / ps[0],
            "velocity_rmse": pr[1], "plain_velocity_rmse": ps[1]}


def ring_bytes_per_pixel_frame(M, nv):
    """Bytes per pixel and frame with the temporal ring: Mz - 1 stored 2-D
    spectra read and one written (Mx*My reals each, FP32), the smoothed
    autocorrelation read + write, and the same 24 bytes of frame, delayed
    frame, output, velocity and index."""
    Mx, My, Mz = M
    return 4 * Mx * My * Mz + 2 * 4 * nv + 4 + 4 + 4 + 8 + 4


def temporal_form_leg(dev, M, g, steps, warmup, temporal, workload=None):
    """The temporal ring (the temporal DFT taken directly over the last Mz 2-D
    spectra instead of the observer) or the direct form (no recursion on any
    axis: direct row and column DFT sums as well) on the same frames:
    pixel-frames/s, the pixel and row kernels' times, and the pixel kernel's
    rate against its own algorithmic bytes."""
    import torch

    from paper_1408_3526_amd import binding
    if tuple(M) != (16, 16, 8):
        return None
    T, H, W = dev.shape
    f = binding.Filter(H, W, *M, g, g, temporal=temporal)
    for i in range(warmup):
        f.push_frame(dev[i % T])
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(steps):
        f.push_frame(dev[(warmup + i) % T])
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    # kernel times from a separate pass (each timed launch adds event records)
    f.set_timing(kernels=[0, 1])
    f.kernel_time(0)
    f.kernel_time(1)
    for i in range(min(steps, 100)):
        f.push_frame(dev[(warmup + steps + i) % T])
    k = f.kernel_time(0)
    kr = f.kernel_time(1)
    f.set_timing(False)
    f.close()
    kms = k[0] / max(k[1], 1)
    bpp = ring_bytes_per_pixel_frame(M, len(g) ** 2)
    ach = bpp * H * W / (kms / 1e3) / 1e9
    form = "ring" if temporal == binding.TEMPORAL_RING else "direct"
    kname = "k_pixel16<%d>" % (4 if form == "ring" else 5)
    return {"value": steps * H * W / (ms / 1e3), "unit": "pixel-frames/s", "ms_per_step": ms / steps,
            "kernel_ms": kms, "row_kernel_ms": kr[0] / max(kr[1], 1),
            "algorithmic_bytes_per_pixel_frame": bpp, "achieved_GBps": ach, "frac": ach / HBM_PEAK_GBS,
            "traffic": measured_traffic(kname, workload, form) if workload else None}


def pair_bytes_per_pixel_frame(M, nv):
    """Bytes per pixel and frame when frames go through the per-pixel kernel
    two at a time: the observer state and the smoothed autocorrelation are
    read and written once per pair; per frame the same 24 bytes of frame,
    delayed frame, output, velocity and index (the pair's first frame writes
    its output only, so 12 of them are not moved for it)."""
    Mx, My, Mz = M
    return (2 * 4 * Mx * My * Mz + 2 * 4 * nv) / 2 + (24 + 12) / 2


def pairs_leg(dev, M, g, steps, warmup, workload=None):
    """Frame pairs (rmdf_push_frames, two frames per pass of the per-pixel
    kernel over the state) on the same frames: pixel-frames/s, the pair
    kernel's time per pair, and its rate against its own algorithmic bytes."""
    import torch

    from paper_1408_3526_amd import binding
    if tuple(M) != (16, 16, 8):
        return None
    T, H, W = dev.shape
    f = binding.Filter(H, W, *M, g, g)
    pairs = max(1, steps // 2)
    for i in range(max(1, warmup // 2)):
        f.push_frames([dev[(2 * i) % T], dev[(2 * i + 1) % T]])
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(pairs):
        f.push_frames([dev[(2 * i) % T], dev[(2 * i + 1) % T]])
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    f.set_timing(kernels=[0])
    f.kernel_time(0)
    for i in range(min(pairs, 50)):
        f.push_frames([dev[(2 * i) % T], dev[(2 * i + 1) % T]])
    k = f.kernel_time(0)
    f.set_timing(False)
    f.close()
    kms = k[0] / max(k[1], 1)
    bpp = pair_bytes_per_pixel_frame(M, len(g) ** 2)
    ach = bpp * 2 * H * W / (kms / 1e3) / 1e9
    return {"value": 2 * pairs * H * W / (ms / 1e3), "unit": "pixel-frames/s", "ms_per_frame": ms / (2 * pairs),
            "pair_kernel_ms": kms, "algorithmic_bytes_per_pixel_frame": bpp, "achieved_GBps": ach,
            "frac": ach / HBM_PEAK_GBS,
            "traffic": measured_traffic("k_pixel16<6>", workload, "pairs") if workload else None}


def detection_leg(dev, sc, M, g, guard=2, train=4, ks=(3.0, 3.5, 4.0, 5.0)):
    """Detection stage after the filter: two-sided CA-CFAR (rmdf_cfar) on the
    prediction error of the last 10 of the first 40 frames, and, for
    comparison, on the raw input frames, at several thresholds k (points of
    the Pd/Pfa curve).  A target counts as detected when a detection lies
    within 2 px of it; detections farther than 4 px from every target count as
    false alarms (15 px away from the frame border).  Pd per target SNR bin,
    false alarms per pixel, and the CFAR kernel's time per frame."""
    import numpy as np
    import torch

    from paper_1408_3526_amd import binding
    if sc.target_snr is None:
        return None
    T, H, W = dev.shape
    dx, dy, dt = M[0] // 2, M[1] // 2, M[2] // 2
    n_eval = min(40, T)
    f = binding.Filter(H, W, *M, g, g)
    ys, xs = np.mgrid[0:H, 0:W]
    bins = [(2, 4), (4, 6), (6, 8.01)]
    snr = sc.target_snr
    cnt = {(n, k): [np.zeros(len(bins)), np.zeros(len(bins)), 0, 0] for n in ("pef", "raw") for k in ks}
    for t in range(n_eval):
        f.push_frame(dev[t])
        if t < n_eval - 10:
            continue
        t_out = t - dt
        for name, img, ox, oy in (("pef", f.output(), dx, dy), ("raw", dev[t_out].contiguous(), 0, 0)):
            near = np.zeros((H, W), bool)
            disc = []
            for i in range(sc.targets.shape[0]):
                d2 = (xs - sc.targets[i, t_out, 0] - ox) ** 2 + (ys - sc.targets[i, t_out, 1] - oy) ** 2
                near |= d2 <= 16.0
                disc.append(d2 <= 4.0)
            valid = ~near & (xs >= 15) & (ys >= 15) & (xs < W - 15) & (ys < H - 15)
            for k in ks:
                det = binding.cfar(img, guard, train, k).cpu().numpy().astype(bool)
                c = cnt[(name, k)]
                for i in range(len(disc)):
                    j = next(j for j, (lo, hi) in enumerate(bins) if lo <= snr[i] < hi)
                    c[0][j] += bool(det[disc[i]].any())
                    c[1][j] += 1
                c[2] += int(det[valid].sum())
                c[3] += int(valid.sum())
    f.close()
    out = dev[n_eval - 1].contiguous()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(5):
        binding.cfar(out, guard, train, ks[0])
    e0.record(stream)
    for _ in range(50):
        binding.cfar(out, guard, train, ks[0])
    e1.record(stream)
    torch.cuda.synchronize()
    res = {"guard": guard, "train": train, "cfar_ms": e0.elapsed_time(e1) / 50,
           "targets_by_snr": {"%g-%g" % (lo, min(hi, 8)): int(n) for (lo, hi), n in zip(bins, cnt[("pef", ks[0])][1])}}
    for name in ("pef", "raw"):
        res[name] = [{"k": k, "pfa": cnt[(name, k)][2] / max(cnt[(name, k)][3], 1),
                      "pd_by_snr": {"%g-%g" % (lo, min(hi, 8)): float(h / n) if n else None
                                    for (lo, hi), h, n in zip(bins, cnt[(name, k)][0], cnt[(name, k)][1])}}
                     for k in ks]
    return res


def cpu_baseline(frames, wl, g, strip_rows=64, n_frames=6, runs=3):
    """The FP64 oracle, as it is, timed on the host's cores over full-width
    strips of the workload's frames: each run takes strip_rows rows plus the
    My - 1 rows above them (the rows the windows of the strip's first rows
    reach into) over the first n_frames frames, and counts only the strip's
    own pixel-frames; the median over `runs` different strips; all host
    cores.  Plus a one-thread sample.  About 20 s of CPU work for the
    640x512 workload on 16 cores."""
    import numpy as np

    import oracle
    T, H, W = frames.shape
    My = wl["M"][1]
    oracle.lib()
    cores = oracle.threads()
    whole = H <= strip_rows           # small frames: the whole workload, every frame
    if whole:
        strip_rows, n_frames = H, T
        starts = [0] * runs
    else:
        starts = [min(H - strip_rows, max(0, (k + 1) * H // (runs + 1) - strip_rows // 2)) for k in range(runs)]
    rates = []
    for y0 in starts:
        ya = max(0, y0 - (My - 1))
        sub = np.ascontiguousarray(frames[:n_frames, ya:y0 + strip_rows, :])
        cfg = oracle.Cfg(H=sub.shape[1], W=W, Mx=wl["M"][0], My=My, Mz=wl["M"][2], gx=g, gy=g)
        t0 = time.perf_counter()
        oracle.run(cfg, sub)
        rates.append(n_frames * strip_rows * W / (time.perf_counter() - t0))
    value = float(np.median(rates))
    # one thread, on a smaller sample of the same frames (a 48x64 crop, 4 frames)
    one = np.ascontiguousarray(frames[:4, :48, :64])
    cfg1 = oracle.Cfg(H=one.shape[1], W=one.shape[2], Mx=wl["M"][0], My=My, Mz=wl["M"][2], gx=g, gy=g)
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.run(cfg1, one)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    n1 = one.shape[0] * one.shape[1] * one.shape[2]
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": value, "unit": "pixel-frames/s", "cores": cores, "kind": "oracle",
            "host": {"cpu": model, "usable_cpus": len(os.sched_getaffinity(0))},
            "sample": ("median of %d runs over the whole workload (%d frames of %dx%d); rates %s pixel-frames/s"
                       % (runs, T, W, H, [round(r) for r in rates])) if whole else
                      ("median of %d runs, each a full-width %d-row strip (+%d rows above, rows %s) of the "
                       "workload's frames over its first %d frames; rates %s pixel-frames/s"
                       % (runs, strip_rows, My - 1, starts, n_frames, [round(r) for r in rates])),
            "one_thread": {"value": n1 / dt1, "cores": 1,
                           "sample": "64x48 crop, 4 frames (%d pixel-frames, %.1f s)" % (n1, dt1)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=24)
    ap.add_argument("--workload", default="640x512", choices=sorted(WORKLOADS))
    ap.add_argument("--frames", type=int, default=0, help="distinct synthetic frames (0: workload default)")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--kernel-variant", type=int, default=0, help="0 auto, 1 generic, 2 wave-per-anchor")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-velocity leg")
    ap.add_argument("--no-refined", action="store_true", help="skip the refined-velocity leg")
    ap.add_argument("--no-detection", action="store_true", help="skip the CFAR detection leg")
    ap.add_argument("--no-ring", action="store_true",
                    help="skip the temporal-ring and direct-spectrum variant legs")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-streams leg")
    ap.add_argument("--no-pairs", action="store_true", help="skip the frame-pairs leg")
    ap.add_argument("--batch24", action="store_true",
                    help="batched-streams benchmark (24 streams of three sizes) instead of the single stream")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (the reference kernel for the PMC byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the per-pixel state would shard by horizontal strips of rows, each with a halo of My - 1 rows)",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.batch24:
        batch_bench(args)
        return

    import numpy as np
    import torch

    from paper_1408_3526_amd import binding, scenes

    # the batched-streams leg's frames, generated by forked workers before the
    # GPU is touched
    batch_in = None if (args.no_batch or args.workload != "640x512") else batch_inputs(4)
    wl = dict(WORKLOADS[args.workload])
    if args.frames:
        wl["frames"] = args.frames
    H, W, M = wl["H"], wl["W"], wl["M"]
    g = scenes.grid(*wl["grid"])
    nv = len(g) ** 2
    t0 = time.perf_counter()
    sc = make_scene(wl)
    frames = sc.frames
    print("generated %d frames in %.1f s" % (frames.shape[0], time.perf_counter() - t0), file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    dev = torch.from_numpy(frames).cuda()
    T = dev.shape[0]
    f = binding.Filter(H, W, *M, g, g, tile_rows=args.tile_rows, kernel_variant=args.kernel_variant)
    stream = torch.cuda.current_stream()

    for i in range(args.warmup):
        f.push_frame(dev[i % T])
    torch.cuda.synchronize()
    # timed region: the dominant (pixel) kernel carries HIP events, for the
    # roofline, on every TIMING_EVERY-th step only: each timed launch adds two
    # event records to the stream, which on small, latency-bound frames would
    # otherwise show up in the step time
    f.kernel_time(0)   # reset counters
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for i in range(args.steps):
        timed = (i % TIMING_EVERY == 0)
        if timed:
            f.set_timing(kernels=[0])
        f.push_frame(dev[(args.warmup + i) % T])
        if timed:
            f.set_timing(False)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    kms = {0: f.kernel_time(0)}
    # the row kernel's time (it also stores the frame into the delay ring)
    # from a short pass after the timed one
    f.set_timing(kernels=[1])
    f.kernel_time(1)
    for i in range(min(args.steps, 100)):
        f.push_frame(dev[(args.warmup + args.steps + i) % T])
    kms[1] = f.kernel_time(1)
    f.set_timing(False)
    out = f.output()
    assert torch.isfinite(out).all()
    kname = f.kernel_name()
    tile_rows = f.tile_rows()
    f.close()

    ceiling = hbm_ceiling()
    px_frames = args.steps * H * W
    value = px_frames / (ms / 1e3)
    bpp = algorithmic_bytes_per_pixel_frame(M, nv)
    pix_ms = kms[0][0] / max(kms[0][1], 1)
    achieved = bpp * H * W / (pix_ms / 1e3) / 1e9
    res = {
        "metric": "pixel-frames/s @640x512, 16x16x8 window; % HBM peak; learned vs plain velocity",
        "value": value,
        "unit": "pixel-frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": (value / PAPER_RATE[args.workload]["value"]) if args.workload in PAPER_RATE else None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%dx%d frames, %dx%dx%d window, %dx%d velocity grid (%.2g px/frame), "
                               "plain autocorrelation search" % (W, H, M[0], M[1], M[2], len(g), len(g), g[1] - g[0])
                               + (", the paper's configuration on its simulated scene" if wl.get("scene") == "paper" else ""),
                   "frames_distinct": int(T), "tile_rows": tile_rows},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(kname, args.workload),
                     "kernel": kname, "kernel_ms": pix_ms,
                     "algorithmic_bytes_per_pixel_frame": bpp,
                     "practical_peak": ceiling["copy"]["GBps"],
                     "frac_practical": achieved / ceiling["copy"]["GBps"],
                     "practical_peak_probe": ceiling},
        "kernel_ms": {"pixel": pix_ms, "row_and_ingest": kms[1][0] / max(kms[1][1], 1)},
        "wall_s": wall,
    }
    if args.workload in PAPER_RATE:
        res["baseline"] = PAPER_RATE[args.workload]
        res["frames_per_s"] = args.steps / (ms / 1e3)
    lr = None if (args.no_learned or tuple(M) != (16, 16, 8)) else learned_leg(dev, sc, M, g, min(args.steps, 200), args.warmup)
    if lr is not None:
        lr["vs_plain"] = lr["value"] / value
        res["learned"] = lr
    if not args.no_refined:
        rf = refined_leg(dev, sc, M, g, min(args.steps, 200), args.warmup)
        rf["vs_plain"] = rf["value"] / value
        res["refined"] = rf
    if not args.no_ring:
        rg = temporal_form_leg(dev, M, g, args.steps, args.warmup, binding.TEMPORAL_RING, args.workload)
        if rg is not None:
            rg["vs_plain"] = rg["value"] / value
            res["temporal_ring"] = rg
        dr = temporal_form_leg(dev, M, g, args.steps, args.warmup, binding.TEMPORAL_DIRECT, args.workload)
        if dr is not None:
            dr["vs_plain"] = dr["value"] / value
            res["direct_spectrum"] = dr
    if not args.no_pairs:
        pr = pairs_leg(dev, M, g, args.steps, args.warmup, args.workload)
        if pr is not None:
            pr["vs_plain"] = pr["value"] / value
            res["frame_pairs"] = pr
    if not args.no_detection:
        dl = detection_leg(dev, sc, M, g)
        if dl is not None:
            res["detection"] = dl
    if batch_in is not None:
        del dev
        torch.cuda.empty_cache()
        res["batch24"] = batch_leg(*batch_in, steps=min(args.steps, 20), warmup=min(args.warmup, 5), tune_iters=3)
        if not args.no_cpu_baseline:
            res["batch24"]["cpu_baseline"] = cpu_baseline_batch(*batch_in)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(frames, wl, g)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
