"""Benchmark of the SSIM hot path on one MI355X.

Workload (one step): 64 frames of 1920x1080 uint8 luma (smooth fields with a
per-frame translation, 8x8 block-DCT quantisation with step 16..48), SSIM with
an 11x11 Gaussian window (sigma 1.5), K1=0.01, K2=0.03, L=255, valid, stride 1:
forward (quality map + pooled score per frame) followed by the pooled
backward (gradient with respect to the distorted frames).  Inputs are resident
in HBM before the timed region.

Prints ONE JSON line.  Throughput counts full-resolution input pixels (one
per reference/distorted pair).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
# Algorithmic HBM bytes per input pixel of the headline step (u8 x and y):
# forward reads x, y (2 B) and writes the float32 map (4 B per map position)
# and one score per frame; the pooled backward reads x, y (2 B) and writes the
# float32 gradient (4 B), plus one upstream value per frame.
FWD_READ_B_PER_PX, MAP_B_PER_POS, BWD_B_PER_PX = 2, 4, 2 + 4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the secondary workloads (box / integral image / stride 4 / MS-SSIM 4K / ragged / loss)")
    ap.add_argument("--fwd-only", action="store_true", help="time the forward alone (profiling)")
    ap.add_argument("--only", default="",
                    help="comma-separated name prefixes: run only these secondary workloads (profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="run one plain device-to-device copy of BYTES (counter calibration) and exit")
    return ap.parse_args()


def copy_calibration(nbytes: int) -> None:
    """One plain copy kernel of known size: the scale for FETCH_SIZE /
    WRITE_SIZE counter readings."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4}))


def kernel_source_hash() -> str:
    """Hash of every kernel and host source of the library: a committed PMC
    figure is used only while the sources it was taken on are unchanged."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2101_06354_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_counters() -> dict:
    """Per-step figures of the headline step from the committed rocprofv3 PMC
    summary (HBM bytes from FETCH_SIZE / WRITE_SIZE scaled by a plain copy's
    reading, VALU activity), if they were taken on the current sources; else
    {}."""
    path = os.path.join(ROOT, "profiles", "pmc_counters.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return {}
    if d.get("source_hash") != kernel_source_hash():
        return {}
    return d


_CPU_FRAMES = None  # (x, y) for the forked oracle workers


def _oracle_frame(args):
    f, with_bwd = args
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass
    import oracle as O
    x, y = _CPU_FRAMES
    p = O.SSIMParams()
    r = O.ssim_map(x[f], y[f], p)
    O.mean_pool(r["map"])
    if with_bwd:
        O.ssim_pooled_backward(x[f], y[f], 1.0, p)
    return f


def _host() -> dict:
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def measured_copy_gbs(torch, dev, stream, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Device-to-device copy bandwidth (bytes read + written per second) of a
    plain 1 GiB copy, HIP events on the launch stream."""
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        b.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(x, y, with_bwd: bool, min_seconds: float = 10.0) -> dict:
    """The FP64 oracle as it stands on a bounded sample of the same workload:
    one process (about min_seconds of frames), then one frame per worker in a
    pool of up to 16 forked processes (the host cores; workers fork before any
    GPU work and never exec).  The pool figure is the headline one."""
    global _CPU_FRAMES
    import multiprocessing as mp
    import resource
    what = "forward+backward" if with_bwd else "forward"
    _CPU_FRAMES = (x, y)
    # single process
    t0 = time.perf_counter()
    done = 0
    while done < 1 or (done < x.shape[0] and time.perf_counter() - t0 < min_seconds):
        _oracle_frame((done, with_bwd))
        done += 1
    dt1 = time.perf_counter() - t0
    px = x.shape[1] * x.shape[2]
    single = {"value": done * px / dt1 / 1e6, "cores": 1,
              "sample": f"{done} of the {x.shape[0]} 1080p frames, {what}, {dt1:.1f} s wall"}
    # process pool over frames
    n = max(1, min(16, os.cpu_count() or 1, x.shape[0]))
    ru0 = resource.getrusage(resource.RUSAGE_CHILDREN)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(n) as pool:
        pool.map(_oracle_frame, [(f, with_bwd) for f in range(n)], chunksize=1)
    dtn = time.perf_counter() - t0
    ru1 = resource.getrusage(resource.RUSAGE_CHILDREN)
    user = (ru1.ru_utime - ru0.ru_utime)
    _CPU_FRAMES = None
    return {"value": n * px / dtn / 1e6, "unit": "Mpixel/s", "cores": n, "kind": "oracle",
            "sample": f"{n} of the {x.shape[0]} 1080p frames, one per worker process, FP64 numpy, {what}, "
                      f"{dtn:.1f} s wall, {user:.1f} s user",
            "single_process": single, "host": _host()}


def main():
    a = parse()
    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the SSIM path is measured on a single MI355X "
              "(frames shard across GPUs with no communication; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import synth

    log("generating 64 x 1080p u8 pairs")
    x, y = synth.config1(frames=a.frames)
    cpu = None
    if not a.no_cpu_baseline:
        # before any GPU work: the oracle workers are forked from this process
        log("CPU baseline (FP64 oracle)")
        cpu = cpu_baseline(x, y, not a.fwd_only)

    import torch

    import paper_2101_06354_amd as P

    dev = torch.device("cuda:0")
    B, H, W = x.shape
    xt = torch.from_numpy(x).to(dev)
    yt = torch.from_numpy(y).to(dev)
    cfg = P.SSIMConfig()
    ho, wo = P.map_shape(cfg, H, W)
    stream = torch.cuda.current_stream(dev)

    # probe the backward once; a build without it times the forward alone
    with_bwd = not a.fwd_only
    if with_bwd:
        try:
            P.ssim_backward(xt[:1], yt[:1], torch.ones(1, device=dev), cfg)
        except P._lib.SSIMXError as e:
            if e.status != P._lib.ENOTSUP:
                raise
            with_bwd = False

    # preallocated outputs / workspaces (outside the timed region)
    import ctypes
    L = P._lib
    pc = cfg.to_c()
    xi, yi = P.ops._image(xt), P.ops._image(yt)
    qmap = torch.empty((B, ho, wo), dtype=torch.float32, device=dev)
    score = torch.empty(B, dtype=torch.float32, device=dev)
    ws_f = torch.empty(P.workspace_size(cfg, L.OP_MAP, L.U8, H, W, B), dtype=torch.uint8, device=dev)
    grad = torch.empty((B, H, W), dtype=torch.float32, device=dev)
    gscore = torch.full((B,), 1.0, dtype=torch.float32, device=dev)
    ws_b = None
    if with_bwd:
        ws_b = torch.empty(P.workspace_size(cfg, L.OP_POOLED_BACKWARD, L.U8, H, W, B), dtype=torch.uint8,
                           device=dev)

    def fwd():
        L.check(L.lib.ssim_map(ctypes.byref(pc), ctypes.byref(xi), ctypes.byref(yi), B, qmap.data_ptr(), wo,
                               ho * wo, score.data_ptr(), ws_f.data_ptr(), ws_f.numel(), stream.cuda_stream),
                "ssim_map")

    def bwd():
        L.check(L.lib.ssim_pooled_backward(ctypes.byref(pc), ctypes.byref(xi), ctypes.byref(yi), B,
                                           gscore.data_ptr(), grad.data_ptr(), W, H * W, ws_b.data_ptr(),
                                           ws_b.numel(), stream.cuda_stream), "ssim_pooled_backward")

    log("warm-up and timed steps")
    for _ in range(a.warmup):
        fwd()
        if with_bwd:
            bwd()
    torch.cuda.synchronize()

    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        ev[s][0].record(stream)
        fwd()
        ev[s][1].record(stream)
        if with_bwd:
            bwd()
        ev[s][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    fwd_ms = [ev[s][0].elapsed_time(ev[s][1]) for s in range(a.steps)]
    bwd_ms = [ev[s][1].elapsed_time(ev[s][2]) for s in range(a.steps)]
    dev_step_ms = [ev[s][0].elapsed_time(ev[s][2]) for s in range(a.steps)]
    step_ms = wall * 1e3 / a.steps

    def spread(v):
        q = np.percentile(v, [25, 50, 75])
        return {"median": float(q[1]), "iqr": float(q[2] - q[0]),
                "median_of_first_5": float(np.median(v[:5]))}

    timing = {"fwd_ms": spread(fwd_ms), "step_ms_device": spread(dev_step_ms)}
    if with_bwd:
        timing["bwd_ms"] = spread(bwd_ms)
    copy_gbs = measured_copy_gbs(torch, dev, stream)
    px = B * H * W
    value = px / (step_ms * 1e-3) / 1e6
    fwd_avg = float(np.mean(fwd_ms))
    out_px = B * ho * wo

    fwd_bytes = px * FWD_READ_B_PER_PX + out_px * MAP_B_PER_POS + B * 4   # x, y in; map and scores out
    bwd_bytes = px * BWD_B_PER_PX + B * 4 if with_bwd else 0               # x, y in; gradient out
    step_bytes = fwd_bytes + bwd_bytes
    bwd_avg = float(np.mean(bwd_ms)) if with_bwd else None
    pmc = measured_counters()

    def hbm(nbytes, ms):
        gbs = nbytes / (ms * 1e-3) / 1e9
        return {"achieved": gbs, "frac": gbs / HBM_PEAK_GBS, "frac_of_copy": gbs / copy_gbs, "ms": ms,
                "alg_bytes": nbytes, "alg_bytes_per_input_px": nbytes / px}

    step = hbm(step_bytes, step_ms)
    kernels = pmc.get("kernels", {})
    res = {
        "metric": "SSIM Mpixel/s fwd & fwd+bwd (1080p luma, Gaussian 11x11); % HBM roofline",
        "value": value,
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8 in, f32 accumulate",
        "data": "synthetic",
        "config": {"workload": f"{B}x1080p u8 luma pairs, SSIM Gaussian 11x11 sigma 1.5, valid, stride 1, "
                               f"{'forward (map+score) + pooled backward' if with_bwd else 'forward (map+score)'}",
                   "frames": B, "height": H, "width": W, "window": "gaussian", "k": 11, "stride": 1},
        "fwd_mpixel_s": px / (fwd_avg * 1e-3) / 1e6,
        "fwd_ms": fwd_avg,
        "fwd_bwd_mpixel_s": value if with_bwd else None,
        "bwd_ms": bwd_avg,
        # The headline step (forward + pooled backward) against the HBM roof:
        # algorithmic bytes over the step time.  `traffic` is the HBM bytes the
        # step's kernels moved per step (rocprofv3 FETCH_SIZE + WRITE_SIZE,
        # scaled by a plain copy's reading), null when the committed counters
        # predate the current sources.  The kernels are bound by VALU issue,
        # not by HBM: `kernels` gives each one's counter-derived VALU activity.
        "roofline": {"bound": "hbm", "scope": "forward + pooled backward step" if with_bwd else "forward",
                     "achieved": step["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": step["frac"],
                     "traffic": pmc.get("bytes_per_step") if with_bwd else pmc.get("fwd_bytes_per_step"),
                     "alg_bytes_per_step": step_bytes, "alg_bytes_per_input_px": step_bytes / px,
                     "measured_copy_gbs": copy_gbs, "frac_of_copy": step["frac_of_copy"],
                     "forward": hbm(fwd_bytes, fwd_avg),
                     "backward": hbm(bwd_bytes, bwd_avg) if with_bwd else None,
                     "kernels": kernels or None,
                     "counters": pmc.get("summary")},
        "timing": timing,
    }
    if not a.no_variants:
        res["variants"] = variants(P, x, y, xt, yt, dev, stream, [o for o in a.only.split(",") if o])
    if cpu is not None:
        res["cpu_baseline"] = cpu
    print(json.dumps(res))


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _time(fn, reps=10, warmup=2, stream=None):
    """Mean device time (ms) of fn() over reps calls, HIP events on `stream`."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def variants(P, x, y, xt, yt, dev, stream, only=()):
    """Secondary workloads, each timed on device-resident inputs (all, or
    those whose names start with one of `only`)."""
    out = {}
    B, H, W = x.shape
    px1 = B * H * W

    def rec(name, ms, px, note):
        out[name] = {"ms": ms, "mpixel_s": px / (ms * 1e-3) / 1e6, "note": note}

    def want(*names):
        return not only or any(n.startswith(o) for n in names for o in only)

    # 64 x 1080p u8: other windows / algorithms / strides (map + score)
    for name, cfg, note in [
        ("c1_gauss11_pooled_only", P.SSIMConfig(), "Gaussian 11x11, score only (no map store)"),
        ("c1_box8_tile_sums", P.SSIMConfig(window="box", k=8), "8x8 box, exact tile-local integer sums, map+score"),
        ("c1_box8_integral_image", P.SSIMConfig(window="box", k=8, algo="integral"),
         "8x8 box via the five uint32 integral images in HBM (the paper's method), map+score"),
        ("c1_gauss11_stride4", P.SSIMConfig(stride=4), "Gaussian 11x11, stride 4, map+score"),
        ("c1_box8_stride4", P.SSIMConfig(window="box", k=8, stride=4), "8x8 box, stride 4, map+score"),
    ]:
        if not want(name):
            continue
        if name.endswith("pooled_only"):
            ms = _time(lambda c=cfg: P.ssim(xt, yt, c), stream=stream)
        else:
            ms = _time(lambda c=cfg: P.ssim(xt, yt, c, return_map=True), stream=stream)
        rec(name, ms, px1, note)
        log(f"{name}: {ms:.3f} ms")
    # one batched launch vs one launch per frame (same frames, Gaussian map+score)
    cfg = P.SSIMConfig()
    if want("c1_batched_launch", "c1_per_frame_launches"):
        ms_b = _time(lambda: P.ssim(xt, yt, cfg, return_map=True), stream=stream)
        ms_f = _time(lambda: [P.ssim(xt[f], yt[f], cfg, return_map=True) for f in range(B)], reps=3, stream=stream)
        rec("c1_batched_launch", ms_b, px1, "64 frames in one launch")
        rec("c1_per_frame_launches", ms_f, px1, "64 single-frame launches")
    # one GPU's share of an 8-way frame split: forward + pooled backward on 8 frames
    if want("c1_shard_8_frames_fwd_bwd"):
        import torch

        ones = torch.ones(8, device=dev)
        ms = _time(lambda: (P.ssim(xt[:8], yt[:8], cfg, return_map=True), P.ssim_backward(xt[:8], yt[:8], ones, cfg)),
                   stream=stream)
        rec("c1_shard_8_frames_fwd_bwd", ms, px1 // 8, "8 of the frames (one GPU's share of 8), forward + backward")
    # spatial pooling of the 64 x 1080p Gaussian map; Enhanced SSIM; colour SSIM
    if want("c1_pool_cov", "c1_pool_five_number"):
        _, qm = P.ssim(xt, yt, cfg, return_map=True)
        for kind in ("cov", "five_number"):
            ms = _time(lambda k=kind: P.pool(qm, k), stream=stream)
            rec(f"c1_pool_{kind}", ms, px1, f"{kind} pooling of the 64 x 1070x1910 map (map given)")
        del qm
    if want("c1_enhanced_ssim"):
        ms = _time(lambda: P.enhanced_ssim(xt, yt), stream=stream)
        rec("c1_enhanced_ssim", ms, px1, "pre-scaling by 5x5 means, 11x11 box at stride 5, CoV pooling")
    if want("c1_color_ssim"):
        xr, yr = xt[:63].reshape(21, 3, H, W), yt[:63].reshape(21, 3, H, W)
        ms = _time(lambda: P.color_ssim(xr, yr, cfg), stream=stream)
        rec("c1_color_ssim", ms, 21 * H * W, "21 RGB 1080p u8 frames (planes from the luma batch), BT.709 "
            "YCbCr, Gaussian 11x11 per channel, 0.8/0.1/0.1")
    if want("c1_ssim3d_kt5", "c1_msssim3d_kt5"):
        # the 64 frames as one clip; 60 map frames of the 11 x 11 x 5 box
        kt, n_out = 5, xt.shape[0] - 4
        box = P.SSIMConfig(window="box", k=11)
        ms = _time(lambda: P.ssim3d(xt, yt, kt, box), stream=stream)
        rec("c1_ssim3d_kt5", ms, n_out * H * W, "SSIM-3D, 64-frame 1080p u8 clip, 11x11x5 box, rolling "
            "temporal sums, per-frame means (60 map frames)")
        ms = _time(lambda: P.ms_ssim3d(xt, yt, kt, box), stream=stream)
        rec("c1_msssim3d_kt5", ms, n_out * H * W, "MS-SSIM-3D, same clip, 5 scales, 11x11x5 box")
    if want("c2_"):
        _variants_c2(P, dev, stream, rec)
    if want("c3_"):
        _variants_c3(P, dev, stream, rec)
    if want("c4_"):
        _variants_c4(P, dev, stream, rec)
    return out


def _variants_c2(P, dev, stream, rec):
    import torch

    import synth

    # MS-SSIM, 32 x 3840x2160 10-bit, 5 scales
    log("generating 32 x 4K u16 pairs")
    r2, d2 = synth.config2()
    x2 = torch.from_numpy(r2).to(dev)
    y2 = torch.from_numpy(d2).to(dev)
    del r2, d2
    c2 = P.SSIMConfig(L=1023.0)
    ms = _time(lambda: P.ms_ssim(x2, y2, c2), reps=5, stream=stream)
    rec("c2_msssim_4k_u16_fwd", ms, x2.numel(), "32x2160x3840 u16, 5 scales, score per frame")
    ms = _time(lambda: P.ms_ssim_backward(x2[:8], y2[:8], torch.ones(8, device=dev), c2), reps=3,
               stream=stream)
    rec("c2_msssim_4k_u16_bwd_8frames", ms, x2[:8].numel(), "adjoint of MS-SSIM on 8 of the frames")
    sc, cs = P.ms_ssim(x2[:8], y2[:8], c2, return_cs=True)
    ms = _time(lambda: P.ms_ssim_backward(x2[:8], y2[:8], torch.ones(8, device=dev), c2, fwd=(sc, cs)), reps=3,
               stream=stream)
    rec("c2_msssim_4k_u16_bwd_8frames_given_fwd", ms, x2[:8].numel(),
        "the same adjoint given the forward's score and per-scale values (msssim_backward_values)")
    del x2, y2


def _variants_c3(P, dev, stream, rec):
    import torch

    import synth
    # ragged batch: 256 pairs, one graph launch vs per-pair launches
    log("generating 256 ragged pairs")
    pairs = synth.config3(workers=8)
    items = [{"ref": torch.from_numpy(p["ref"]).to(dev), "dis": torch.from_numpy(p["dis"]).to(dev),
              "cfg": P.SSIMConfig(window=p["window"], k=p["k"], stride=p["stride"])} for p in pairs]
    tuned = set()
    for it in items:  # tile shapes from the autotuner, before the plan is built
        h, w = it["ref"].shape
        key = (it["cfg"].window, it["cfg"].k, it["cfg"].stride, h, w)
        if key not in tuned:
            P.autotune(it["cfg"], torch.uint8, h, w, 1)
            tuned.add(key)
    log(f"autotuned {len(tuned)} shapes; building the plan")
    plan = P.BatchPlan(items)
    pxr = sum(int(it["ref"].numel()) for it in items)
    sc = torch.empty(len(items), dtype=torch.float32, device=dev)
    ms_g = _time(lambda: plan.run(sc), stream=stream)
    ms_u = _time(lambda: plan.run_unbatched(sc), stream=stream)
    ni, nb = plan.info()
    rec("c3_ragged_graph", ms_g, pxr, f"256 ladder pairs, one hipGraph launch ({ni} tiles, {nb} blocks)")
    rec("c3_ragged_per_pair", ms_u, pxr, "same pairs, per-pair kernel launches")
    plan.close()
    del items


def _variants_c4(P, dev, stream, rec):
    import torch

    import synth
    log("differentiable loss workload")
    # differentiable loss: 16 x 3 x 512 x 512 RGB, 1 - MS-SSIM (3 scales) forward + backward
    r4, d4 = synth.config4()
    rt = torch.from_numpy(r4).to(dev)
    dt = torch.from_numpy(d4).to(dev).requires_grad_(True)
    c4 = P.SSIMConfig(L=1.0)
    px = 16 * 512 * 512

    def step(loss_fn):
        dt.grad = None
        loss = loss_fn(rt, dt, c4, n_scales=3, renorm=True)
        loss.backward()
    ms = _time(lambda: step(P.autograd.ms_ssim_loss_rgb), stream=stream)
    rec("c4_msssim_loss_fwd_bwd", ms, px, "16x3x512x512 f32 RGB, BT.601 luma, 3 scales, loss + gradient "
        "(autograd: one graph replay of a cached loss plan, then the upstream scaling)")
    plan = P.LossPlan(c4, torch.float32, 16, 512, 512, device=dev)
    ms = _time(lambda: plan.run(rt, dt.detach()), stream=stream)
    rec("c4_msssim_loss_plan_replay", ms, px, "the same loss and gradient, one LossPlan graph replay per step")
    plan.close()
    ms = _time(lambda: P.msssim_loss_rgb(rt, dt.detach(), c4), stream=stream)
    rec("c4_msssim_loss_eager_call", ms, px, "the same loss and gradient, one eager library call per step")
    ms = _time(lambda: step(P.autograd.ms_ssim_loss_rgb_composed), stream=stream)
    rec("c4_msssim_loss_composed", ms, px, "the same loss from the separate differentiable pieces (luma, "
        "MS-SSIM, torch mean) under autograd")


if __name__ == "__main__":
    main()
