"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle
checks.

This module only draws inputs: it holds none of the SSIM arithmetic, imports
neither the oracle nor the HIP package, and both sides receive the same arrays
from it.  The paper measured on subjective databases that are not available
here; these planes stand in for them with the paper's shapes and distortion
types (8-bit luma with L=255; encode-ladder resolutions; compression and noise
distortions).

Recipes (all numpy float64 before the final rounding):
  smooth field   N(0,1) on (H+2P)x(W+2P), separable Gaussian blur sigma=4
                 (radius 16, reflect), crop, min-max rescale to [lo, hi],
                 round half to even.
  config 0       256x256 u8 field in [16,235]; dis = clip(round(ref+N(0,10^2))).
  config 1       B frames HxW u8 cropped with a per-frame integer translation
                 (dx,dy) in U{-4..4}^2 from one field; dis = 8x8 block DCT-II
                 (orthonormal) of (x-128), coefficients quantised with an
                 integer step q ~ U{qlo..qhi} per frame, inverse, +128, round,
                 clip [0,255].
  config 2       B frames HxW u16 10-bit (L=1023) in [64,940]; dis = ref +
                 N(0,20^2), then each aligned 4x4 block is replaced by its
                 mean with probability 0.25; round, clip [0,1023].
  config 3       ragged list of u8 pairs at resolutions drawn from the ladder
                 {426x240, 640x360, 854x480, 1280x720, 1920x1080, 2560x1440},
                 config-1 distortion with q ~ U{8..64}, each pair with its own
                 window (Gaussian 11 or box 8) and stride (1 or 4).
  config 4       B x 3 x H x W float32 RGB fields in [16/255, 235/255];
                 dis = ref + N(0, 0.05^2), not clipped.
  video clip     T frames HxW u8 panning across one field (frame f is the crop
                 at (f*vy, f*vx), a constant integer pan), dis = config-1 DCT
                 quantisation per frame with q ~ U{qlo..qhi}; the clips of
                 SSIM-3D (temporally correlated, as in the video databases).
"""
from __future__ import annotations

import numpy as np
from scipy import fft as sfft
from scipy import ndimage

ROOT_SEED = 20210115

LADDER = ((426, 240), (640, 360), (854, 480), (1280, 720), (1920, 1080), (2560, 1440))


def rng_for(config: int, stream: int = 0) -> np.random.Generator:
    ss = np.random.SeedSequence([ROOT_SEED, config, stream])
    return np.random.Generator(np.random.PCG64(ss))


def smooth_field(rng: np.random.Generator, h: int, w: int, lo: float, hi: float,
                 blur_sigma: float = 4.0, pad: int = 16) -> np.ndarray:
    n = rng.standard_normal((h + 2 * pad, w + 2 * pad))
    b = ndimage.gaussian_filter(n, blur_sigma, mode="reflect", truncate=pad / blur_sigma)
    b = b[pad:pad + h, pad:pad + w]
    b = (b - b.min()) / max(b.max() - b.min(), 1e-300)
    return lo + (hi - lo) * b


def _round_clip(a: np.ndarray, lo: float, hi: float, dtype) -> np.ndarray:
    return np.clip(np.rint(a), lo, hi).astype(dtype)


def dct_quantise(frame: np.ndarray, q: int) -> np.ndarray:
    """8x8 block DCT coefficient quantisation of a u8 plane (edge-replicated to
    a multiple of 8, then cropped back)."""
    h, w = frame.shape
    hp, wp = -(-h // 8) * 8, -(-w // 8) * 8
    a = np.pad(frame.astype(np.float64) - 128.0, ((0, hp - h), (0, wp - w)), mode="edge")
    blk = a.reshape(hp // 8, 8, wp // 8, 8).transpose(0, 2, 1, 3)
    c = sfft.dctn(blk, type=2, norm="ortho", axes=(-2, -1))
    c = q * np.rint(c / q)
    r = sfft.idctn(c, type=2, norm="ortho", axes=(-2, -1))
    r = r.transpose(0, 2, 1, 3).reshape(hp, wp)[:h, :w] + 128.0
    return _round_clip(r, 0, 255, np.uint8)


def config0(h: int = 256, w: int = 256, stream: int = 0):
    rng = rng_for(0, stream)
    ref = _round_clip(smooth_field(rng, h, w, 16, 235), 0, 255, np.uint8)
    dis = _round_clip(ref + rng.normal(0.0, 10.0, ref.shape), 0, 255, np.uint8)
    return ref, dis


def config1(frames: int = 64, h: int = 1080, w: int = 1920, qlo: int = 16, qhi: int = 48,
            stream: int = 0):
    rng = rng_for(1, stream)
    field = smooth_field(rng, h + 8, w + 8, 16, 235)
    base = _round_clip(field, 0, 255, np.uint8)
    ref = np.empty((frames, h, w), np.uint8)
    dis = np.empty((frames, h, w), np.uint8)
    for f in range(frames):
        dy, dx = rng.integers(-4, 5, size=2)
        ref[f] = base[4 + dy:4 + dy + h, 4 + dx:4 + dx + w]
        dis[f] = dct_quantise(ref[f], int(rng.integers(qlo, qhi + 1)))
    return ref, dis


def config2(frames: int = 32, h: int = 2160, w: int = 3840, stream: int = 0):
    rng = rng_for(2, stream)
    field = smooth_field(rng, h + 8, w + 8, 64, 940)
    ref = np.empty((frames, h, w), np.uint16)
    dis = np.empty((frames, h, w), np.uint16)
    for f in range(frames):
        dy, dx = rng.integers(-4, 5, size=2)
        r = np.rint(field[4 + dy:4 + dy + h, 4 + dx:4 + dx + w])
        ref[f] = np.clip(r, 0, 1023).astype(np.uint16)
        d = ref[f].astype(np.float64) + rng.normal(0.0, 20.0, (h, w))
        h4, w4 = h // 4, w // 4
        sel = rng.random((h4, w4)) < 0.25
        blk = d[: 4 * h4, : 4 * w4].reshape(h4, 4, w4, 4)
        mean = blk.mean(axis=(1, 3), keepdims=True)
        blk[:] = np.where(sel[:, None, :, None], mean, blk)
        dis[f] = _round_clip(d, 0, 1023, np.uint16)
    return ref, dis


def _config3_pair(args):
    seed, w, h, q, gauss, stride = args
    rng = np.random.Generator(np.random.PCG64(seed))
    ref = _round_clip(smooth_field(rng, h, w, 16, 235), 0, 255, np.uint8)
    dis = dct_quantise(ref, q)
    return {"ref": ref, "dis": dis, "window": "gaussian" if gauss else "box",
            "k": 11 if gauss else 8, "stride": stride}


def config3(pairs: int = 256, ladder=LADDER, stream: int = 0, workers: int = 0):
    """Returns a list of dicts {ref, dis, window, k, stride}.  `workers` > 1
    generates the pairs in a process pool (same result)."""
    rng = rng_for(3, stream)
    jobs = []
    seeds = np.random.SeedSequence([ROOT_SEED, 3, stream, 1]).spawn(pairs)
    for i in range(pairs):
        w, h = ladder[int(rng.integers(0, len(ladder)))]
        q = int(rng.integers(8, 65))
        gauss = bool(rng.integers(0, 2))
        stride = int((1, 4)[int(rng.integers(0, 2))])
        jobs.append((seeds[i], w, h, q, gauss, stride))
    if workers and workers > 1:
        import concurrent.futures as cf
        with cf.ProcessPoolExecutor(max_workers=workers) as ex:
            return list(ex.map(_config3_pair, jobs, chunksize=4))
    return [_config3_pair(j) for j in jobs]


def config4(batch: int = 16, h: int = 512, w: int = 512, stream: int = 0):
    rng = rng_for(4, stream)
    ref = np.empty((batch, 3, h, w), np.float32)
    for b in range(batch):
        for c in range(3):
            ref[b, c] = smooth_field(rng, h, w, 16 / 255, 235 / 255)
    dis = (ref.astype(np.float64) + rng.normal(0.0, 0.05, ref.shape)).astype(np.float32)
    return ref, dis


def stress_pairs(h: int = 61, w: int = 77, stream: int = 0):
    """Adversarial u8 pairs for parity: flat extremes, checkerboards,
    saturated edges, constant frames, noise."""
    rng = rng_for(9, stream)
    yy, xx = np.mgrid[0:h, 0:w]
    cases = {}
    cases["flat_0_255"] = (np.zeros((h, w), np.uint8), np.full((h, w), 255, np.uint8))
    cases["flat_equal"] = (np.full((h, w), 200, np.uint8), np.full((h, w), 200, np.uint8))
    cb = (((yy // 4) + (xx // 4)) % 2 * 255).astype(np.uint8)
    cases["checker"] = (cb, (255 - cb).astype(np.uint8))
    edge = np.where(xx < w // 2, 16, 235).astype(np.uint8)
    cases["edge"] = (edge, np.where(yy < h // 3, 16, 235).astype(np.uint8))
    cases["sat_edge"] = (np.where((xx + yy) % 23 < 11, 0, 255).astype(np.uint8),
                         np.where((xx * 3 + yy) % 29 < 13, 0, 255).astype(np.uint8))
    cases["noise"] = (rng.integers(0, 256, (h, w)).astype(np.uint8),
                      rng.integers(0, 256, (h, w)).astype(np.uint8))
    cases["identical"] = (cases["noise"][0], cases["noise"][0].copy())
    cases["blocky_flat"] = (np.where((yy // 16 + xx // 16) % 2 == 0, 20, 230).astype(np.uint8),
                            np.where((yy // 16 + xx // 16) % 2 == 0, 22, 229).astype(np.uint8))
    return cases


def video_clip(frames: int = 16, h: int = 270, w: int = 480, vy: int = 1, vx: int = 2, qlo: int = 16,
               qhi: int = 48, stream: int = 0):
    rng = rng_for(5, stream)
    field = smooth_field(rng, h + abs(vy) * frames, w + abs(vx) * frames, 16, 235)
    base = _round_clip(field, 0, 255, np.uint8)
    ref = np.empty((frames, h, w), np.uint8)
    dis = np.empty((frames, h, w), np.uint8)
    oy = 0 if vy >= 0 else abs(vy) * frames
    ox = 0 if vx >= 0 else abs(vx) * frames
    for f in range(frames):
        r0, c0 = oy + f * vy, ox + f * vx
        ref[f] = base[r0:r0 + h, c0:c0 + w]
        dis[f] = dct_quantise(ref[f], int(rng.integers(qlo, qhi + 1)))
    return ref, dis
