"""Pins of the SSIM-3D / MS-SSIM-3D oracle (Spatio-Temporal SSIM subsection)
against what the definition fixes independently of the oracle's own code:
the 2-D SSIM at kt = 1 and on static clips, brute force on a tiny clip, the
paper's rolling temporal sums with integral images, identity and symmetry."""
import math

import numpy as np
import pytest

import oracle as O
import synth



def _clip(T, H, W, seed, lo=0, hi=256):
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi, (T, H, W)).astype(np.uint8)


def _pair(T, H, W, seed):
    """Correlated u8 clips: a smooth moving field and a noisy copy."""
    rng = np.random.default_rng(seed)
    base = synth.smooth_field(rng, H + T, W + T, 20, 230)
    x = np.stack([base[t:t + H, t:t + W] for t in range(T)])
    y = np.clip(x + rng.normal(0, 15, x.shape), 0, 255)
    return np.rint(x).astype(np.uint8), np.rint(y).astype(np.uint8)


BOX = O.SSIMParams(window="box", k=5)


def test_kt1_is_framewise_box_ssim():
    x, y = _pair(4, 23, 29, 1)
    m3 = O.ssim3d_map(x, y, BOX, 1)["map"]
    for t in range(4):
        np.testing.assert_allclose(m3[t], O.ssim_map(x[t], y[t], BOX)["map"], rtol=0, atol=1e-14)


@pytest.mark.parametrize("kt", [2, 3, 7])
def test_static_clip_equals_2d(kt):
    x0, y0 = _pair(1, 30, 26, 2)
    x = np.repeat(x0, kt + 2, axis=0)
    y = np.repeat(y0, kt + 2, axis=0)
    m3 = O.ssim3d_map(x, y, BOX, kt)["map"]
    m2 = O.ssim_map(x0[0], y0[0], BOX)["map"]
    assert m3.shape == (3, 26, 22)
    for t in range(3):
        np.testing.assert_array_equal(m3[t], m2)


def test_brute_force_tiny():
    x = _clip(4, 5, 6, 3)
    y = _clip(4, 5, 6, 4)
    p = O.SSIMParams(window="box", k=3)
    kt = 2
    got = O.ssim3d_map(x, y, p, kt)["map"]
    for t in range(3):
        for i in range(3):
            for j in range(4):
                xs = [float(x[t + a, i + b, j + c]) for a in range(kt) for b in range(3) for c in range(3)]
                ys = [float(y[t + a, i + b, j + c]) for a in range(kt) for b in range(3) for c in range(3)]
                n = len(xs)
                mx, my = sum(xs) / n, sum(ys) / n
                vx = sum((v - mx) ** 2 for v in xs) / n
                vy = sum((v - my) ** 2 for v in ys) / n
                cv = sum((a - mx) * (b - my) for a, b in zip(xs, ys)) / n
                q = ((2 * mx * my + p.C1) * (2 * cv + p.C2)) / ((mx * mx + my * my + p.C1) * (vx + vy + p.C2))
                assert abs(got[t, i, j] - q) < 1e-12, (t, i, j)


def test_rolling_temporal_sums_and_integral_images():
    """The paper's O(MN)-per-frame scheme: temporal sums updated frame by frame
    (add the entering frame, drop the one leaving), then four-corner sums of
    their integral images."""
    x, y = _pair(9, 21, 24, 5)
    k, kt = 4, 3
    want = O.box_sums3d(x, y, k, kt)
    planes = [a.astype(np.int64) for a in (x, y)]
    mom = [planes[0], planes[1], planes[0] ** 2, planes[1] ** 2, planes[0] * planes[1]]
    T = x.shape[0]
    run = [np.zeros(x.shape[1:], np.int64) for _ in range(5)]
    for f in range(T):
        for q in range(5):
            run[q] += mom[q][f]
            if f >= kt:
                run[q] -= mom[q][f - kt]
        if f < kt - 1:
            continue
        t = f - kt + 1
        for q in range(5):
            sat = np.zeros((run[q].shape[0] + 1, run[q].shape[1] + 1), np.int64)
            sat[1:, 1:] = run[q].cumsum(0).cumsum(1)
            ho, wo = want[q].shape[1:]
            box = sat[k:k + ho, k:k + wo] - sat[0:ho, k:k + wo] - sat[k:k + ho, 0:wo] + sat[0:ho, 0:wo]
            np.testing.assert_array_equal(box, want[q][t])


def test_identity_symmetry_and_range():
    x, y = _pair(6, 25, 27, 6)
    p = O.SSIMParams(window="box", k=11)
    assert np.all(O.ssim3d(x, x, p, 4) == 1.0)
    a = O.ssim3d_map(x, y, p, 4)["map"]
    b = O.ssim3d_map(y, x, p, 4)["map"]
    np.testing.assert_array_equal(a, b)
    assert np.all(a <= 1.0) and np.all(a > -1.0)
    s = O.ssim3d(x, y, p, 4)
    np.testing.assert_allclose(s, [a[t].mean() for t in range(3)], rtol=0, atol=1e-15)


def test_float_clip_matches_integer_clip():
    x, y = _pair(5, 20, 19, 7)
    a = O.ssim3d_map(x, y, BOX, 2)["map"]
    b = O.ssim3d_map(x.astype(np.float32), y.astype(np.float64), BOX, 2)["map"]
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12)


def test_msssim3d_kt1_is_framewise_msssim():
    x, y = _pair(3, 64, 72, 8)
    r3 = O.msssim3d(x, y, BOX, 1, n_scales=3, renorm=True)
    for t in range(3):
        r2 = O.msssim(x[t], y[t], BOX, n_scales=3, renorm=True)
        assert abs(r3["score"][t] - r2["score"]) < 1e-12
        np.testing.assert_allclose(r3["cs"][t], r2["cs"], rtol=0, atol=1e-12)
    rs = O.msssim3d(x, y, BOX, 1, n_scales=3, aggregation="sum")
    for t in range(3):
        assert abs(rs["score"][t] - O.msssim(x[t], y[t], BOX, n_scales=3, aggregation="sum")["score"]) < 1e-12


def test_msssim3d_static_clip_and_identity():
    x0, y0 = _pair(1, 64, 64, 9)
    x = np.repeat(x0, 5, axis=0)
    y = np.repeat(y0, 5, axis=0)
    r = O.msssim3d(x, y, BOX, 3, n_scales=3, renorm=True)
    want = O.msssim(x0[0], y0[0], BOX, n_scales=3, renorm=True)["score"]
    assert np.all(np.abs(r["score"] - want) < 1e-12)
    assert np.all(np.abs(O.msssim3d(x, x, BOX, 3, n_scales=3)["score"] - 1.0) < 1e-13)
    assert math.isfinite(float(r["score"][0]))
