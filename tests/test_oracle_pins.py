"""Pins of the FP64 oracle against facts that the paper and mathematics fix
(not against the oracle itself): library routines, closed forms, invariants,
hand-worked values, exact integer identities and finite differences."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import signal

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_u8(shape, seed):
    return np.random.default_rng(seed).integers(0, 256, shape).astype(np.uint8)


# ---------------------------------------------------------------- windows
@pytest.mark.parametrize("k,sigma", [(11, 1.5), (7, 1.0), (15, 2.5), (3, 0.5)])
def test_gaussian_taps_match_scipy_window(k, sigma):
    ref = signal.windows.gaussian(k, std=sigma, sym=True)
    ref = ref / ref.sum()
    np.testing.assert_allclose(O.window_1d("gaussian", k, sigma), ref, rtol=0, atol=1e-15)


def test_window_2d_sums_to_one_and_is_separable():
    w = O.window_2d("gaussian", 11, 1.5)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.linalg.matrix_rank(w) == 1
    np.testing.assert_array_equal(w, w.T)
    assert np.allclose(O.window_2d("box", 8), 1 / 64)


# ---------------------------------------------------------------- moments
@pytest.mark.parametrize("window,k,stride", [("gaussian", 11, 1), ("gaussian", 7, 3), ("box", 8, 1), ("box", 5, 4)])
def test_direct_equals_separable(window, k, stride):
    x = _rand_u8((37, 45), 1).astype(np.float64)
    y = _rand_u8((37, 45), 2).astype(np.float64)
    a = O.moments_direct(x, y, O.window_2d(window, k), stride)
    b = O.moments_separable(x, y, O.window_1d(window, k), stride)
    for u, v in zip(a, b):
        np.testing.assert_allclose(u, v, rtol=1e-12, atol=1e-9)


def test_moments_match_scipy_correlate2d():
    x = _rand_u8((29, 33), 3).astype(np.float64)
    y = _rand_u8((29, 33), 4).astype(np.float64)
    w = O.window_2d("gaussian", 11, 1.5)
    got = O.moments_direct(x, y, w)
    want = [signal.correlate2d(a, w, mode="valid") for a in (x, y, x * x, y * y, x * y)]
    for u, v in zip(got, want):
        np.testing.assert_allclose(u, v, rtol=1e-12, atol=1e-9)


def test_hand_worked_golden_cases():
    rows = [r for r in open(os.path.join(GOLDEN, "hand_worked.txt")) if r.strip() and not r.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        name, xs, ys, c1, c2, l, cs, q = [f.strip() for f in r.split("|")]
        x = np.array([int(t) for t in xs.split()], dtype=np.uint8).reshape(2, 2)
        y = np.array([int(t) for t in ys.split()], dtype=np.uint8).reshape(2, 2)
        p = O.SSIMParams(window="box", k=2, C1=float(c1), C2=float(c2))
        for form in ("separable", "direct"):
            res = O.ssim_map(x, y, p, form)
            assert res["map"].shape == (1, 1), name
            assert abs(res["l"][0, 0] - float(l)) < 1e-15, name
            assert abs(res["cs"][0, 0] - float(cs)) < 1e-15, name
            assert abs(res["map"][0, 0] - float(q)) < 1e-15, name
        # same values through the float path (non-integer planes)
        res = O.ssim_map(x.astype(np.float64), y.astype(np.float64), p)
        assert abs(res["map"][0, 0] - float(q)) < 1e-15, name


def _fraction_ssim(x, y, k, C1, C2):
    """Exact rational SSIM of every box window of tiny integer planes."""
    h, w = len(x), len(x[0])
    out = []
    n = Fraction(1, k * k)
    for i in range(h - k + 1):
        row = []
        for j in range(w - k + 1):
            vx = [x[i + m][j + c] for m in range(k) for c in range(k)]
            vy = [y[i + m][j + c] for m in range(k) for c in range(k)]
            mx = sum(Fraction(v) for v in vx) * n
            my = sum(Fraction(v) for v in vy) * n
            dx = [v - mx for v in vx]
            dy = [v - my for v in vy]
            sxx = sum(d * d for d in dx) * n
            syy = sum(d * d for d in dy) * n
            sxy = sum(a * b for a, b in zip(dx, dy)) * n
            l = (2 * mx * my + C1) / (mx * mx + my * my + C1)
            cs = (2 * sxy + C2) / (sxx + syy + C2)
            row.append(l * cs)
        out.append(row)
    return out


@pytest.mark.parametrize("k", [2, 3])
def test_exact_rational_brute_force_central_moments(k):
    # central (two-pass) moments in exact rationals: a different formula from
    # the oracle's raw-moment form, equal in exact arithmetic
    x = _rand_u8((6, 7), 11)
    y = _rand_u8((6, 7), 12)
    C1, C2 = Fraction(13, 2), Fraction(117, 2)
    want = _fraction_ssim(x.tolist(), y.tolist(), k, C1, C2)
    got = O.ssim_map(x, y, O.SSIMParams(window="box", k=k, C1=float(C1), C2=float(C2)))["map"]
    np.testing.assert_allclose(got, np.array([[float(v) for v in r] for r in want]), rtol=0, atol=1e-14)


# ---------------------------------------------------------------- invariants
def test_identity_is_one_and_unique_max():
    x = _rand_u8((40, 50), 5)
    p = O.SSIMParams()
    m = O.ssim_map(x, x, p)["map"]
    np.testing.assert_allclose(m, 1.0, rtol=0, atol=1e-13)
    y = x.copy()
    y[20, 25] ^= 1
    assert O.ssim_pooled(x, y, p) < 1.0


@pytest.mark.parametrize("window,k", [("gaussian", 11), ("box", 8)])
def test_symmetry_and_boundedness(window, k):
    x = _rand_u8((33, 41), 6)
    y = _rand_u8((33, 41), 7)
    p = O.SSIMParams(window=window, k=k)
    a = O.ssim_map(x, y, p)["map"]
    b = O.ssim_map(y, x, p)["map"]
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)
    assert np.all(np.abs(a) <= 1.0 + 1e-12)
    # anti-correlated patterns give negative local quality
    assert a.min() < 0


@pytest.mark.parametrize("a,b", [(16, 235), (100, 120), (0, 0), (255, 254), (3, 7)])
def test_constant_images_luminance_closed_form(a, b):
    p = O.SSIMParams()
    x = np.full((20, 23), a, np.uint8)
    y = np.full((20, 23), b, np.uint8)
    r = O.ssim_map(x, y, p)
    want = (2 * a * b + p.C1) / (a * a + b * b + p.C1)
    np.testing.assert_allclose(r["cs"], 1.0, atol=1e-12)
    np.testing.assert_allclose(r["map"], want, rtol=0, atol=1e-12)
    if a > 0:
        lam = (b - a) / a
        weber = (2 * (1 + lam) + p.C1 / a**2) / (1 + (1 + lam) ** 2 + p.C1 / a**2)
        np.testing.assert_allclose(r["l"], weber, rtol=0, atol=1e-12)


def test_affine_pair_gives_weber_contrast_form():
    # y = alpha x + beta  ->  s = 1 and cs = c(Sigma) with 1+Sigma = alpha
    x = _rand_u8((25, 25), 8).astype(np.float64)
    alpha, beta = 0.6, 40.0
    y = alpha * x + beta
    p = O.SSIMParams()
    r = O.ssim_map(x, y, p)
    w = O.window_2d("gaussian", 11, 1.5)
    for (i, j) in [(0, 0), (3, 9), (14, 14), (7, 2)]:
        win = x[i:i + 11, j:j + 11]
        mu = np.average(win, weights=w)
        var1 = np.average((win - mu) ** 2, weights=w)
        want = (2 * alpha + p.C2 / var1) / (1 + alpha**2 + p.C2 / var1)
        assert abs(r["cs"][i, j] - want) < 1e-12


# ---------------------------------------------------------------- rectangular windows
def test_integral_image_four_corner_equals_direct_sums():
    x = _rand_u8((45, 52), 9)
    y = _rand_u8((45, 52), 10)
    for k, s in [(8, 1), (8, 4), (11, 1), (3, 2)]:
        direct = O.box_sums_direct(x, y, k, s)
        ho, wo = O.map_shape(45, 52, k, s, "valid")
        via = O.box_sums_integral(O.integral_images(x, y), k, s, ho, wo)
        for u, v in zip(direct, via):
            np.testing.assert_array_equal(u, v)


def test_integral_image_wraps_and_stays_exact():
    x = np.full((300, 300), 255, np.uint8)
    y = np.full((300, 300), 254, np.uint8)
    sats = O.integral_images(x, y)
    full = 300 * 300 * 255 * 255
    assert full > 2**32
    assert int(sats[2][-1, -1]) == full % 2**32
    via = O.box_sums_integral(sats, 8, 1, 293, 293)
    direct = O.box_sums_direct(x, y, 8, 1)
    for u, v in zip(direct, via):
        np.testing.assert_array_equal(u, v)


def test_box_stats_match_numpy_var():
    x = _rand_u8((30, 30), 13)
    y = _rand_u8((30, 30), 14)
    mu_x, mu_y, sxx, syy, sxy = O.box_stats(O.box_sums_direct(x, y, 8, 1), 8)
    for (i, j) in [(0, 0), (5, 17), (22, 22)]:
        wx = x[i:i + 8, j:j + 8].astype(np.float64).ravel()
        wy = y[i:i + 8, j:j + 8].astype(np.float64).ravel()
        assert abs(mu_x[i, j] - wx.mean()) < 1e-12
        assert abs(sxx[i, j] - wx.var()) < 1e-10
        assert abs(syy[i, j] - wy.var()) < 1e-10
        assert abs(sxy[i, j] - np.cov(wx, wy, ddof=0)[0, 1]) < 1e-10


# ---------------------------------------------------------------- stride / padding
@pytest.mark.parametrize("window,k,s", [("gaussian", 11, 4), ("box", 8, 4), ("gaussian", 11, 3)])
def test_stride_is_subsample_of_stride_one(window, k, s):
    x = _rand_u8((50, 61), 15)
    y = _rand_u8((50, 61), 16)
    full = O.ssim_map(x, y, O.SSIMParams(window=window, k=k))["map"]
    st = O.ssim_map(x, y, O.SSIMParams(window=window, k=k, stride=s))["map"]
    np.testing.assert_allclose(st, full[::s, ::s], rtol=0, atol=1e-14)


def test_padding_modes():
    x = _rand_u8((20, 26), 17)
    assert O.pad_image(x, 11, "reflect").shape == (30, 36)
    np.testing.assert_array_equal(O.pad_image(x, 11, "reflect")[:5, 5:-5], x[4::-1])
    np.testing.assert_array_equal(O.pad_image(x, 8, "zero")[:3], 0)
    for mode in ("zero", "reflect"):
        y = _rand_u8((20, 26), 18)
        p = O.SSIMParams(padding=mode)
        m = O.ssim_map(x, y, p)["map"]
        assert m.shape == x.shape
        # interior positions see no padding and equal the valid map
        v = O.ssim_map(x, y, O.SSIMParams())["map"]
        np.testing.assert_allclose(m[5:5 + v.shape[0], 5:5 + v.shape[1]], v, atol=1e-14)


def test_map_shape():
    assert O.map_shape(256, 256, 11, 1, "valid") == (246, 246)
    assert O.map_shape(1080, 1920, 11, 4, "valid") == (268, 478)
    assert O.map_shape(1080, 1920, 8, 4, "valid") == (269, 479)
    assert O.map_shape(1080, 1920, 8, 1, "valid") == (1073, 1913)
    assert O.map_shape(10, 10, 11, 1, "valid") == (0, 0)
    assert O.map_shape(10, 10, 11, 1, "zero") == (10, 10)


# ---------------------------------------------------------------- MS-SSIM
def test_pyramid_exact_quarter_multiples_and_mean_preserving():
    x = _rand_u8((67, 90), 19).astype(np.float64)
    lv = O.pyramid(x, 5)
    assert [a.shape for a in lv] == [(67, 90), (33, 45), (16, 22), (8, 11), (4, 5)]
    for j, a in enumerate(lv):
        scaled = a * 4**j
        np.testing.assert_array_equal(scaled, np.rint(scaled))
    np.testing.assert_allclose(lv[1].sum() * 4, x[:66, :90].sum())
    np.testing.assert_array_equal(O.downsample2x2(np.full((7, 9), 3.0)), 3.0)


def test_renormalised_three_scale_weights():
    w = np.array(O.MS_WEIGHTS[:3]) / sum(O.MS_WEIGHTS[:3])
    np.testing.assert_allclose(w, [0.071055, 0.452974, 0.475971], atol=1e-6)


def test_msssim_pins():
    x = _rand_u8((96, 96), 20)
    y = _rand_u8((96, 96), 21)
    p = O.SSIMParams()
    # one scale is plain SSIM with exponent 1
    one = O.msssim(x, y, p, weights=(1.0,), n_scales=1)["score"]
    assert abs(one - O.ssim_pooled(x, y, p)) < 1e-15
    # identity
    assert abs(O.msssim(x, x, p, n_scales=3)["score"] - 1.0) < 1e-13
    # symmetry
    a = O.msssim(x, y, p, n_scales=3, cs_clamp=True)["score"]
    b = O.msssim(y, x, p, n_scales=3, cs_clamp=True)["score"]
    assert abs(a - b) < 1e-14
    # constant planes: every CS_j = 1, score = l^{w_M}
    xc = np.full((200, 200), 60, np.uint8)
    yc = np.full((200, 200), 90, np.uint8)
    r = O.msssim(xc, yc, p, n_scales=4, renorm=True)
    l = (2 * 60 * 90 + p.C1) / (60**2 + 90**2 + p.C1)
    wM = O.MS_WEIGHTS[3] / sum(O.MS_WEIGHTS[:4])
    assert abs(r["score"] - l**wM) < 1e-13
    assert all(abs(c - 1) < 1e-12 for c in r["cs"])


def test_msssim_negative_cs_nan_or_clamped():
    x = (((np.mgrid[0:120, 0:120][0] // 3) % 2) * 255).astype(np.uint8)
    y = (255 - x).astype(np.uint8)
    p = O.SSIMParams()
    r = O.msssim(x, y, p, n_scales=2)
    assert r["cs"][0] < 0 and math.isnan(r["score"])
    assert O.msssim(x, y, p, n_scales=2, cs_clamp=True)["score"] == 0.0


def _block2(a):
    """2x2 block means by reshaping (odd trailing row / column dropped)."""
    h, w = a.shape[0] // 2 * 2, a.shape[1] // 2 * 2
    return a[:h, :w].astype(np.float64).reshape(h // 2, 2, w // 2, 2).mean(axis=(1, 3))


def test_msssim_sum_aggregation_pins():
    """'Sum' aggregation: a convex combination of the product's per-scale
    terms with the exponents normalised to sum to one."""
    rng = np.random.default_rng(40)
    x = synth.smooth_field(rng, 90, 96, 20, 230)
    y = np.clip(x + rng.normal(0, 12, x.shape), 0, 255)
    p = O.SSIMParams()
    # one scale: plain mean SSIM
    assert abs(O.msssim(x, y, p, (0.7,), 1, aggregation="sum")["score"] - O.ssim_pooled(x, y, p)) < 1e-15
    # one-hot weights pick one scale's term: CS at the finest, S_M at the coarsest
    cs0 = O.ssim_map(x, y, p)["cs"].mean()
    assert abs(O.msssim(x, y, p, (2.0, 0.0, 0.0), 3, aggregation="sum")["score"] - cs0) < 1e-14
    x2, y2 = _block2(_block2(x)), _block2(_block2(y))
    s2 = O.ssim_pooled(x2, y2, p)
    assert abs(O.msssim(x, y, p, (0.0, 0.0, 5.0), 3, aggregation="sum")["score"] - s2) < 1e-14
    # weighted AM-GM: the product with the same normalised weights is never larger
    r_sum = O.msssim(x, y, p, n_scales=3, aggregation="sum")
    r_prod = O.msssim(x, y, p, n_scales=3, renorm=True)
    terms = r_sum["cs"] + [r_sum["s_M"]]
    assert min(terms) > 0 and max(terms) - min(terms) > 1e-3
    assert r_prod["score"] < r_sum["score"] - 1e-6
    assert min(terms) <= r_sum["score"] <= max(terms)
    # renorm has no effect on the sum; identity gives one
    assert O.msssim(x, y, p, n_scales=3, renorm=False, aggregation="sum")["score"] == r_sum["score"]
    assert abs(O.msssim(x, x, p, n_scales=3, aggregation="sum")["score"] - 1.0) < 1e-13


def test_msssim_sum_gradient_matches_fd():
    rng = np.random.default_rng(41)
    x = synth.smooth_field(rng, 64, 70, 16 / 255, 235 / 255)
    y = x + rng.normal(0, 0.05, x.shape)
    C1, C2 = O.constants(0.01, 0.03, 1.0)
    p = O.SSIMParams(C1=C1, C2=C2, k=7, sigma=1.0)
    g = O.msssim_backward(x, y, 1.0, p, n_scales=3, aggregation="sum")
    f = lambda yy: O.msssim(x, yy, p, n_scales=3, aggregation="sum")["score"]  # noqa: E731
    for idx in [(0, 0), (31, 40), (63, 69), (10, 50)]:
        assert abs(_fd(f, y, idx, 1e-5) - g[idx]) <= 1e-6 * abs(g).max(), idx


def test_msssim_coarse_separate_reading():
    """Coarsest term mean(l) * mean(cs) instead of mean(l * cs): the two differ
    by exactly the population covariance of the l and cs maps."""
    rng = np.random.default_rng(42)
    x = synth.smooth_field(rng, 80, 90, 20, 230)
    y = np.clip(0.7 * x + 40 + rng.normal(0, 10, x.shape), 0, 255)
    p = O.SSIMParams()
    r = O.ssim_map(x, y, p)
    cov = np.cov(r["l"].ravel(), r["cs"].ravel(), bias=True)[0, 1]
    assert abs(cov) > 1e-5
    d = O.msssim(x, y, p, (1.0,), 1)["score"]
    sep = O.msssim(x, y, p, (1.0,), 1, coarse_separate=True)["score"]
    assert abs((d - sep) - cov) < 1e-13
    # spatially constant luminance term: both readings agree
    xc = np.full((60, 60), 70.0)
    yc = np.full((60, 60), 90.0)
    assert abs(O.msssim(xc, yc, p, n_scales=2, renorm=True)["score"]
               - O.msssim(xc, yc, p, n_scales=2, renorm=True, coarse_separate=True)["score"]) < 1e-15
    assert abs(O.msssim(x, x, p, n_scales=3, coarse_separate=True)["score"] - 1.0) < 1e-13


def test_msssim_coarse_separate_gradient_matches_fd():
    rng = np.random.default_rng(43)
    x = synth.smooth_field(rng, 64, 70, 16 / 255, 235 / 255)
    y = x + rng.normal(0, 0.05, x.shape)
    C1, C2 = O.constants(0.01, 0.03, 1.0)
    p = O.SSIMParams(C1=C1, C2=C2, k=7, sigma=1.0)
    for agg in ("product", "sum"):
        g = O.msssim_backward(x, y, 1.0, p, n_scales=3, renorm=True, aggregation=agg, coarse_separate=True)
        f = lambda yy: O.msssim(x, yy, p, n_scales=3, renorm=True, aggregation=agg,  # noqa: E731
                                coarse_separate=True)["score"]
        for idx in [(0, 0), (31, 40), (63, 69), (10, 50)]:
            assert abs(_fd(f, y, idx, 1e-5) - g[idx]) <= 1e-6 * abs(g).max(), (agg, idx)


# ---------------------------------------------------------------- adjoint
def _fd(f, y, idx, h=1e-3):
    yp = y.copy()
    ym = y.copy()
    yp[idx] += h
    ym[idx] -= h
    return (f(yp) - f(ym)) / (2 * h)


@pytest.mark.parametrize("padding,stride,window,k", [("valid", 1, "gaussian", 11), ("zero", 2, "gaussian", 7),
                                                   ("reflect", 1, "gaussian", 5), ("valid", 3, "box", 4)])
def test_ssim_gradient_matches_fp64_central_differences(padding, stride, window, k):
    rng = np.random.default_rng(22)
    x = synth.smooth_field(rng, 28, 31, 16, 235)
    y = x + rng.normal(0, 8, x.shape)
    p = O.SSIMParams(window=window, k=k, padding=padding, stride=stride)
    g = O.ssim_pooled_backward(x, y, 1.0, p)
    f = lambda yy: O.ssim_pooled(x, yy, p)  # noqa: E731
    for idx in [(0, 0), (13, 17), (27, 30), (5, 29), (20, 3)]:
        num = _fd(f, y, idx)
        assert abs(num - g[idx]) <= 1e-7 * max(abs(g).max(), 1e-12), (idx, num, g[idx])


def test_ssim_map_gradient_with_random_upstream():
    rng = np.random.default_rng(23)
    x = synth.smooth_field(rng, 24, 24, 16, 235)
    y = x + rng.normal(0, 8, x.shape)
    p = O.SSIMParams()
    up = rng.normal(size=O.map_shape(24, 24, 11, 1, "valid"))
    g = O.ssim_map_backward(x, y, up, p)
    f = lambda yy: float((O.ssim_map(x, yy, p)["map"] * up).sum())  # noqa: E731
    for idx in [(0, 0), (12, 12), (23, 5)]:
        assert abs(_fd(f, y, idx) - g[idx]) <= 1e-7 * abs(g).max()


def test_msssim_gradient_matches_fd_and_vanishes_at_identity():
    rng = np.random.default_rng(24)
    x = synth.smooth_field(rng, 64, 70, 16 / 255, 235 / 255)
    y = x + rng.normal(0, 0.05, x.shape)
    C1, C2 = O.constants(0.01, 0.03, 1.0)
    p = O.SSIMParams(C1=C1, C2=C2, k=7, sigma=1.0)
    g = O.msssim_backward(x, y, 1.0, p, n_scales=3, renorm=True)
    f = lambda yy: O.msssim(x, yy, p, n_scales=3, renorm=True)["score"]  # noqa: E731
    for idx in [(0, 0), (31, 40), (63, 69), (10, 50)]:
        assert abs(_fd(f, y, idx, 1e-5) - g[idx]) <= 1e-6 * abs(g).max(), idx
    g0 = O.msssim_backward(x, x, 1.0, p, n_scales=3, renorm=True)
    assert np.abs(g0).max() < 1e-12
    g1 = O.ssim_pooled_backward(x, x, 1.0, p)
    assert np.abs(g1).max() < 1e-12


def test_rgb_luma():
    rgb = np.stack([np.full((4, 4), 0.3)] * 3)
    np.testing.assert_allclose(O.rgb_to_y_bt601(rgb), 0.3, atol=1e-15)
    assert abs(sum(O.BT601) - 1.0) < 1e-15
    np.testing.assert_allclose(O.y_grad_to_rgb_bt601(np.ones((2, 2)))[:, 0, 0], O.BT601)


def test_rgb_luma_pure_primaries():
    """BT.601 luma of the pure primaries (channel order R, G, B on the leading
    axis): red 0.299, green 0.587, blue 0.114 (Kr = 0.299, Kb = 0.114,
    Kg = 1 - Kr - Kb); a swap of any two channel weights fails here."""
    for c, want in enumerate((0.299, 0.587, 0.114)):
        rgb = np.zeros((3, 2, 3))
        rgb[c] = 1.0
        np.testing.assert_allclose(O.rgb_to_y_bt601(rgb), want, rtol=0, atol=1e-15)
    assert abs((1 - 0.299 - 0.114) - 0.587) < 1e-15
    # yellow = red + green, cyan = green + blue, magenta = red + blue
    for pair, want in (((0, 1), 0.886), ((1, 2), 0.701), ((0, 2), 0.413)):
        rgb = np.zeros((3, 1, 1))
        rgb[list(pair)] = 1.0
        assert abs(float(O.rgb_to_y_bt601(rgb)[0, 0]) - want) < 1e-15


def test_rgb_luma_gradient_is_the_adjoint():
    """<Y(rgb), g> = <rgb, Y^T g> for random planes: the gradient map is the
    transpose of the luma map (and channel c of it is w_c g)."""
    rng = np.random.default_rng(5)
    rgb = rng.normal(size=(3, 7, 9))
    g = rng.normal(size=(7, 9))
    lhs = float(np.sum(O.rgb_to_y_bt601(rgb) * g))
    rhs = float(np.sum(rgb * O.y_grad_to_rgb_bt601(g)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_msssim_product_one_hot_and_two_hot_weights():
    """Product aggregation with one-hot exponents gives exactly one scale's
    term, CS_j at scale j < M (j = 1, 2) or S_M at the coarsest, each
    recomputed from independently block-averaged planes; two non-zero
    exponents give CS_1^a S_M^b.  A scale/exponent mix-up fails here."""
    rng = np.random.default_rng(43)
    x = synth.smooth_field(rng, 100, 104, 20, 230)
    y = np.clip(0.9 * x + 10 + rng.normal(0, 12, x.shape), 0, 255)
    p = O.SSIMParams()
    x1, y1 = _block2(x), _block2(y)
    x2, y2 = _block2(x1), _block2(y1)
    cs0 = O.ssim_map(x, y, p)["cs"].mean()
    cs1 = O.ssim_map(x1, y1, p)["cs"].mean()
    s2 = O.ssim_pooled(x2, y2, p)
    assert min(abs(cs0 - cs1), abs(cs1 - s2), abs(cs0 - s2)) > 1e-3  # the three terms are distinct
    assert abs(O.msssim(x, y, p, (1.0, 0.0, 0.0), 3)["score"] - cs0) < 1e-14
    assert abs(O.msssim(x, y, p, (0.0, 1.0, 0.0), 3)["score"] - cs1) < 1e-14
    assert abs(O.msssim(x, y, p, (0.0, 0.0, 1.0), 3)["score"] - s2) < 1e-14
    a, b = 0.7, 1.9
    got = O.msssim(x, y, p, (a, 0.0, b), 3)["score"]
    assert abs(got - cs0 ** a * s2 ** b) < 1e-14
    got = O.msssim(x, y, p, (0.0, a, b), 3)["score"]
    assert abs(got - cs1 ** a * s2 ** b) < 1e-14


@pytest.mark.parametrize("padding,stride,window,k", [("valid", 1, "gaussian", 7), ("zero", 2, "gaussian", 5),
                                                   ("reflect", 3, "gaussian", 7), ("reflect", 1, "box", 4),
                                                   ("zero", 1, "box", 3)])
def test_adjoint_dot_product_over_the_whole_map(padding, stride, window, k):
    """<J dy, g> = <dy, J^T g> for random directions dy and random upstream maps
    g: J dy by FP64 central differences of the map, J^T g by the adjoint (the
    transposed window, the border fold and the per-pixel combine together)."""
    rng = np.random.default_rng(77)
    x = synth.smooth_field(rng, 29, 33, 20, 230)
    y = np.clip(x + rng.normal(0, 12, x.shape), 0, 255)
    C1, C2 = O.constants(0.01, 0.03, 255.0)
    p = O.SSIMParams(window=window, k=k, sigma=1.2, C1=C1, C2=C2, stride=stride, padding=padding)
    q0 = O.ssim_map(x, y, p)["map"]
    g = rng.normal(size=q0.shape)
    dy = rng.normal(size=y.shape)
    h = 1e-4
    jdy = (O.ssim_map(x, y + h * dy, p)["map"] - O.ssim_map(x, y - h * dy, p)["map"]) / (2 * h)
    lhs = float((jdy * g).sum())
    rhs = float((dy * O.ssim_map_backward(x, y, g, p)).sum())
    assert abs(lhs - rhs) <= 1e-7 * max(abs(lhs), 1e-12), (lhs, rhs)


def test_msssim_directional_derivative():
    rng = np.random.default_rng(78)
    x = synth.smooth_field(rng, 80, 72, 20, 230)
    y = np.clip(x + rng.normal(0, 10, x.shape), 0, 255)
    p = O.SSIMParams(k=7, sigma=1.0)
    dy = rng.normal(size=y.shape)
    h = 1e-4
    for agg, sep in (("product", False), ("sum", True)):
        f = lambda yy: O.msssim(x, yy, p, n_scales=3, renorm=True, aggregation=agg,  # noqa: E731
                                coarse_separate=sep)["score"]
        lhs = (f(y + h * dy) - f(y - h * dy)) / (2 * h)
        rhs = float((dy * O.msssim_backward(x, y, 1.0, p, n_scales=3, renorm=True, aggregation=agg,
                                            coarse_separate=sep)).sum())
        assert abs(lhs - rhs) <= 1e-7 * abs(lhs), (agg, lhs, rhs)
