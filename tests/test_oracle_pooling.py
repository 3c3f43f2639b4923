"""Pins of the oracle's spatial pooling functions (Spatial and Temporal
Aggregation section) against closed forms, numpy's own statistics and brute
force on small maps."""
import itertools
import math

import numpy as np
import pytest

import oracle as O


def _map(seed, shape=(37, 53), lo=-0.2, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, shape)


def test_mean_is_the_baseline_pool():
    q = _map(0)
    assert O.pool_mean(q) == O.mean_pool(q)


@pytest.mark.parametrize("c", [0.3, 0.97, 1.0])
def test_constant_map_closed_forms(c):
    q = np.full((9, 7), c)
    assert O.pool_cov(q) == 0.0
    assert O.pool_md(q, 2, 1) == 0.0
    assert O.pool_minkowski(q, 4) == pytest.approx((1 - c) ** 4, abs=1e-15)
    assert O.pool_distortion_weighted(q, 2) == pytest.approx(c, abs=1e-15)
    assert O.pool_five_number(q) == pytest.approx(c, abs=1e-15)
    n, m = q.size, math.ceil(6 * q.size / 100)
    assert O.pool_percentile(q, 6, 4000) == pytest.approx((m * c / 4000 + (n - m) * c) / n, abs=1e-15)


def test_cov_of_a_two_valued_map():
    a, b = 0.9, 0.5
    q = np.array([a, b] * 50)
    # sigma = |a - b| / 2, mu = (a + b) / 2
    assert O.pool_cov(q) == pytest.approx(abs(a - b) / (a + b), rel=1e-14)


def test_cov_and_mean_deviation_against_numpy():
    q = _map(1)
    assert O.pool_cov(q) == pytest.approx(np.std(q) / np.mean(q), rel=1e-12)
    assert O.pool_md(q, 2, 1) == pytest.approx(np.std(q), rel=1e-12)
    assert O.pool_md(q, 2, 3) == pytest.approx(np.std(q) ** 3, rel=1e-12)
    d4 = np.mean(np.abs(q - q.mean()) ** 4) ** 0.25
    assert O.pool_md(q, 4, 1) == pytest.approx(d4, rel=1e-12)


def test_minkowski_order_one_is_one_minus_the_mean():
    q = _map(2)
    assert O.pool_minkowski(q, 1) == pytest.approx(1 - q.mean(), abs=1e-14)


def test_distortion_weighted_limits():
    q = _map(3, lo=0.0, hi=0.99)
    # p = 0: every weight is one -> the mean
    assert O.pool_distortion_weighted(q, 0) == pytest.approx(q.mean(), abs=1e-14)
    # weights (1 - Q)^p for p = 1 written out
    w = 1 - q
    assert O.pool_distortion_weighted(q, 1) == pytest.approx((w * q).sum() / w.sum(), rel=1e-13)
    # the weighted mean lies below the mean (low scores weigh more)
    assert O.pool_distortion_weighted(q, 2) < q.mean()


def test_five_number_summary_against_numpy_percentiles():
    for seed, shape in ((4, (37, 53)), (5, (1, 1)), (6, (2, 3)), (7, (4, 4))):
        q = _map(seed, shape)
        want = (q.min() + np.percentile(q, 25) + np.median(q) + np.percentile(q, 75) + q.max()) / 5
        assert O.pool_five_number(q) == pytest.approx(want, rel=1e-14, abs=1e-15)


def test_percentile_pooling_brute_force():
    q = _map(8, (5, 6))
    n = q.size
    for p_s, r_s in itertools.product((0.0, 6.0, 25.0, 50.0, 100.0), (1.0, 4.0, 4000.0)):
        m = math.ceil(p_s * n / 100)
        order = sorted(q.ravel().tolist())
        want = (sum(v / r_s for v in order[:m]) + sum(order[m:])) / n
        assert O.pool_percentile(q, p_s, r_s) == pytest.approx(want, rel=1e-13, abs=1e-15)
    # r_s = 1 leaves the map unchanged
    assert O.pool_percentile(q, 30, 1.0) == pytest.approx(q.mean(), abs=1e-15)


def test_scale_factor_rule():
    assert [O.scale_factor(h) for h in (1, 255, 256, 257, 512, 513, 1080, 2160)] == [1, 1, 1, 2, 2, 3, 5, 9]


def test_block_average_downsampling():
    a = np.arange(7 * 11, dtype=np.float64).reshape(7, 11)
    d = O.downsample_avg(a, 3)
    assert d.shape == (2, 3)
    assert d[1, 2] == a[3:6, 6:9].mean()
    # factor 2 is the pyramid's 2x2 average
    np.testing.assert_array_equal(O.downsample_avg(a, 2), O.downsample2x2(a))
    np.testing.assert_array_equal(O.downsample_avg(a, 1), a)
    # a constant plane stays constant at every factor
    assert np.all(O.downsample_avg(np.full((20, 30), 7.0), 4) == 7.0)


def test_enhanced_ssim_composition():
    rng = np.random.default_rng(9)
    x = rng.integers(0, 256, (300, 400)).astype(np.uint8)
    y = np.clip(x + rng.integers(-20, 21, x.shape), 0, 255).astype(np.uint8)
    # identical inputs: a map of ones, CoV 0
    assert O.enhanced_ssim(x, x) == 0.0
    # written out: factor 2 (H = 300), 11x11 box at stride 5, CoV pooling
    C1, C2 = O.constants(0.01, 0.03, 255.0)
    xs, ys = O.downsample_avg(x, 2), O.downsample_avg(y, 2)
    q = O.ssim_map(xs, ys, O.SSIMParams(window="box", k=11, C1=C1, C2=C2, stride=5))["map"]
    assert q.shape == ((150 - 11) // 5 + 1, (200 - 11) // 5 + 1)
    assert O.enhanced_ssim(x, y) == pytest.approx(np.std(q) / np.mean(q), rel=1e-12)


def test_ycbcr_transform_closed_forms():
    white = np.full((3, 2, 2), 255.0)
    ycc = O.rgb_to_ycbcr_bt709(white)
    assert np.allclose(ycc[0], 255.0) and np.allclose(ycc[1:], 0.0)  # Y weights sum to one: grey has no chroma
    red = np.zeros((3, 1, 1))
    red[0] = 100.0
    ycc = O.rgb_to_ycbcr_bt709(red)
    assert ycc[0, 0, 0] == pytest.approx(21.3)
    assert ycc[1, 0, 0] == pytest.approx(0.539 * (0 - 21.3))
    assert ycc[2, 0, 0] == pytest.approx(0.635 * (100 - 21.3))


def test_color_ssim_reductions():
    rng = np.random.default_rng(12)
    g = rng.uniform(20, 230, (40, 50))
    x = np.stack([g, g, g])
    y = np.clip(x + rng.normal(0, 8, x.shape), 0, 255)
    y_grey = np.stack([y[0], y[0], y[0]])
    p = O.SSIMParams()
    # grey inputs: zero chroma planes have SSIM 1 in both channels
    r = O.color_ssim(x, y_grey, p, alpha=0.125, beta=0.125)
    assert r["channels"][1] == 1.0 and r["channels"][2] == 1.0
    assert r["score"] == pytest.approx((O.ssim_pooled(g, y[0], p) + 0.25) / 1.25, rel=1e-14)
    # alpha = beta = 0 is SSIM of the luma plane
    r = O.color_ssim(x, y, p, alpha=0.0, beta=0.0)
    assert r["score"] == pytest.approx(O.ssim_pooled(O.rgb_to_ycbcr_bt709(x)[0], O.rgb_to_ycbcr_bt709(y)[0], p))
    # the 0.8 / 0.1 / 0.1 weights
    r = O.color_ssim(x, y, p)
    s = r["channels"]
    assert r["score"] == pytest.approx(0.8 * s[0] + 0.1 * s[1] + 0.1 * s[2], rel=1e-14)


# ---------------------------------------------------------------- temporal pooling
def _series(n, seed, lo=0.3, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, n)


def test_pythagorean_means_against_scipy_and_closed_forms():
    from scipy import stats
    s = _series(257, 50)
    assert abs(O.pool_geometric(s) - stats.gmean(s)) < 1e-14
    assert abs(O.pool_harmonic(s) - stats.hmean(s)) < 1e-14
    assert O.pool_mean(s) > O.pool_geometric(s) > O.pool_harmonic(s)
    a, b = 0.36, 0.81
    assert abs(O.pool_geometric(np.array([a, b])) - math.sqrt(a * b)) < 1e-15
    assert abs(O.pool_harmonic(np.array([a, b])) - 2 * a * b / (a + b)) < 1e-15
    c = np.full(9, 0.7)
    assert abs(O.pool_geometric(c) - 0.7) < 1e-15 and abs(O.pool_harmonic(c) - 0.7) < 1e-15
    assert O.pool_geometric(np.array([0.5, 0.0])) == 0.0 and O.pool_harmonic(np.array([0.5, 0.0])) == 0.0
    assert math.isnan(O.pool_geometric(np.array([0.5, -0.1])))


@pytest.mark.parametrize("n", [1, 2, 7, 100])
def test_median_against_numpy(n):
    s = _series(n, 51 + n)
    assert O.pool_median(s) == float(np.median(s))


def test_windowed_means_reduce_at_the_ends():
    from numpy.lib.stride_tricks import sliding_window_view
    from scipy import stats
    s = _series(60, 52)
    n = s.size
    for m in ("am", "gm", "hm"):
        assert abs(O.pool_windowed(s, 1, m) - s.mean()) < 1e-14
    assert O.pool_windowed(s, 1, "cov") == 0.0
    assert abs(O.pool_windowed(s, n, "am") - s.mean()) < 1e-14
    assert abs(O.pool_windowed(s, n, "gm") - stats.gmean(s)) < 1e-14
    assert abs(O.pool_windowed(s, n, "hm") - stats.hmean(s)) < 1e-14
    assert abs(O.pool_windowed(s, n, "cov") - s.std() / s.mean()) < 1e-13
    # brute force with library windows at an interior length
    win = sliding_window_view(s, 9)
    assert abs(O.pool_windowed(s, 9, "gm") - stats.gmean(win, axis=1).mean()) < 1e-14
    assert abs(O.pool_windowed(s, 9, "hm") - stats.hmean(win, axis=1).mean()) < 1e-14
    assert abs(O.pool_windowed(s, 9, "cov") - (win.std(axis=1) / win.mean(axis=1)).mean()) < 1e-13
    # windowed AM weights interior values more than the ends
    w = np.zeros(n)
    w[0] = 1.0
    assert abs(O.pool_windowed(w, 5, "am") - 1.0 / (5 * (n - 4))) < 1e-16
    with pytest.raises(ValueError):
        O.pool_windowed(s, n + 1, "am")


# Luminance-Weighted Pooling subsection
def test_lw_weight_shape():
    a_s, b_s = 40.0, 20.0
    mu = np.array([0.0, 39.999, 40.0, 45.0, 50.0, 59.999, 60.0, 255.0])
    w = O.lw_weights(mu, a_s, b_s)
    assert w[0] == 0 and w[1] == 0 and w[2] == 0        # below and at the lower limit
    assert w[4] == 0.5 and w[6] == 1 and w[7] == 1       # midpoint, upper limit and above
    assert np.all(np.diff(w) >= 0) and 0 < w[3] < w[4] < w[5] < 1
    # b_s = 0: a step at a_s
    assert list(O.lw_weights(np.array([9.9, 10.0, 10.1]), 10.0, 0.0)) == [0.0, 1.0, 1.0]


def test_lw_zero_limits_is_the_baseline():
    rng = np.random.default_rng(5)
    x = rng.integers(0, 256, (40, 48)).astype(np.uint8)
    y = np.clip(x.astype(int) + rng.integers(-20, 21, x.shape), 0, 255).astype(np.uint8)
    p = O.SSIMParams()
    assert O.pool_luminance_weighted(x, y, p, 0.0, 0.0) == pytest.approx(O.ssim_pooled(x, y, p), abs=1e-15)
    # a lower limit above every local mean weighs everything out
    assert O.pool_luminance_weighted(x, y, p, 300.0, 10.0) == 0.0


def test_lw_constant_reference_closed_form():
    rng = np.random.default_rng(6)
    x = np.full((30, 34), 120.0)
    y = x + rng.normal(0, 8, x.shape)
    p = O.SSIMParams()
    base = O.ssim_pooled(x, y, p)
    # mu1 = 120 everywhere: weight (120 - a_s) / b_s inside the ramp, 1 above it
    assert O.pool_luminance_weighted(x, y, p, 100.0, 40.0) == pytest.approx(0.5 * base, rel=1e-12)
    assert O.pool_luminance_weighted(x, y, p, 60.0, 40.0) == pytest.approx(base, rel=1e-12)


def test_lw_brute_force_direct_window():
    """Direct 2-D window sums on a tiny half-dark, half-bright pair, position by
    position, against the separable oracle."""
    rng = np.random.default_rng(7)
    h, w, k = 14, 18, 5
    x = np.where(np.arange(w)[None, :] < 8, 10.0, 180.0) + rng.integers(0, 6, (h, w))
    y = x + rng.integers(-9, 10, (h, w))
    p = O.SSIMParams(window="gaussian", k=k, sigma=1.5)
    g = O.window_2d("gaussian", k, 1.5)
    C1, C2 = p.C1, p.C2
    for a_s, b_s in [(60.0, 0.0), (30.0, 90.0), (100.0, 25.0)]:
        tot, n = 0.0, 0
        for i in range(h - k + 1):
            for j in range(w - k + 1):
                px, py = x[i:i + k, j:j + k], y[i:i + k, j:j + k]
                mx, my = (g * px).sum(), (g * py).sum()
                vx, vy = (g * (px - mx) ** 2).sum(), (g * (py - my) ** 2).sum()
                cxy = (g * (px - mx) * (py - my)).sum()
                q = (2 * mx * my + C1) * (2 * cxy + C2) / ((mx * mx + my * my + C1) * (vx + vy + C2))
                wt = 0.0 if mx < a_s else (1.0 if mx >= a_s + b_s else (mx - a_s) / b_s)
                tot += wt * q
                n += 1
        assert O.pool_luminance_weighted(x, y, p, a_s, b_s) == pytest.approx(tot / n, rel=1e-10, abs=1e-13)
