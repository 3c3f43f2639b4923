"""GPU parity of the forward path (ssim_map / ssim_pooled / msssim / box sums /
integral images) against the FP64 oracle, through the C-ABI."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _helpers import MAP_TOL, SCORE_TOL, bf16_round, device, oparams, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2101_06354_amd as P
    return P


@pytest.fixture(scope="module")
def dev():
    return device()


def _gpu_map(P, x, y, cfg, dev):
    s, m = P.ssim(to_dev(x, dev), to_dev(y, dev), cfg, return_map=True)
    torch.cuda.synchronize()
    return s.cpu().numpy().astype(np.float64), m.cpu().numpy().astype(np.float64)


def _check_map(P, x, y, cfg, dev, xo=None, yo=None, tol=MAP_TOL):
    s, m = _gpu_map(P, x, y, cfg, dev)
    ref = O.ssim_map(x if xo is None else xo, y if yo is None else yo, oparams(cfg))["map"]
    assert m.shape[1:] == ref.shape
    err = np.abs(m[0] - ref).max()
    assert err <= tol, f"map error {err}"
    serr = abs(s[0] - O.mean_pool(ref))
    assert serr <= SCORE_TOL, f"score error {serr}"
    return m[0], ref


def test_config0_gaussian_parity(P, dev):
    x, y = synth.config0()
    cfg = P.SSIMConfig()
    m, ref = _check_map(P, x, y, cfg, dev)
    assert m.shape == (246, 246)


@pytest.mark.parametrize("case", sorted(synth.stress_pairs().keys()))
@pytest.mark.parametrize("window,k,stride", [("gaussian", 11, 1), ("gaussian", 11, 4), ("box", 8, 1), ("box", 8, 4),
                                             ("gaussian", 7, 3)])
def test_stress_parity(P, dev, case, window, k, stride):
    x, y = synth.stress_pairs()[case]
    sig = 1.5 if k == 11 else 1.0
    _check_map(P, x, y, P.SSIMConfig(window=window, k=k, sigma=sig, stride=stride), dev)


@pytest.mark.parametrize("padding", ["zero", "reflect"])
@pytest.mark.parametrize("window,k,stride", [("gaussian", 11, 1), ("box", 8, 1), ("gaussian", 5, 2), ("box", 3, 3)])
def test_padding_parity(P, dev, padding, window, k, stride):
    rng = np.random.default_rng(3)
    x = synth.smooth_field(rng, 61, 77, 16, 235).round().astype(np.uint8)
    y = np.clip(x + rng.normal(0, 12, x.shape).round(), 0, 255).astype(np.uint8)
    sig = 1.5 if k == 11 else 1.0
    m, ref = _check_map(P, x, y, P.SSIMConfig(window=window, k=k, sigma=sig, stride=stride, padding=padding), dev)
    if stride == 1:
        assert m.shape == x.shape


@pytest.mark.parametrize("h,w", [(11, 11), (11, 12), (12, 11), (45, 300), (300, 45), (129, 257)])
def test_ragged_and_minimal_sizes(P, dev, h, w):
    rng = np.random.default_rng(h * 1000 + w)
    x = rng.integers(0, 256, (h, w)).astype(np.uint8)
    y = rng.integers(0, 256, (h, w)).astype(np.uint8)
    for window, k in (("gaussian", 11), ("box", 8)):
        _check_map(P, x, y, P.SSIMConfig(window=window, k=k), dev)


def test_identity_exact_and_bitwise_symmetry(P, dev):
    x, y = synth.config0()
    for cfg in (P.SSIMConfig(), P.SSIMConfig(window="box", k=8), P.SSIMConfig(stride=4, padding="reflect")):
        _, mxx = _gpu_map(P, x, x, cfg, dev)
        assert np.all(mxx == 1.0)
        _, mxy = _gpu_map(P, x, y, cfg, dev)
        _, myx = _gpu_map(P, y, x, cfg, dev)
        np.testing.assert_array_equal(mxy, myx)
        assert np.all(np.abs(mxy) <= 1.0)


def test_u16_ten_bit(P, dev):
    x, y = synth.config2(frames=1, h=150, w=203)
    cfg = P.SSIMConfig(L=1023.0)
    _check_map(P, x[0], y[0], cfg, dev)
    _check_map(P, x[0], y[0], P.SSIMConfig(L=1023.0, window="box", k=8), dev)


def test_float32_and_bf16_planes(P, dev):
    r, d = synth.config4(batch=1, h=96, w=120)
    x, y = r[0, 1], d[0, 1]
    cfg = P.SSIMConfig(L=1.0)
    _check_map(P, x, y, cfg, dev)
    _check_map(P, x, y, P.SSIMConfig(L=1.0, window="box", k=8), dev)
    xb, yb = bf16_round(x), bf16_round(y)
    s, m = P.ssim(to_dev(x, dev).bfloat16(), to_dev(y, dev).bfloat16(), cfg, return_map=True)
    ref = O.ssim_map(xb, yb, oparams(cfg))["map"]
    assert np.abs(m[0].cpu().numpy() - ref).max() <= MAP_TOL
    assert abs(float(s[0]) - O.mean_pool(ref)) <= SCORE_TOL


def test_batch_with_pitch_and_frame_stride(P, dev):
    rng = np.random.default_rng(5)
    big = rng.integers(0, 256, (3, 70, 100)).astype(np.uint8)
    big2 = np.clip(big + rng.integers(-20, 21, big.shape), 0, 255).astype(np.uint8)
    xt, yt = to_dev(big, dev)[:, 3:63, 5:90], to_dev(big2, dev)[:, 3:63, 5:90]
    cfg = P.SSIMConfig()
    s, m = P.ssim(xt, yt, cfg, return_map=True)
    for f in range(3):
        ref = O.ssim_map(big[f, 3:63, 5:90], big2[f, 3:63, 5:90], oparams(cfg))["map"]
        assert np.abs(m[f].cpu().numpy() - ref).max() <= MAP_TOL
        assert abs(float(s[f]) - O.mean_pool(ref)) <= SCORE_TOL


@pytest.mark.parametrize("k,stride", [(8, 1), (8, 4), (11, 1), (3, 2)])
@pytest.mark.parametrize("algo", ["separable", "integral"])
def test_box_sums_bit_exact(P, dev, k, stride, algo):
    rng = np.random.default_rng(7)
    x = rng.integers(0, 256, (2, 53, 71)).astype(np.uint8)
    y = rng.integers(0, 256, (2, 53, 71)).astype(np.uint8)
    got = P.box_sums(to_dev(x, dev), to_dev(y, dev), k, stride, algo).cpu().numpy()
    for f in range(2):
        want = O.box_sums_direct(x[f], y[f], k, stride)
        for q in range(5):
            np.testing.assert_array_equal(got[q, f], want[q])


def test_integral_images_bit_exact_with_wraparound(P, dev):
    rng = np.random.default_rng(8)
    x = rng.integers(200, 256, (1, 300, 311)).astype(np.uint8)   # sum x^2 over the frame > 2^32
    y = rng.integers(0, 256, (1, 300, 311)).astype(np.uint8)
    got = P.integral_images(to_dev(x, dev), to_dev(y, dev)).cpu().numpy().view(np.uint32)
    want = O.integral_images(x[0], y[0])
    assert int(want[2][-1, -1]) != int(np.sum(x.astype(np.int64) ** 2))  # wrapped
    for q in range(5):
        np.testing.assert_array_equal(got[q, 0], want[q])


@pytest.mark.parametrize("algo", ["separable", "integral"])
@pytest.mark.parametrize("stride", [1, 4])
def test_box_window_ssim_both_algorithms(P, dev, algo, stride):
    x, y = synth.config1(frames=1, h=120, w=200)
    _check_map(P, x[0], y[0], P.SSIMConfig(window="box", k=8, stride=stride, algo=algo), dev)


def test_u16_box_sums_integral(P, dev):
    x, y = synth.config2(frames=1, h=64, w=80)
    got = P.box_sums(to_dev(x, dev), to_dev(y, dev), 8, 1, "integral").cpu().numpy()
    want = O.box_sums_direct(x[0], y[0], 8, 1)
    for q in range(5):
        np.testing.assert_array_equal(got[q, 0], want[q])


@pytest.mark.parametrize("n_scales,renorm", [(5, False), (3, True), (1, False)])
def test_msssim_u16_parity(P, dev, n_scales, renorm):
    x, y = synth.config2(frames=2, h=270, w=480)
    cfg = P.SSIMConfig(L=1023.0)
    w = P.MS_WEIGHTS if n_scales > 1 else (1.0,)
    s, cs = P.ms_ssim(to_dev(x, dev), to_dev(y, dev), cfg, weights=w, n_scales=n_scales, renorm=renorm,
                      return_cs=True)
    s, cs = s.cpu().numpy(), cs.cpu().numpy()
    for f in range(2):
        r = O.msssim(x[f], y[f], oparams(cfg), w, n_scales, renorm)
        assert abs(s[f] - r["score"]) <= SCORE_TOL
        np.testing.assert_allclose(cs[f, :-1], r["cs"], rtol=0, atol=SCORE_TOL)
        assert abs(cs[f, -1] - r["s_M"]) <= SCORE_TOL


def test_msssim_float_rgb_luma_planes(P, dev):
    r, d = synth.config4(batch=2, h=128, w=160)
    x = (0.299 * r[:, 0] + 0.587 * r[:, 1] + 0.114 * r[:, 2]).astype(np.float32)
    y = (0.299 * d[:, 0] + 0.587 * d[:, 1] + 0.114 * d[:, 2]).astype(np.float32)
    cfg = P.SSIMConfig(L=1.0)
    s = P.ms_ssim(to_dev(x, dev), to_dev(y, dev), cfg, n_scales=3, renorm=True).cpu().numpy()
    for f in range(2):
        assert abs(s[f] - O.msssim(x[f], y[f], oparams(cfg), n_scales=3, renorm=True)["score"]) <= SCORE_TOL


@pytest.mark.parametrize("n_scales", [5, 3])
def test_msssim_sum_aggregation(P, dev, n_scales):
    x, y = synth.config2(frames=2, h=270, w=480)
    cfg = P.SSIMConfig(L=1023.0)
    s, cs = P.ms_ssim(to_dev(x, dev), to_dev(y, dev), cfg, n_scales=n_scales, aggregation="sum", return_cs=True)
    s, cs = s.cpu().numpy(), cs.cpu().numpy()
    for f in range(2):
        r = O.msssim(x[f], y[f], oparams(cfg), P.MS_WEIGHTS, n_scales, aggregation="sum")
        assert abs(s[f] - r["score"]) <= SCORE_TOL
        np.testing.assert_allclose(cs[f, :-1], r["cs"], rtol=0, atol=SCORE_TOL)
    # same per-scale terms as the product; identity gives exactly one
    _, cs_p = P.ms_ssim(to_dev(x, dev), to_dev(y, dev), cfg, n_scales=n_scales, return_cs=True)
    assert torch.equal(cs_p.cpu(), torch.from_numpy(cs))
    xi = to_dev(x, dev)
    one = P.ms_ssim(xi, xi, cfg, n_scales=n_scales, aggregation="sum").cpu().numpy()
    assert np.all(np.abs(one - 1.0) <= 1e-6)
    with pytest.raises(ValueError):
        P.ms_ssim(xi, xi, cfg, aggregation="mean")


def test_msssim_identity_and_clamp(P, dev):
    x, _ = synth.config0()
    cfg = P.SSIMConfig()
    s = P.ms_ssim(to_dev(x, dev), to_dev(x, dev), cfg, n_scales=4, renorm=True)
    assert float(s[0]) == 1.0
    xx = (((np.mgrid[0:120, 0:120][0] // 3) % 2) * 255).astype(np.uint8)
    yy = (255 - xx).astype(np.uint8)
    s = P.ms_ssim(to_dev(xx, dev), to_dev(yy, dev), cfg, n_scales=2)
    assert np.isnan(float(s[0]))
    s = P.ms_ssim(to_dev(xx, dev), to_dev(yy, dev), cfg, n_scales=2, cs_clamp=True)
    assert float(s[0]) == 0.0


def test_deterministic(P, dev):
    x, y = synth.config1(frames=2, h=200, w=300)
    xt, yt = to_dev(x, dev), to_dev(y, dev)
    a = P.ssim(xt, yt, P.SSIMConfig(), return_map=True)
    b = P.ssim(xt, yt, P.SSIMConfig(), return_map=True)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


@pytest.mark.parametrize("k,sigma", [(7, 1.0), (9, 1.5), (13, 2.0), (11, 1.5)])
@pytest.mark.parametrize("padding", ["valid", "reflect", "zero"])
@pytest.mark.parametrize("h,w", [(150, 203), (45, 64), (300, 77)])
def test_stride1_band_kernel_window_sizes(P, dev, k, sigma, padding, h, w):
    rng = np.random.default_rng(k * 7 + h)
    x = synth.smooth_field(rng, h, w, 16, 235).round().astype(np.uint8)
    y = np.clip(x + rng.normal(0, 15, x.shape).round(), 0, 255).astype(np.uint8)
    _check_map(P, x, y, P.SSIMConfig(k=k, sigma=sigma, padding=padding), dev)


def test_tile_configs_agree_and_unaligned_planes(P, dev):
    x, y = synth.config1(frames=2, h=333, w=501)
    xt, yt = to_dev(x, dev), to_dev(y, dev)
    cfg = P.SSIMConfig()
    maps, scores = [], []
    try:
        for t in range(P.num_tile_configs()):
            P.set_tile_override(t)
            s, m = P.ssim(xt, yt, cfg, return_map=True)
            maps.append(m)
            scores.append(s)
    finally:
        P.set_tile_override(-1)
    for m in maps[1:]:
        assert torch.equal(m, maps[0])
    for s in scores[1:]:
        assert torch.allclose(s, scores[0], rtol=0, atol=2e-7)
    # the same frames at an odd byte offset (no vector loads) give the same map
    bx = torch.zeros((2, 333, 503), dtype=torch.uint8, device=dev)
    by = torch.zeros_like(bx)
    bx[:, :, 1:502] = xt
    by[:, :, 1:502] = yt
    s2, m2 = P.ssim(bx[:, :, 1:502], by[:, :, 1:502], cfg, return_map=True)
    assert torch.equal(m2, maps[0])
    for f in range(2):
        ref = O.ssim_map(x[f], y[f], oparams(cfg))["map"]
        assert np.abs(maps[0][f].cpu().numpy() - ref).max() <= MAP_TOL


def test_row_pitch_beyond_vector_offsets(P, dev):
    """Rows 2^24 + 64 elements apart (beyond the 32-bit in-chunk offsets of
    the vector loads) take the element-wise loads: the map equals the one of
    the same frames stored densely, and the oracle's."""
    x, y = synth.config1(frames=1, h=24, w=150)
    xt, yt = to_dev(x, dev), to_dev(y, dev)
    cfg = P.SSIMConfig()
    s, m = P.ssim(xt, yt, cfg, return_map=True)
    pitch = (1 << 24) + 64
    bx = torch.zeros((24 * pitch,), dtype=torch.uint8, device=dev)
    by = torch.zeros_like(bx)
    vx = bx.as_strided((1, 24, 150), (24 * pitch, pitch, 1))
    vy = by.as_strided((1, 24, 150), (24 * pitch, pitch, 1))
    vx.copy_(xt)
    vy.copy_(yt)
    s2, m2 = P.ssim(vx, vy, cfg, return_map=True)
    assert torch.equal(m2, m) and torch.equal(s2, s)
    ref = O.ssim_map(x[0], y[0], oparams(cfg))["map"]
    assert np.abs(m2[0].cpu().numpy() - ref).max() <= MAP_TOL
    del bx, by, vx, vy


@pytest.mark.parametrize("dtype", ["u16", "f32", "bf16"])
def test_band_kernel_other_dtypes(P, dev, dtype):
    if dtype == "u16":
        x, y = synth.config2(frames=1, h=200, w=300)
        x, y, L = x[0], y[0], 1023.0
        xo, yo = x, y
        xt, yt = to_dev(x, dev), to_dev(y, dev)
    else:
        r, d = synth.config4(batch=1, h=200, w=300)
        x, y, L = r[0, 0], d[0, 0], 1.0
        xt, yt = to_dev(x, dev), to_dev(y, dev)
        xo, yo = x, y
        if dtype == "bf16":
            xt, yt = xt.bfloat16(), yt.bfloat16()
            xo, yo = bf16_round(x), bf16_round(y)
    cfg = P.SSIMConfig(L=L)
    s, m = P.ssim(xt, yt, cfg, return_map=True)
    ref = O.ssim_map(xo, yo, oparams(cfg))["map"]
    assert np.abs(m[0].cpu().numpy() - ref).max() <= MAP_TOL
    assert abs(float(s[0]) - O.mean_pool(ref)) <= SCORE_TOL


# 8-bit rectangular windows with valid borders run on the band kernel for these
# window/stride pairs (the others on the generic tile kernel).
BAND_CASES = [(k, 1) for k in range(2, 17)] + [(k, 2) for k in (2, 4, 6, 8, 16)] + [(k, 4) for k in (4, 8, 12, 16)]


def _band_frames(k, stride, h, w):
    rng = np.random.default_rng(1000 + 17 * k + stride)
    x = np.empty((2, h, w), np.uint8)
    y = np.empty((2, h, w), np.uint8)
    for f in range(2):
        x[f] = synth.smooth_field(rng, h, w, 16, 235).round().astype(np.uint8)
        y[f] = np.clip(x[f] + rng.normal(0, 14, (h, w)).round(), 0, 255).astype(np.uint8)
    # saturated patches: the largest window sums (x = 255, y = 0) and a 0/255 checkerboard
    x[0, :40, :70] = 255
    y[0, :40, :70] = 0
    yy, xx = np.mgrid[0:50, 0:90]
    x[1, -50:, -90:] = ((yy + xx) % 2) * 255
    y[1, -50:, -90:] = ((yy // 2 + xx // 3) % 2) * 255
    return x, y


@pytest.mark.parametrize("k,stride", BAND_CASES)
def test_box_band_kernel_windows_and_strides(P, dev, k, stride):
    # several 256-column tiles and row tiles, ragged tails, two frames
    h, w = (300, 600) if stride == 1 else (290, 1100)
    x, y = _band_frames(k, stride, h, w)
    cfg = P.SSIMConfig(window="box", k=k, stride=stride)
    s, m = P.ssim(to_dev(x, dev), to_dev(y, dev), cfg, return_map=True)
    s, m = s.cpu().numpy().astype(np.float64), m.cpu().numpy().astype(np.float64)
    for f in range(2):
        ref = O.ssim_map(x[f], y[f], oparams(cfg))["map"]
        assert m[f].shape == ref.shape
        err = np.abs(m[f] - ref).max()
        assert err <= MAP_TOL, f"frame {f} map error {err}"
        assert abs(s[f] - O.mean_pool(ref)) <= SCORE_TOL


@pytest.mark.parametrize("k,stride", [(2, 1), (5, 1), (8, 1), (16, 1), (6, 2), (8, 4), (16, 4)])
def test_box_band_identity_and_symmetry(P, dev, k, stride):
    x, y = _band_frames(k, stride, 270, 700)
    xt, yt = to_dev(x, dev), to_dev(y, dev)
    cfg = P.SSIMConfig(window="box", k=k, stride=stride)
    _, mxx = P.ssim(xt, xt, cfg, return_map=True)
    assert bool(torch.all(mxx == 1.0))
    _, mxy = P.ssim(xt, yt, cfg, return_map=True)
    _, myx = P.ssim(yt, xt, cfg, return_map=True)
    assert torch.equal(mxy, myx)
    assert bool(torch.all(mxy.abs() <= 1.0))


@pytest.mark.parametrize("stride", [1, 4])
def test_box_band_tile_configs_agree(P, dev, stride):
    x, y = synth.config1(frames=2, h=333, w=1100)
    xt, yt = to_dev(x, dev), to_dev(y, dev)
    cfg = P.SSIMConfig(window="box", k=8, stride=stride)
    maps, scores = [], []
    try:
        for t in range(P.num_tile_configs()):
            P.set_tile_override(t)
            s, m = P.ssim(xt, yt, cfg, return_map=True)
            maps.append(m)
            scores.append(s)
    finally:
        P.set_tile_override(-1)
    for m in maps[1:]:
        assert torch.equal(m, maps[0])
    for s in scores[1:]:
        assert torch.allclose(s, scores[0], rtol=0, atol=2e-7)
    # odd byte offset: the generic tile kernel takes the call; both match the oracle
    bx = torch.zeros((2, 333, 1102), dtype=torch.uint8, device=dev)
    by = torch.zeros_like(bx)
    bx[:, :, 1:1101] = xt
    by[:, :, 1:1101] = yt
    _, m2 = P.ssim(bx[:, :, 1:1101], by[:, :, 1:1101], cfg, return_map=True)
    for f in range(2):
        ref = O.ssim_map(x[f], y[f], oparams(cfg))["map"]
        assert np.abs(maps[0][f].cpu().numpy() - ref).max() <= MAP_TOL
        assert np.abs(m2[f].cpu().numpy() - ref).max() <= MAP_TOL


@pytest.mark.parametrize("dtype,h,w", [("u8", 70, 5000), ("u16", 45, 4700), ("u8", 37, 8300), ("u8", 333, 97)])
def test_integral_images_group_scan_shapes(P, dev, dtype, h, w):
    # row groups, several 64-lane waves per row, 16 columns per thread, and
    # the row/column-scan fallback beyond 8192 columns
    rng = np.random.default_rng(h + w)
    hi = 256 if dtype == "u8" else 1024
    npt = np.uint8 if dtype == "u8" else np.uint16
    x = rng.integers(0, hi, (2, h, w)).astype(npt)
    y = rng.integers(0, hi, (2, h, w)).astype(npt)
    got = P.integral_images(to_dev(x, dev), to_dev(y, dev)).cpu().numpy().view(np.uint32)
    for f in range(2):
        want = O.integral_images(x[f], y[f])
        for q in range(5):
            np.testing.assert_array_equal(got[q, f], want[q])


@pytest.mark.parametrize("k,stride", [(5, 1), (8, 1), (16, 1), (8, 2), (8, 4), (7, 3)])
def test_integral_image_ssim_windows(P, dev, k, stride):
    h, w = (300, 600) if stride < 4 else (290, 1100)
    x, y = _band_frames(k, 1, h, w)
    cfg = P.SSIMConfig(window="box", k=k, stride=stride, algo="integral")
    s, m = P.ssim(to_dev(x, dev), to_dev(y, dev), cfg, return_map=True)
    s, m = s.cpu().numpy().astype(np.float64), m.cpu().numpy().astype(np.float64)
    for f in range(2):
        ref = O.ssim_map(x[f], y[f], oparams(cfg))["map"]
        assert np.abs(m[f] - ref).max() <= MAP_TOL
        assert abs(s[f] - O.mean_pool(ref)) <= SCORE_TOL
    _, mxx = P.ssim(to_dev(x, dev), to_dev(x, dev), cfg, return_map=True)
    assert bool(torch.all(mxx == 1.0))


@pytest.mark.parametrize("k", [7, 9, 11, 13])
@pytest.mark.parametrize("stride", [2, 3, 4])
@pytest.mark.parametrize("padding", ["valid", "reflect", "zero"])
def test_strided_gaussian_kernel(P, dev, k, stride, padding):
    # several 64-column tiles and row tiles with ragged tails, two frames
    h, w = 300, 200 * stride + 37
    x, y = _band_frames(k, stride, h, w)
    cfg = P.SSIMConfig(k=k, sigma=1.5 if k == 11 else 0.8 + 0.1 * k, stride=stride, padding=padding)
    s, m = P.ssim(to_dev(x, dev), to_dev(y, dev), cfg, return_map=True)
    s, m = s.cpu().numpy().astype(np.float64), m.cpu().numpy().astype(np.float64)
    for f in range(2):
        ref = O.ssim_map(x[f], y[f], oparams(cfg))["map"]
        assert m[f].shape == ref.shape
        err = np.abs(m[f] - ref).max()
        assert err <= MAP_TOL, f"frame {f} map error {err}"
        assert abs(s[f] - O.mean_pool(ref)) <= SCORE_TOL


@pytest.mark.parametrize("dtype", ["u16", "f32", "bf16"])
def test_strided_gaussian_dtypes_identity_and_tiles(P, dev, dtype):
    if dtype == "u16":
        x, y = synth.config2(frames=2, h=260, w=530)
        xo, yo, L = x, y, 1023.0
        xt, yt = to_dev(x, dev), to_dev(y, dev)
    else:
        r, d = synth.config4(batch=2, h=260, w=530)
        x, y, L = r[:, 0], d[:, 0], 1.0
        xt, yt = to_dev(x, dev), to_dev(y, dev)
        xo, yo = x, y
        if dtype == "bf16":
            xt, yt = xt.bfloat16(), yt.bfloat16()
            xo, yo = bf16_round(x), bf16_round(y)
    cfg = P.SSIMConfig(L=L, stride=4)
    maps = []
    try:
        for t in range(P.num_tile_configs()):
            P.set_tile_override(t)
            s, m = P.ssim(xt, yt, cfg, return_map=True)
            maps.append(m)
    finally:
        P.set_tile_override(-1)
    for m in maps[1:]:
        assert torch.equal(m, maps[0])
    for f in range(2):
        ref = O.ssim_map(xo[f], yo[f], oparams(cfg))["map"]
        assert np.abs(maps[0][f].cpu().numpy() - ref).max() <= MAP_TOL
    _, mxx = P.ssim(xt, xt, cfg, return_map=True)
    assert bool(torch.all(mxx == 1.0))
    _, mxy = P.ssim(xt, yt, cfg, return_map=True)
    _, myx = P.ssim(yt, xt, cfg, return_map=True)
    assert torch.equal(mxy, myx)


@pytest.mark.parametrize("window,k,algo,n_scales,aggregation", [
    ("gaussian", 11, "auto", 3, "product"), ("gaussian", 11, "auto", 1, "product"),
    ("gaussian", 11, "auto", 4, "sum"), ("box", 8, "separable", 1, "product"),
    ("box", 8, "auto", 1, "product"), ("box", 8, "auto", 2, "product")])
def test_msssim_coarse_separate(P, dev, window, k, algo, n_scales, aggregation):
    """Coarsest term mean(l) * mean(cs): every forward kernel family's l mode."""
    x, y = synth.config1(frames=2, h=200, w=260)
    cfg = P.SSIMConfig(window=window, k=k, algo=algo)
    w = P.MS_WEIGHTS if n_scales > 1 else (1.0,)
    s, cs = P.ms_ssim(to_dev(x, dev), to_dev(y, dev), cfg, weights=w, n_scales=n_scales, renorm=True,
                      aggregation=aggregation, coarse_separate=True, return_cs=True)
    s, cs = s.cpu().numpy(), cs.cpu().numpy()
    for f in range(2):
        r = O.msssim(x[f], y[f], oparams(cfg), w, n_scales, True, aggregation=aggregation, coarse_separate=True)
        assert abs(s[f] - r["score"]) <= SCORE_TOL
        assert abs(cs[f, -1] - r["s_M"]) <= SCORE_TOL
    xi = to_dev(x, dev)
    one = P.ms_ssim(xi, xi, cfg, weights=w, n_scales=n_scales, renorm=True, coarse_separate=True).cpu().numpy()
    assert np.all(np.abs(one - 1.0) <= 1e-6)


@pytest.mark.parametrize("window,k,stride", [("gaussian", 11, 1), ("gaussian", 11, 4), ("box", 8, 1),
                                             ("gaussian", 5, 1), ("gaussian", 7, 2)])
def test_nan_and_inf_inputs_propagate(P, dev, window, k, stride):
    """A NaN or Inf input pixel makes exactly the map positions whose windows
    cover it non-finite (shared centring values must not leak it to other
    windows), and the pooled score NaN; MS-SSIM's score is NaN too."""
    r, d = synth.config4(batch=1, h=70, w=90)
    cfg = P.SSIMConfig(L=1.0, window=window, k=k, stride=stride, sigma=1.5 if k == 11 else 1.0)
    for bad, (pr, pc), which in ((np.nan, (33, 41), 0), (np.inf, (9, 70), 1), (-np.inf, (60, 5), 0)):
        x, y = r[0, 0].copy(), d[0, 0].copy()
        (x if which == 0 else y)[pr, pc] = bad
        s, m = P.ssim(to_dev(x, dev), to_dev(y, dev), cfg, return_map=True)
        m = m[0].cpu().numpy()
        ho, wo = m.shape
        ii = np.arange(ho)[:, None] * stride
        jj = np.arange(wo)[None, :] * stride
        cover = (ii <= pr) & (pr < ii + k) & (jj <= pc) & (pc < jj + k)
        assert cover.any()
        assert not np.isfinite(m[cover]).any(), (bad, np.isfinite(m[cover]).sum())
        assert np.isfinite(m[~cover]).all(), (bad, (~np.isfinite(m[~cover])).sum())
        assert np.isnan(float(s[0]))
    x = r[0, 0].copy()
    x[40, 40] = np.nan
    ms = P.ms_ssim(to_dev(x, dev), to_dev(d[0, 0], dev), P.SSIMConfig(L=1.0), n_scales=2, renorm=True)
    assert np.isnan(float(ms[0]))


@pytest.mark.parametrize("kind,h,w,n_scales,path", [
    ("u8", 270, 480, 5, "fused"), ("u8", 133, 201, 4, "fused"), ("u16", 271, 479, 5, "fused"),
    ("u16", 97, 131, 3, "fused"), ("u8", 133, 201, 4, "reflect"), ("u16", 150, 187, 3, "box"),
    ("u8", 131, 190, 3, "stride2")])
def test_msssim_pyramid_levels_bit_exact(P, dev, kind, h, w, n_scales, path):
    """The 2x2 levels msssim builds (read back from its workspace through
    ssimx_msssim_pyramid_layout) equal the oracle's pyramid bit for bit on
    integer planes, odd sizes floored: both from the windowed pass that writes
    the next scale (stride-1 Gaussian, valid borders) and from the separate
    down-sampling pass (other borders, windows and strides)."""
    if kind == "u8":
        x, y = synth.config1(frames=2, h=h, w=w)
        cfg = P.SSIMConfig()
    else:
        x, y = synth.config2(frames=2, h=h, w=w)
        cfg = P.SSIMConfig(L=1023.0)
    if path == "reflect":
        cfg = P.SSIMConfig(padding="reflect")
    elif path == "box":
        cfg = P.SSIMConfig(window="box", k=8, L=1023.0)
    elif path == "stride2":
        cfg = P.SSIMConfig(stride=2)
    score, levels = P.ms_ssim(to_dev(x, dev), to_dev(y, dev), cfg, n_scales=n_scales, renorm=True,
                              return_pyramid=True)
    assert len(levels) == n_scales - 1
    for f in range(2):
        px, py = O.pyramid(x[f], n_scales), O.pyramid(y[f], n_scales)
        for j, (lx, ly) in enumerate(levels, start=1):
            gx, gy = lx[f].cpu().numpy(), ly[f].cpu().numpy()
            assert gx.shape == (h >> j, w >> j) and px[j].shape == gx.shape
            # exact: the oracle's FP64 means are multiples of 4^-j with <= 20 significant bits
            assert np.array_equal(px[j].astype(np.float32).astype(np.float64), px[j])
            np.testing.assert_array_equal(gx.astype(np.float64), px[j])
            np.testing.assert_array_equal(gy.astype(np.float64), py[j])
        ms = O.msssim(x[f], y[f], oparams(cfg), n_scales=n_scales, renorm=True)["score"]
        assert abs(float(score[f]) - ms) <= SCORE_TOL


def test_msssim_pyramid_levels_float_planes(P, dev):
    """On float planes the windowed pass forms the next scale from the staged
    sums u = x + y and v = x - y ((u + v) / 8 over a block), which differs from
    the plain 2x2 mean by float32 rounding only: within 4 ulp of the level's
    magnitude, and the MS-SSIM score stays within the pooled tolerance."""
    r, d = synth.config4(batch=2, h=200, w=262)
    x, y = r[:, 0], d[:, 0]
    cfg = P.SSIMConfig(L=1.0)
    score, levels = P.ms_ssim(to_dev(x, dev), to_dev(y, dev), cfg, n_scales=3, renorm=True, return_pyramid=True)
    for f in range(2):
        px, py = O.pyramid(x[f].astype(np.float64), 3), O.pyramid(y[f].astype(np.float64), 3)
        for j, (lx, ly) in enumerate(levels, start=1):
            for got, want in ((lx[f], px[j]), (ly[f], py[j])):
                got = got.cpu().numpy().astype(np.float64)
                assert np.abs(got - want).max() <= 4 * np.finfo(np.float32).eps * np.abs(want).max()
        ms = O.msssim(x[f], y[f], oparams(cfg), n_scales=3, renorm=True)["score"]
        assert abs(float(score[f]) - ms) <= SCORE_TOL
