"""GPU parity of SSIM-3D / MS-SSIM-3D (ssimx_ssim3d, ssimx_msssim3d) against
the FP64 oracle: element-wise maps and per-frame scores over several tiles
with ragged tails, split frame runs, every dtype, pitched clips, exact
identity and symmetry for 8-bit clips, and sampled windows of a 1080p clip."""
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


def _box(P, k, L=255.0):
    return P.SSIMConfig(window="box", k=k, L=L)


# (frames, H, W, k, kt): 150 x 100 frames are 3 x 6 tiles with ragged tails;
# 20 frames at kt 2 are split into several frame runs.
U8_CASES = [(12, 100, 150, 11, 3), (20, 100, 150, 11, 2), (9, 70, 90, 11, 1), (8, 60, 70, 7, 5),
            (6, 45, 140, 16, 4), (7, 33, 200, 13, 6), (5, 20, 20, 1, 3), (4, 16, 16, 16, 4)]


@pytest.mark.parametrize("T,H,W,k,kt", U8_CASES)
def test_ssim3d_u8_parity(P, dev, T, H, W, k, kt):
    x, y = synth.video_clip(T, H, W, stream=T + k)
    cfg = _box(P, k)
    s, m = P.ssim3d(to_dev(x, dev), to_dev(y, dev), kt, cfg, return_map=True)
    s, m = s.cpu().numpy(), m.cpu().numpy()
    r = O.ssim3d_map(x, y, oparams(cfg), kt)
    assert m.shape == r["map"].shape
    err = np.abs(m - r["map"]).max()
    assert err <= MAP_TOL, f"map error {err}"
    want = [O.mean_pool(r["map"][t]) for t in range(m.shape[0])]
    np.testing.assert_allclose(s, want, rtol=0, atol=SCORE_TOL)


def test_ssim3d_identity_and_symmetry_exact(P, dev):
    x, y = synth.video_clip(10, 90, 130, stream=3)
    xt, yt = to_dev(x, dev), to_dev(y, dev)
    cfg = _box(P, 11)
    s, m = P.ssim3d(xt, xt, 4, cfg, return_map=True)
    assert torch.all(m == 1.0) and torch.all(s == 1.0)
    _, a = P.ssim3d(xt, yt, 4, cfg, return_map=True)
    _, b = P.ssim3d(yt, xt, 4, cfg, return_map=True)
    assert torch.equal(a, b)
    # pooled-only call gives the same scores as the map call
    s1 = P.ssim3d(xt, yt, 4, cfg)
    s2, _ = P.ssim3d(xt, yt, 4, cfg, return_map=True)
    assert torch.equal(s1, s2)


def test_ssim3d_static_clip_and_kt1_match_2d(P, dev):
    x, y = synth.video_clip(1, 80, 120, stream=4)
    xs, ys = np.repeat(x, 6, axis=0), np.repeat(y, 6, axis=0)
    cfg = _box(P, 11)
    s3 = P.ssim3d(to_dev(xs, dev), to_dev(ys, dev), 3, cfg).cpu().numpy()
    s2 = P.ssim(to_dev(x, dev), to_dev(y, dev), cfg).cpu().numpy()
    np.testing.assert_allclose(s3, s2[0], rtol=0, atol=SCORE_TOL)
    xc, yc = synth.video_clip(5, 80, 120, stream=5)
    s3 = P.ssim3d(to_dev(xc, dev), to_dev(yc, dev), 1, cfg).cpu().numpy()
    s2 = P.ssim(to_dev(xc, dev), to_dev(yc, dev), cfg).cpu().numpy()
    np.testing.assert_allclose(s3, s2, rtol=0, atol=SCORE_TOL)


@pytest.mark.parametrize("dtype", ["f32", "u16", "bf16"])
def test_ssim3d_float_paths(P, dev, dtype):
    x, y = synth.video_clip(9, 75, 140, stream=6)
    kt, k = 3, 11
    if dtype == "f32":
        xa, ya = x.astype(np.float32) / 255, y.astype(np.float32) / 255
        cfg, xt, yt = _box(P, k, 1.0), to_dev(xa, dev), to_dev(ya, dev)
    elif dtype == "u16":
        xa, ya = x.astype(np.uint16) * 4 + 3, y.astype(np.uint16) * 4
        cfg, xt, yt = _box(P, k, 1023.0), to_dev(xa, dev), to_dev(ya, dev)
    else:
        xa = bf16_round(x.astype(np.float32) / 255)
        ya = bf16_round(y.astype(np.float32) / 255)
        cfg = _box(P, k, 1.0)
        xt = torch.from_numpy(xa).to(dev).to(torch.bfloat16)
        yt = torch.from_numpy(ya).to(dev).to(torch.bfloat16)
    s, m = P.ssim3d(xt, yt, kt, cfg, return_map=True)
    r = O.ssim3d_map(xa.astype(np.float64), ya.astype(np.float64), oparams(cfg), kt)
    err = np.abs(m.cpu().numpy() - r["map"]).max()
    assert err <= MAP_TOL, f"{dtype} map error {err}"
    np.testing.assert_allclose(s.cpu().numpy(), [O.mean_pool(r["map"][t]) for t in range(m.shape[0])], rtol=0,
                               atol=SCORE_TOL)


def test_ssim3d_pitched_clip(P, dev):
    x, y = synth.video_clip(7, 64, 100, stream=7)
    big_x = torch.zeros((7, 70, 130), dtype=torch.uint8, device=dev)
    big_y = torch.zeros((7, 70, 130), dtype=torch.uint8, device=dev)
    big_x[:, :64, :100] = to_dev(x, dev)
    big_y[:, :64, :100] = to_dev(y, dev)
    cfg = _box(P, 11)
    s, m = P.ssim3d(big_x[:, :64, :100], big_y[:, :64, :100], 3, cfg, return_map=True)
    r = O.ssim3d_map(x, y, oparams(cfg), 3)
    assert np.abs(m.cpu().numpy() - r["map"]).max() <= MAP_TOL
    # unequal row pitches of the two clips (the kernel derives the distorted
    # clip's offsets from the reference's)
    wide_y = torch.zeros((7, 66, 171), dtype=torch.uint8, device=dev)
    wide_y[:, :64, :100] = to_dev(y, dev)
    s2, m2 = P.ssim3d(big_x[:, :64, :100], wide_y[:, :64, :100], 3, cfg, return_map=True)
    assert torch.equal(m2, m) and torch.equal(s2, s)


@pytest.mark.parametrize("n_scales,aggregation", [(3, "product"), (2, "sum"), (1, "product")])
def test_msssim3d_parity(P, dev, n_scales, aggregation):
    x, y = synth.video_clip(8, 120, 150, stream=8)
    cfg = _box(P, 11)
    kt = 3
    w = P.MS_WEIGHTS if n_scales > 1 else (1.0,)
    s, cs = P.ms_ssim3d(to_dev(x, dev), to_dev(y, dev), kt, cfg, weights=w, n_scales=n_scales, renorm=True,
                        aggregation=aggregation, return_cs=True)
    s, cs = s.cpu().numpy(), cs.cpu().numpy()
    r = O.msssim3d(x, y, oparams(cfg), kt, w, n_scales, renorm=True, aggregation=aggregation)
    np.testing.assert_allclose(s, r["score"], rtol=0, atol=SCORE_TOL)
    np.testing.assert_allclose(cs[:, :-1], r["cs"], rtol=0, atol=SCORE_TOL)
    np.testing.assert_allclose(cs[:, -1], r["s_M"], rtol=0, atol=SCORE_TOL)
    one = P.ms_ssim3d(to_dev(x, dev), to_dev(x, dev), kt, cfg, weights=w, n_scales=n_scales, renorm=True)
    assert torch.all(torch.abs(one - 1.0) <= 1e-6)


def test_ssim3d_1080p_clip_sampled(P, dev):
    """The 64-frame 1080p clip of the benchmark at kt = 5: sampled boxes one at a
    time (a k x k x kt crop is a 1 x 1 x 1 map), two map frames in full, and
    every map frame's score against the mean of its own map."""
    x, y = synth.config1()
    T, H, W = x.shape
    k, kt = 11, 5
    cfg = _box(P, k)
    s, m = P.ssim3d(to_dev(x, dev), to_dev(y, dev), kt, cfg, return_map=True)
    torch.cuda.synchronize()
    s = s.cpu().numpy().astype(np.float64)
    m = m.cpu().numpy()
    to, ho, wo = m.shape
    assert (to, ho, wo) == (T - kt + 1, H - k + 1, W - k + 1)
    p = oparams(cfg)
    rng = np.random.default_rng(31)
    worst = 0.0
    for t, i, j in zip(rng.integers(0, to, 400), rng.integers(0, ho, 400), rng.integers(0, wo, 400)):
        want = O.ssim3d_map(x[t:t + kt, i:i + k, j:j + k], y[t:t + kt, i:i + k, j:j + k], p, kt)["map"][0, 0, 0]
        worst = max(worst, abs(float(m[t, i, j]) - want))
    assert worst <= MAP_TOL, f"sampled map error {worst}"
    for t in range(to):
        assert abs(s[t] - m[t].astype(np.float64).mean()) <= SCORE_TOL
    for t in (0, to - 1):
        ref = O.ssim3d_map(x[t:t + kt], y[t:t + kt], p, kt)["map"][0]
        assert np.abs(m[t] - ref).max() <= MAP_TOL


@pytest.mark.parametrize("kt,T,dtype", [(36, 38, "u8"), (3, 7, "u16")])
def test_msssim3d_float_pyramid_cases(P, dev, kt, T, dtype):
    """MS-SSIM-3D where the second scale is not kept as exact 8-bit block sums:
    kt too long for uint32 sums of 2x2 sums, and 10-bit clips."""
    x, y = synth.video_clip(T, 64, 80, stream=9)
    cfg = _box(P, 11)
    if dtype == "u16":
        x, y = x.astype(np.uint16) * 4 + 1, y.astype(np.uint16) * 4
        cfg = _box(P, 11, 1023.0)
    s, cs = P.ms_ssim3d(to_dev(x, dev), to_dev(y, dev), kt, cfg, n_scales=2, renorm=True, return_cs=True)
    r = O.msssim3d(x, y, oparams(cfg), kt, P.MS_WEIGHTS, 2, renorm=True)
    np.testing.assert_allclose(s.cpu().numpy(), r["score"], rtol=0, atol=SCORE_TOL)
    np.testing.assert_allclose(cs.cpu().numpy()[:, 0], r["cs"][:, 0], rtol=0, atol=SCORE_TOL)


@pytest.mark.parametrize("T,H,W,k,kt", [(5, 11, 11, 11, 5), (64, 24, 70, 3, 64), (3, 40, 64, 11, 1),
                                        (70, 30, 300, 11, 2)])
def test_ssim3d_edge_shapes(P, dev, T, H, W, k, kt):
    """One-position maps, a single map frame, kt at its limit, many frame runs."""
    x, y = synth.video_clip(T, H, W, stream=10 + T)
    cfg = _box(P, k)
    s, m = P.ssim3d(to_dev(x, dev), to_dev(y, dev), kt, cfg, return_map=True)
    r = O.ssim3d_map(x, y, oparams(cfg), kt)
    assert np.abs(m.cpu().numpy() - r["map"]).max() <= MAP_TOL
    np.testing.assert_allclose(s.cpu().numpy(), [O.mean_pool(r["map"][t]) for t in range(m.shape[0])], rtol=0,
                               atol=SCORE_TOL)


def test_msssim3d_bf16_clip(P, dev):
    x, y = synth.video_clip(6, 100, 120, stream=12)
    xa = bf16_round(x.astype(np.float32) / 255)
    ya = bf16_round(y.astype(np.float32) / 255)
    cfg = _box(P, 11, 1.0)
    xt = torch.from_numpy(xa).to(dev).to(torch.bfloat16)
    yt = torch.from_numpy(ya).to(dev).to(torch.bfloat16)
    s = P.ms_ssim3d(xt, yt, 3, cfg, n_scales=3, renorm=True).cpu().numpy()
    r = O.msssim3d(xa, ya, oparams(cfg), 3, P.MS_WEIGHTS, 3, renorm=True)
    np.testing.assert_allclose(s, r["score"], rtol=0, atol=SCORE_TOL)


def test_msssim3d_coarse_separate(P, dev):
    x, y = synth.video_clip(7, 96, 120, stream=13)
    cfg = _box(P, 11)
    s = P.ms_ssim3d(to_dev(x, dev), to_dev(y, dev), 3, cfg, n_scales=2, renorm=True,
                    coarse_separate=True).cpu().numpy()
    r = O.msssim3d(x, y, oparams(cfg), 3, P.MS_WEIGHTS, 2, renorm=True, coarse_separate=True)
    np.testing.assert_allclose(s, r["score"], rtol=0, atol=SCORE_TOL)
