"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times: 64 x 1080p u8 frames (Gaussian 11x11, 8x8 box by tile sums and
by integral images, stride 4) with the pooled backward, and 32 x 4K 10-bit
frames with 5-scale MS-SSIM.  (The 256-pair ragged batch is in
test_gpu_batch.py, the 16 x 3 x 512^2 loss in test_gpu_backward.py.)

The oracle cannot redo a whole 64-frame batch in seconds, so it checks
  * sampled map positions one window at a time: a k x k crop of the planes is
    a 1 x 1 map;
  * two frames of each batch in full (map and pooled score);
  * every frame's pooled score against the mean of its own GPU map;
  * sampled gradient entries: the crop of rows / columns q-k+1 .. q+k-1 holds
    exactly the windows that cover pixel q, so the crop's adjoint with the
    full-frame upstream 1/(H_o W_o) gives the full-frame gradient at q.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _helpers import MAP_TOL, SCORE_TOL, device, oparams, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2101_06354_amd as P
    return P


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture(scope="module")
def c1(dev):
    x, y = synth.config1()
    return x, y, to_dev(x, dev), to_dev(y, dev)


C1_CASES = [("gaussian", 11, 1, "separable"), ("box", 8, 1, "separable"), ("box", 8, 1, "integral"),
            ("gaussian", 11, 4, "separable"), ("box", 8, 4, "separable")]


@pytest.mark.parametrize("window,k,stride,algo", C1_CASES)
def test_config1_full_batch(P, dev, c1, window, k, stride, algo):
    x, y, xt, yt = c1
    B = x.shape[0]
    cfg = P.SSIMConfig(window=window, k=k, stride=stride, algo=algo)
    s, m = P.ssim(xt, yt, cfg, return_map=True)
    torch.cuda.synchronize()
    s = s.cpu().numpy().astype(np.float64)
    m = m.cpu().numpy()
    p = oparams(cfg)
    ho, wo = m.shape[1:]
    assert (ho, wo) == O.map_shape(x.shape[1], x.shape[2], p.k, p.stride, p.padding)
    rng = np.random.default_rng(11 * k + stride)
    worst = 0.0
    for f in range(B):
        for i, j in zip(rng.integers(0, ho, 24), rng.integers(0, wo, 24)):
            r0, c0 = stride * i, stride * j
            want = O.ssim_map(x[f, r0:r0 + k, c0:c0 + k], y[f, r0:r0 + k, c0:c0 + k], p)["map"][0, 0]
            worst = max(worst, abs(float(m[f, i, j]) - want))
        # pooled score = mean of the frame's own map (fixed-order compensated sum)
        assert abs(s[f] - m[f].astype(np.float64).mean()) <= SCORE_TOL
    assert worst <= MAP_TOL, f"sampled map error {worst}"
    for f in (0, B - 1):
        ref = O.ssim_map(x[f], y[f], p)["map"]
        assert np.abs(m[f] - ref).max() <= MAP_TOL
        assert abs(s[f] - O.mean_pool(ref)) <= SCORE_TOL


def test_config1_full_batch_pooled_backward(P, dev, c1):
    x, y, xt, yt = c1
    B, H, W = x.shape
    cfg = P.SSIMConfig()
    g = P.ssim_backward(xt, yt, torch.ones(B, device=dev), cfg)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    p = oparams(cfg)
    k = cfg.k
    ho, wo = O.map_shape(H, W, p.k, p.stride, p.padding)
    rng = np.random.default_rng(5)
    got, want = [], []
    for f in range(0, B, 4):
        qs = list(zip(rng.integers(0, H, 12), rng.integers(0, W, 12))) + [(0, 0), (H - 1, W - 1), (5, W - 3)]
        for qy, qx in qs:
            r0, r1 = max(0, qy - k + 1), min(H, qy + k)
            c0, c1_ = max(0, qx - k + 1), min(W, qx + k)
            cx, cy = x[f, r0:r1, c0:c1_], y[f, r0:r1, c0:c1_]
            mh, mw = O.map_shape(r1 - r0, c1_ - c0, p.k, p.stride, p.padding)
            gm = np.full((mh, mw), 1.0 / (ho * wo))
            gc = O.ssim_map_backward(cx, cy, gm, p)
            got.append(float(g[f, qy, qx]))
            want.append(float(gc[qy - r0, qx - c0]))
    got, want = np.array(got), np.array(want)
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 1e-3 * scale
    assert np.linalg.norm(got - want) <= 1e-4 * np.linalg.norm(want)


def test_config2_full_batch_msssim(P, dev):
    x, y = synth.config2()
    B = x.shape[0]
    xt, yt = to_dev(x, dev), to_dev(y, dev)
    cfg = P.SSIMConfig(L=1023.0)
    s, cs = P.ms_ssim(xt, yt, cfg, return_cs=True)
    torch.cuda.synchronize()
    s, cs = s.cpu().numpy(), cs.cpu().numpy()
    p = oparams(cfg)
    for f in (0, B - 1):
        r = O.msssim(x[f], y[f], p, P.MS_WEIGHTS, 5, False)
        assert abs(s[f] - r["score"]) <= SCORE_TOL
        np.testing.assert_allclose(cs[f, :-1], r["cs"], rtol=0, atol=SCORE_TOL)
        assert abs(cs[f, -1] - r["s_M"]) <= SCORE_TOL
    # every frame of the batch matches its own single-frame call (a single
    # frame is cut into shorter tiles, which only regroups the pooled sums)
    for f in (1, 7, 16, B - 2):
        s1 = P.ms_ssim(xt[f:f + 1], yt[f:f + 1], cfg)
        assert abs(float(s1[0]) - float(s[f])) <= 2e-7


@pytest.mark.parametrize("window,k,stride", [("gaussian", 11, 1), ("box", 8, 1), ("gaussian", 11, 4), ("box", 8, 4)])
def test_single_frame_shorter_tiles(P, dev, c1, window, k, stride):
    """One 1080p frame alone is cut into shorter tiles than inside the batch
    (so that it spreads over all CUs): its map equals the batched frame's map
    bit for bit, and the oracle's map, and its score matches."""
    x, y, xt, yt = c1
    cfg = P.SSIMConfig(window=window, k=k, stride=stride)
    sb, mb = P.ssim(xt[:4], yt[:4], cfg, return_map=True)
    s1, m1 = P.ssim(xt[2:3], yt[2:3], cfg, return_map=True)
    torch.cuda.synchronize()
    assert torch.equal(m1[0], mb[2])
    assert abs(float(s1[0]) - float(sb[2])) <= 2e-7
    ref = O.ssim_map(x[2], y[2], oparams(cfg))["map"]
    assert np.abs(m1[0].cpu().numpy() - ref).max() <= MAP_TOL
    assert abs(float(s1[0]) - O.mean_pool(ref)) <= SCORE_TOL
