"""GPU parity of the adjoint kernels (ssim_map_backward, ssim_pooled_backward,
msssim_backward, luma front end) against the FP64 oracle gradient, plus the
differentiable-loss workload (batch 16 of 3x512x512 RGB) checked against the
FP64 gradient and FP64 central differences."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _helpers import bf16_round, device, oparams, to_dev

pytestmark = pytest.mark.gpu

REL_L2 = 1e-4      # ||g - g*|| / ||g*||
PIX_REL = 1e-3     # max |g - g*| / max |g*|


@pytest.fixture(scope="module")
def P():
    import paper_2101_06354_amd as P
    return P


@pytest.fixture(scope="module")
def dev():
    return device()


def _cmp(g, gref, what=""):
    g = np.asarray(g, dtype=np.float64)
    rel = np.linalg.norm(g - gref) / max(np.linalg.norm(gref), 1e-300)
    pix = np.abs(g - gref).max() / max(np.abs(gref).max(), 1e-300)
    assert rel <= REL_L2 and pix <= PIX_REL, f"{what}: rel L2 {rel:.3g}, max pix {pix:.3g}"


def test_pooled_backward_config0(P, dev):
    x, y = synth.config0()
    cfg = P.SSIMConfig()
    g = P.ssim_backward(to_dev(x, dev), to_dev(y, dev), torch.tensor([1.0], device=dev), cfg)
    _cmp(g.cpu().numpy(), O.ssim_pooled_backward(x, y, 1.0, oparams(cfg)), "config0")


@pytest.mark.parametrize("window,k,stride,padding", [("gaussian", 11, 1, "valid"), ("gaussian", 11, 4, "valid"),
                                                     ("gaussian", 7, 2, "zero"), ("gaussian", 11, 1, "reflect"),
                                                     ("box", 8, 1, "valid"), ("box", 8, 4, "reflect"),
                                                     ("gaussian", 5, 3, "reflect")])
def test_map_backward_random_upstream(P, dev, window, k, stride, padding):
    rng = np.random.default_rng(k * 10 + stride)
    x = synth.smooth_field(rng, 67, 93, 16, 235).round().astype(np.uint8)
    y = np.clip(x + rng.normal(0, 10, x.shape).round(), 0, 255).astype(np.uint8)
    cfg = P.SSIMConfig(window=window, k=k, sigma=1.5 if k == 11 else 1.0, stride=stride, padding=padding)
    ho, wo = P.map_shape(cfg, 67, 93)
    up = rng.normal(size=(ho, wo))
    g = P.ssim_map_backward(to_dev(x, dev), to_dev(y, dev), to_dev(up.astype(np.float32), dev), cfg)
    gref = O.ssim_map_backward(x, y, up.astype(np.float32).astype(np.float64), oparams(cfg))
    _cmp(g.cpu().numpy(), gref, f"{window}{k}/s{stride}/{padding}")


def test_pooled_backward_batch_and_scaling(P, dev):
    x, y = synth.config1(frames=3, h=120, w=160)
    cfg = P.SSIMConfig()
    gs = np.array([1.0, -2.5, 0.25], dtype=np.float32)
    g = P.ssim_backward(to_dev(x, dev), to_dev(y, dev), to_dev(gs, dev), cfg).cpu().numpy()
    for f in range(3):
        _cmp(g[f], O.ssim_pooled_backward(x[f], y[f], float(gs[f]), oparams(cfg)), f"frame {f}")


def test_gradient_vanishes_at_identity(P, dev):
    x, _ = synth.config0()
    cfg = P.SSIMConfig()
    g = P.ssim_backward(to_dev(x, dev), to_dev(x, dev), torch.tensor([1.0], device=dev), cfg)
    assert float(g.abs().max()) == 0.0
    xf = synth.config4(batch=1, h=64, w=64)[0][0, 0]
    g = P.ms_ssim_backward(to_dev(xf, dev), to_dev(xf, dev), torch.tensor([1.0], device=dev), P.SSIMConfig(L=1.0),
                           n_scales=3, renorm=True)
    assert float(g.abs().max()) == 0.0


@pytest.mark.parametrize("n_scales,padding", [(3, "valid"), (5, "valid"), (2, "reflect")])
def test_msssim_backward_u16(P, dev, n_scales, padding):
    x, y = synth.config2(frames=2, h=200, w=260)
    cfg = P.SSIMConfig(L=1023.0, padding=padding)
    g = P.ms_ssim_backward(to_dev(x, dev), to_dev(y, dev), torch.tensor([1.0, 0.5], device=dev), cfg,
                           n_scales=n_scales, renorm=n_scales < 5).cpu().numpy()
    for f, gs in enumerate((1.0, 0.5)):
        gref = O.msssim_backward(x[f], y[f], gs, oparams(cfg), n_scales=n_scales, renorm=n_scales < 5)
        _cmp(g[f], gref, f"frame {f}")


def test_msssim_sum_backward(P, dev):
    x, y = synth.config2(frames=2, h=200, w=260)
    cfg = P.SSIMConfig(L=1023.0)
    g = P.ms_ssim_backward(to_dev(x, dev), to_dev(y, dev), torch.tensor([1.0, -2.0], device=dev), cfg,
                           n_scales=4, aggregation="sum").cpu().numpy()
    for f, gs in enumerate((1.0, -2.0)):
        gref = O.msssim_backward(x[f], y[f], gs, oparams(cfg), n_scales=4, aggregation="sum")
        _cmp(g[f], gref, f"frame {f}")
    # autograd wrapper routes the aggregation through
    xt = to_dev(x, dev)
    yt = to_dev(y, dev).float().requires_grad_(True)
    P.autograd.ms_ssim(xt.float(), yt, cfg, n_scales=4, aggregation="sum").sum().backward()
    gsum = P.ms_ssim_backward(xt.float(), yt.detach(), torch.ones(2, device=dev), cfg, n_scales=4,
                              aggregation="sum")
    assert torch.equal(yt.grad, gsum)


def test_luma_kernels(P, dev):
    r, _ = synth.config4(batch=2, h=40, w=56)
    yv = P.rgb_to_luma(to_dev(r, dev)).cpu().numpy()
    for b in range(2):
        np.testing.assert_allclose(yv[b], O.rgb_to_y_bt601(r[b]), rtol=0, atol=2e-7)
    gy = np.random.default_rng(1).normal(size=(2, 40, 56)).astype(np.float32)
    grgb = P.luma_grad_to_rgb(to_dev(gy, dev)).cpu().numpy()
    for b in range(2):
        np.testing.assert_allclose(grgb[b], O.y_grad_to_rgb_bt601(gy[b]), rtol=1e-7, atol=0)


def test_autograd_matches_direct_calls(P, dev):
    x, y = synth.config0()
    xt, yt = to_dev(x.astype(np.float32), dev), to_dev(y.astype(np.float32), dev).requires_grad_(True)
    cfg = P.SSIMConfig()
    s = P.autograd.ssim(xt, yt, cfg)
    (2.0 * s.sum()).backward()
    g = P.ssim_backward(xt, yt.detach(), torch.tensor([2.0], device=dev), cfg)
    assert torch.equal(yt.grad, g)


def test_autograd_reference_plane_gradient(P, dev):
    """Gradients flow to both planes: the reference plane's is the adjoint with
    the planes swapped (SSIM and MS-SSIM are symmetric), checked against the
    oracle's adjoint of the swapped pair."""
    x, y = synth.config1(frames=2, h=96, w=120)
    x32, y32 = x.astype(np.float32), y.astype(np.float32)
    xt = to_dev(x32, dev).requires_grad_(True)
    yt = to_dev(y32, dev).requires_grad_(True)
    cfg = P.SSIMConfig()
    P.autograd.ssim(xt, yt, cfg).sum().backward()
    for f in range(2):
        _cmp(xt.grad[f].cpu().numpy(), O.ssim_pooled_backward(y[f], x[f], 1.0, oparams(cfg)), f"ssim dx {f}")
        _cmp(yt.grad[f].cpu().numpy(), O.ssim_pooled_backward(x[f], y[f], 1.0, oparams(cfg)), f"ssim dy {f}")
    xt.grad = None
    yt.grad = None
    P.autograd.ms_ssim(xt, yt, cfg, n_scales=3, renorm=True).sum().backward()
    for f in range(2):
        gx = O.msssim_backward(y[f], x[f], 1.0, oparams(cfg), n_scales=3, renorm=True)
        _cmp(xt.grad[f].cpu().numpy(), gx, f"ms dx {f}")
        gy = O.msssim_backward(x[f], y[f], 1.0, oparams(cfg), n_scales=3, renorm=True)
        _cmp(yt.grad[f].cpu().numpy(), gy, f"ms dy {f}")


def test_bf16_storage_fp32_adjoint_full_contract(P, dev):
    """The BF16-storage variant of the differentiable workload: bf16 planes,
    float32 accumulation, the float32 adjoint returned by ms_ssim_backward
    compared with the FP64 oracle gradient of the bf16-rounded planes at the
    float32 contract (1e-4 relative L2, 1e-3 max per pixel) and with FP64
    central differences (h = 1e-3) at 64 random pixels."""
    B = 4
    r, d = synth.config4(batch=B)
    yr = np.stack([O.rgb_to_y_bt601(bf16_round(r[b])) for b in range(B)])
    yd = np.stack([O.rgb_to_y_bt601(bf16_round(d[b])) for b in range(B)])
    # luma planes rounded to bf16 storage (what the kernel reads)
    yr16, yd16 = bf16_round(yr.astype(np.float32)), bf16_round(yd.astype(np.float32))
    xt = to_dev(yr16.astype(np.float32), dev).bfloat16()
    yt = to_dev(yd16.astype(np.float32), dev).bfloat16()
    assert torch.equal(xt.double().cpu(), torch.from_numpy(yr16))
    cfg = P.SSIMConfig(L=1.0)
    ocfg = oparams(cfg)
    ups = (1.0, -0.25, 0.5, 2.0)
    g = P.ms_ssim_backward(xt, yt, torch.tensor(ups, device=dev), cfg, n_scales=3, renorm=True)
    assert g.dtype == torch.float32
    g = g.cpu().numpy()
    score = P.ms_ssim(xt, yt, cfg, n_scales=3, renorm=True).cpu().numpy()
    grefs = []
    for b in range(B):
        ms = O.msssim(yr16[b], yd16[b], ocfg, n_scales=3, renorm=True)["score"]
        assert abs(float(score[b]) - ms) <= 1e-6
        grefs.append(O.msssim_backward(yr16[b], yd16[b], ups[b], ocfg, n_scales=3, renorm=True))
        _cmp(g[b], grefs[b], f"bf16 frame {b}")
    rng = np.random.default_rng(65)
    for _ in range(64):
        b = int(rng.integers(0, 2))
        i, j = int(rng.integers(0, 512)), int(rng.integers(0, 512))
        dp, dm = yd16[b].copy(), yd16[b].copy()
        dp[i, j] += 1e-3
        dm[i, j] -= 1e-3
        f = lambda dd: ups[b] * O.msssim(yr16[b], dd, ocfg, n_scales=3, renorm=True)["score"]  # noqa: E731
        fd = (f(dp) - f(dm)) / 2e-3
        assert abs(g[b, i, j] - fd) <= 1e-3 * np.abs(grefs[b]).max(), (b, i, j, g[b, i, j], fd)


def _loss_grad_oracle(r, d, cfg, B):
    """FP64 gradient of mean_b(1 - MS(Y(r_b), Y(d_b))) with respect to d."""
    out = np.empty(d.shape)
    for b in range(len(d)):
        yr, yd = O.rgb_to_y_bt601(r[b]), O.rgb_to_y_bt601(d[b])
        gy = O.msssim_backward(yr, yd, -1.0 / B, cfg, n_scales=3, renorm=True)
        out[b] = O.y_grad_to_rgb_bt601(gy)
    return out


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_differentiable_loss_workload_full_size(P, dev, storage):
    """Batch 16 of 3x512x512 RGB, loss = mean(1 - MS-SSIM) on BT.601 luma,
    3 scales with renormalised weights, C1=(0.01)^2, C2=(0.03)^2."""
    B = 16
    r, d = synth.config4(batch=B)
    if storage == "bf16":
        rt = to_dev(r, dev).bfloat16()
        dt = to_dev(d, dev).bfloat16().requires_grad_(True)
        r64, d64 = bf16_round(r), bf16_round(d)
    else:
        rt, dt = to_dev(r, dev), to_dev(d, dev).requires_grad_(True)
        r64, d64 = r.astype(np.float64), d.astype(np.float64)
    cfg = P.SSIMConfig(L=1.0)
    loss = P.autograd.ms_ssim_loss_rgb(rt, dt, cfg, n_scales=3, renorm=True)
    loss.backward()
    g = dt.grad.float().cpu().numpy()
    ocfg = oparams(cfg)
    # loss value
    ms = [O.msssim(O.rgb_to_y_bt601(r64[b]), O.rgb_to_y_bt601(d64[b]), ocfg, n_scales=3, renorm=True)["score"]
          for b in range(B)]
    assert abs(float(loss.detach()) - np.mean([1 - m for m in ms])) <= 1e-6
    # FP64 analytic gradient on 4 frames (bf16 storage: the gradient is returned in bf16)
    gref = _loss_grad_oracle(r64[:4], d64[:4], ocfg, B)
    if storage == "f32":
        _cmp(g[:4], gref, "loss grad")
    else:
        rel = np.linalg.norm(g[:4] - gref) / np.linalg.norm(gref)
        assert rel <= 1e-2, rel  # bf16 rounding of the returned gradient
    # FP64 central differences (h = 1e-3) of the oracle loss at 64 random pixels
    rng = np.random.default_rng(64)
    fd_frames = 2
    for _ in range(64 if storage == "f32" else 16):
        b = int(rng.integers(0, fd_frames))
        c, i, j = int(rng.integers(0, 3)), int(rng.integers(0, 512)), int(rng.integers(0, 512))

        def loss_b(dd):
            return (1 - O.msssim(O.rgb_to_y_bt601(r64[b]), O.rgb_to_y_bt601(dd), ocfg, n_scales=3,
                                 renorm=True)["score"]) / B
        dp, dm = d64[b].copy(), d64[b].copy()
        dp[c, i, j] += 1e-3
        dm[c, i, j] -= 1e-3
        fd = (loss_b(dp) - loss_b(dm)) / 2e-3
        scale = np.abs(gref[b]).max()
        tol = 1e-3 * scale if storage == "f32" else 1e-2 * scale
        assert abs(g[b, c, i, j] - fd) <= tol, (b, c, i, j, g[b, c, i, j], fd)


@pytest.mark.parametrize("k,sigma", [(7, 1.0), (9, 1.5), (13, 2.0)])
@pytest.mark.parametrize("h,w", [(150, 203), (40, 300)])
def test_band_adjoint_window_sizes(P, dev, k, sigma, h, w):
    rng = np.random.default_rng(k + h)
    x = synth.smooth_field(rng, h, w, 16, 235).round().astype(np.uint8)
    y = np.clip(x + rng.normal(0, 10, x.shape).round(), 0, 255).astype(np.uint8)
    cfg = P.SSIMConfig(k=k, sigma=sigma)
    g = P.ssim_backward(to_dev(x, dev), to_dev(y, dev), torch.tensor([1.0], device=dev), cfg)
    _cmp(g.cpu().numpy(), O.ssim_pooled_backward(x, y, 1.0, oparams(cfg)), f"k{k}")


@pytest.mark.parametrize("window,k,n_scales", [("gaussian", 11, 3), ("box", 8, 2), ("gaussian", 7, 1)])
def test_msssim_coarse_separate_backward(P, dev, window, k, n_scales):
    """Adjoint of the mean(l) * mean(cs) coarsest term through both coefficient
    kernels (the stride-1 Gaussian band kernel and the generic one)."""
    x, y = synth.config2(frames=2, h=160, w=200)
    cfg = P.SSIMConfig(window=window, k=k, L=1023.0)
    w = P.MS_WEIGHTS if n_scales > 1 else (1.0,)
    g = P.ms_ssim_backward(to_dev(x, dev), to_dev(y, dev), torch.tensor([1.0, 0.5], device=dev), cfg,
                           weights=w, n_scales=n_scales, renorm=True, coarse_separate=True).cpu().numpy()
    for f, gs in enumerate((1.0, 0.5)):
        gref = O.msssim_backward(x[f], y[f], gs, oparams(cfg), weights=w, n_scales=n_scales, renorm=True,
                                 coarse_separate=True)
        _cmp(g[f], gref, f"frame {f}")


def test_backward_row_pitch_beyond_vector_offsets(P, dev):
    """Inputs whose rows lie 2^24 + 64 elements apart take the element-wise
    loads in both backward kernels: the gradient equals the one of the same
    frames stored densely."""
    x, y = synth.config1(frames=1, h=40, w=150)
    xt, yt = to_dev(x, dev), to_dev(y, dev)
    cfg = P.SSIMConfig()
    up = torch.tensor([1.0], device=dev)
    g = P.ssim_backward(xt, yt, up, cfg)
    pitch = (1 << 24) + 64
    bx = torch.zeros((40 * pitch,), dtype=torch.uint8, device=dev)
    by = torch.zeros_like(bx)
    vx = bx.as_strided((1, 40, 150), (40 * pitch, pitch, 1))
    vy = by.as_strided((1, 40, 150), (40 * pitch, pitch, 1))
    vx.copy_(xt)
    vy.copy_(yt)
    g2 = P.ssim_backward(vx, vy, up, cfg)
    assert torch.equal(g2, g)
    _cmp(g2[0].cpu().numpy(), O.ssim_pooled_backward(x[0], y[0], 1.0, oparams(cfg)), "wide pitch")
    del bx, by, vx, vy


@pytest.mark.parametrize("frames,h,w", [(3, 150, 173), (2, 1080, 1920), (1, 40, 64)])
def test_outputs_outside_the_map_stay_untouched(P, dev, frames, h, w):
    """The band kernels store every row and lane of a chunk, positions past
    the tile's last row or the plane's last column with an offset the
    hardware drops: the pitch padding and the slack between frames of the
    map and of the gradient keep their prior contents, and the valid parts
    equal the densely stored results."""
    import ctypes
    L = P._lib
    rng = np.random.default_rng(frames * 1000 + w)
    x = rng.integers(0, 256, (frames, h, w)).astype(np.uint8)
    y = np.clip(x.astype(np.int32) + rng.integers(-20, 21, x.shape), 0, 255).astype(np.uint8)
    xt, yt = to_dev(x, dev), to_dev(y, dev)
    cfg = P.SSIMConfig()
    pc = cfg.to_c()
    xi, yi = P.ops._image(xt), P.ops._image(yt)
    ho, wo = P.map_shape(cfg, h, w)
    sentinel = 12345.0
    # map: 37 columns of pitch padding, 5 rows of slack per frame
    mp, mrows = wo + 37, ho + 5
    qmap = torch.full((frames * mrows * mp,), sentinel, dtype=torch.float32, device=dev)
    score = torch.empty(frames, dtype=torch.float32, device=dev)
    ws = torch.empty(P.workspace_size(cfg, L.OP_MAP, L.U8, h, w, frames), dtype=torch.uint8, device=dev)
    L.check(L.lib.ssim_map(ctypes.byref(pc), ctypes.byref(xi), ctypes.byref(yi), frames, qmap.data_ptr(), mp,
                           mrows * mp, score.data_ptr(), ws.data_ptr(), ws.numel(), None), "ssim_map")
    # gradient: 29 columns of pitch padding, 3 rows of slack per frame
    gp, grows = w + 29, h + 3
    grad = torch.full((frames * grows * gp,), sentinel, dtype=torch.float32, device=dev)
    up = torch.ones(frames, dtype=torch.float32, device=dev)
    wsb = torch.empty(P.workspace_size(cfg, L.OP_POOLED_BACKWARD, L.U8, h, w, frames), dtype=torch.uint8,
                      device=dev)
    L.check(L.lib.ssim_pooled_backward(ctypes.byref(pc), ctypes.byref(xi), ctypes.byref(yi), frames, up.data_ptr(),
                                       grad.data_ptr(), gp, grows * gp, wsb.data_ptr(), wsb.numel(), None),
            "ssim_pooled_backward")
    torch.cuda.synchronize()
    m = qmap.view(frames, mrows, mp)
    assert bool((m[:, :ho, wo:] == sentinel).all()) and bool((m[:, ho:, :] == sentinel).all())
    _, dense_map = P.ssim(xt, yt, cfg, return_map=True)
    assert torch.equal(m[:, :ho, :wo], dense_map)
    g = grad.view(frames, grows, gp)
    assert bool((g[:, :h, w:] == sentinel).all()) and bool((g[:, h:, :] == sentinel).all())
    assert torch.equal(g[:, :h, :w], P.ssim_backward(xt, yt, up, cfg))


@pytest.mark.parametrize("kind,n_scales,padding,aggregation",
                         [("u16", 5, "valid", "product"), ("u16", 3, "reflect", "product"),
                          ("u8", 4, "valid", "sum"), ("f32", 3, "valid", "product")])
def test_msssim_backward_from_forward_values(P, dev, kind, n_scales, padding, aggregation):
    """msssim_backward_values with the forward's score and per-scale values
    gives msssim_backward's gradient: bit for bit on integer planes (the same
    exact pyramid), to rounding on float planes, and the oracle's."""
    if kind == "f32":
        r, d = synth.config4(batch=2, h=200, w=260)
        x, y = r[:, 0], d[:, 0]
        cfg = P.SSIMConfig(L=1.0, padding=padding)
    elif kind == "u16":
        x, y = synth.config2(frames=2, h=200, w=260)
        cfg = P.SSIMConfig(L=1023.0, padding=padding)
    else:
        x, y = synth.config1(frames=2, h=200, w=260)
        cfg = P.SSIMConfig(padding=padding)
    xt, yt = to_dev(x, dev), to_dev(y, dev)
    gs = torch.tensor([1.0, -0.5], device=dev)
    kw = dict(n_scales=n_scales, renorm=n_scales < 5, aggregation=aggregation)
    score, cs = P.ms_ssim(xt, yt, cfg, return_cs=True, **kw)
    g0 = P.ms_ssim_backward(xt, yt, gs, cfg, **kw)
    g1 = P.ms_ssim_backward(xt, yt, gs, cfg, fwd=(score, cs), **kw)
    if kind == "f32":
        # the rebuilt 2x2 pyramid and the forward's (means formed from the
        # staged sums x + y, x - y) differ by rounding on float planes
        rel = float(torch.linalg.vector_norm(g1 - g0) / torch.linalg.vector_norm(g0))
        assert rel <= 1e-5, rel
    else:
        assert torch.equal(g1, g0)
    g1 = g1.cpu().numpy()
    for f, v in enumerate((1.0, -0.5)):
        gref = O.msssim_backward(x[f], y[f], v, oparams(cfg), n_scales=n_scales, renorm=n_scales < 5,
                                 aggregation=aggregation)
        _cmp(g1[f], gref, f"frame {f}")
    with pytest.raises(Exception):
        P.ms_ssim_backward(xt, yt, gs, cfg, fwd=(score, cs), coarse_separate=True, **kw)


def test_msssim_autograd_uses_forward_values(P, dev):
    """The differentiable MS-SSIM keeps its forward's values for the backward;
    the gradient equals the recomputing adjoint's bit for bit (8-bit planes)."""
    x, y = synth.config1(frames=2, h=200, w=260)
    xt, yt = to_dev(x, dev), to_dev(y, dev).float().requires_grad_(True)
    cfg = P.SSIMConfig()
    s = P.autograd.ms_ssim(xt.float(), yt, cfg, n_scales=3, renorm=True)
    (s * torch.tensor([1.0, 2.0], device=dev)).sum().backward()
    g = P.ms_ssim_backward(xt.float(), yt.detach(), torch.tensor([1.0, 2.0], device=dev), cfg, n_scales=3,
                           renorm=True)
    assert torch.equal(yt.grad, g)
