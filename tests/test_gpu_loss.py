"""The differentiable MS-SSIM loss entry point (ssimx_msssim_loss_rgb) and its
graph-replaying plan, through the C-ABI: the loss, scores and gradient
against the FP64 oracle (BT.601 luma, 3 scales, renormalised weights),
against the composed path, and graph replays against the eager call bit for
bit, with eager work and synchronisations between replays and new tensors on
some of them."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from _helpers import bf16_round, device, oparams, to_dev

pytestmark = pytest.mark.gpu

REL_L2, PIX_REL = 1e-4, 1e-3


@pytest.fixture(scope="module")
def P():
    import paper_2101_06354_amd as P
    return P


@pytest.fixture(scope="module")
def dev():
    return device()


def _oracle(r64, d64, cfg, B):
    ms = [O.msssim(O.rgb_to_y_bt601(r64[b]), O.rgb_to_y_bt601(d64[b]), cfg, n_scales=3, renorm=True)["score"]
          for b in range(len(r64))]
    g = np.stack([O.y_grad_to_rgb_bt601(O.msssim_backward(O.rgb_to_y_bt601(r64[b]), O.rgb_to_y_bt601(d64[b]),
                                                          -1.0 / B, cfg, n_scales=3, renorm=True))
                  for b in range(len(r64))])
    return float(np.mean([1 - m for m in ms])), np.array(ms), g


def _cmp(g, gref, what):
    g = np.asarray(g, dtype=np.float64)
    rel = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    pix = np.abs(g - gref).max() / np.abs(gref).max()
    assert rel <= REL_L2 and pix <= PIX_REL, f"{what}: rel {rel:.3g} pix {pix:.3g}"


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_loss_call_against_oracle(P, dev, storage):
    B = 3
    r, d = synth.config4(batch=B, h=160, w=200)
    rt, dt = to_dev(r, dev), to_dev(d, dev)
    if storage == "bf16":
        rt, dt = rt.bfloat16(), dt.bfloat16()
        r64, d64 = bf16_round(r), bf16_round(d)
    else:
        r64, d64 = r.astype(np.float64), d.astype(np.float64)
    cfg = P.SSIMConfig(L=1.0)
    loss, score, grad = P.msssim_loss_rgb(rt, dt, cfg, grad_dtype=torch.float32)
    lref, msref, gref = _oracle(r64, d64, oparams(cfg), B)
    assert abs(float(loss) - lref) <= 1e-6
    assert np.abs(score.cpu().numpy() - msref).max() <= 1e-6
    _cmp(grad.cpu().numpy(), gref, storage)
    # the gradient in the storage dtype is the float32 one rounded
    _, _, g16 = P.msssim_loss_rgb(rt, dt, cfg)
    assert g16.dtype == dt.dtype
    if storage == "bf16":
        assert torch.equal(g16, grad.bfloat16())
    # forward only: same loss and scores, no gradient
    l2, s2, g2 = P.msssim_loss_rgb(rt, dt, cfg, with_grad=False)
    assert g2 is None and torch.equal(l2, loss) and torch.equal(s2, score)


def _composed(P, rt, dt, cfg, **ms_kw):
    yr, yd = P.rgb_to_luma(rt.contiguous()), P.rgb_to_luma(dt.contiguous())
    ms = P.ms_ssim(yr, yd, cfg, **ms_kw)
    B = rt.shape[0]
    gy = P.ms_ssim_backward(yr, yd, torch.full((B,), -1.0 / B, device=rt.device), cfg, **ms_kw)
    return ms, P.luma_grad_to_rgb(gy)


def test_loss_call_against_composed_path(P, dev):
    """The same luma map and windowed kernels as the separate calls.  The
    loss builds its pyramid from the luma planes directly (the composed
    forward forms the 2x2 means from its staged u = x + y, v = x - y), so
    scores agree to float32 rounding, within the pooled-score bound."""
    r, d = synth.config4(batch=4, h=130, w=171)
    rt, dt = to_dev(r, dev), to_dev(d, dev)
    cfg = P.SSIMConfig(L=1.0)
    loss, score, grad = P.msssim_loss_rgb(rt, dt, cfg)
    ms, g2 = _composed(P, rt, dt, cfg, n_scales=3, renorm=True)
    assert float((score - ms).abs().max()) <= 1e-6
    assert abs(float(loss) - float((1 - ms.double()).mean())) <= 1e-6
    rel = float(torch.linalg.vector_norm(grad - g2) / torch.linalg.vector_norm(g2))
    assert rel <= 1e-5, rel


# Options of the loss call: the one-launch-per-pass route at five scales (two
# pyramid levels from the luma kernel, the rest down-sampled), with the split
# coarsest term (a seventh pass), cs clamping and the weighted-sum
# aggregation; the level-by-level route with padded borders; rows that are not
# 16-byte aligned (a view of wider planes) and bfloat16 storage.
@pytest.mark.parametrize("case", ["five_scales_split_clamp", "sum", "reflect", "unaligned_rows", "bf16_unaligned",
                                  "one_scale_split", "two_scales", "gaussian_k7"])
def test_loss_options_against_composed_path(P, dev, case):
    h, w, kw = 144, 186, dict(n_scales=3, renorm=True)
    cfg = P.SSIMConfig(L=1.0)
    if case == "five_scales_split_clamp":
        h, w, kw = 181, 195, dict(n_scales=5, renorm=True, cs_clamp=True, coarse_separate=True)
    elif case == "one_scale_split":  # no pyramid level; the split l pass on the luma planes
        kw = dict(n_scales=1, renorm=True, coarse_separate=True)
    elif case == "two_scales":  # one level from the luma kernel, none from the second level
        kw = dict(n_scales=2, renorm=True)
    elif case == "gaussian_k7":
        cfg = P.SSIMConfig(L=1.0, k=7, sigma=1.0)
    elif case == "sum":
        kw = dict(n_scales=4, renorm=False, aggregation="sum")
    elif case == "reflect":
        cfg = P.SSIMConfig(L=1.0, padding="reflect")
    r, d = synth.config4(batch=3, h=h, w=w + 1, stream=2)
    rt, dt = to_dev(r, dev), to_dev(d, dev)
    if case.startswith("bf16"):
        rt, dt = rt.bfloat16(), dt.bfloat16()
    if case.endswith("unaligned"):
        rt, dt = rt[..., 1:], dt[..., 1:]  # row pitch w + 1, planes start one element in
        assert rt.stride(2) == w + 1 and rt.data_ptr() % 16 != 0
    else:
        rt, dt = rt[..., :w].contiguous(), dt[..., :w].contiguous()
    loss, score, grad = P.msssim_loss_rgb(rt, dt, cfg, grad_dtype=torch.float32, **kw)
    ms, g2 = _composed(P, rt, dt, cfg, **kw)
    assert float((score - ms).abs().max()) <= 1e-6, case
    assert abs(float(loss) - float((1 - ms.double()).mean())) <= 1e-6, case
    rel = float(torch.linalg.vector_norm(grad - g2) / torch.linalg.vector_norm(g2))
    assert rel <= 1e-5, (case, rel)


def test_five_scale_loss_against_oracle(P, dev):
    """Five scales: levels 3 and 4 of the pyramid come from the stand-alone
    down-sampling of the luma kernel's level 2."""
    B = 2
    r, d = synth.config4(batch=B, h=176, w=180, stream=3)
    cfg = P.SSIMConfig(L=1.0)
    loss, score, grad = P.msssim_loss_rgb(to_dev(r, dev), to_dev(d, dev), cfg, n_scales=5, renorm=True)
    oc = oparams(cfg)
    r64, d64 = r.astype(np.float64), d.astype(np.float64)
    yr = [O.rgb_to_y_bt601(r64[b]) for b in range(B)]
    yd = [O.rgb_to_y_bt601(d64[b]) for b in range(B)]
    ms = np.array([O.msssim(yr[b], yd[b], oc, n_scales=5, renorm=True)["score"] for b in range(B)])
    g = np.stack([O.y_grad_to_rgb_bt601(O.msssim_backward(yr[b], yd[b], -1.0 / B, oc, n_scales=5, renorm=True))
                  for b in range(B)])
    assert np.abs(score.cpu().numpy() - ms).max() <= 1e-6
    assert abs(float(loss) - float(np.mean(1 - ms))) <= 1e-6
    _cmp(grad.cpu().numpy(), g, "five scales")


def test_plan_graph_replays_equal_the_eager_call(P, dev):
    B = 4
    r, d = synth.config4(batch=B, h=144, w=176)
    r2, d2 = synth.config4(batch=B, h=144, w=176, stream=1)
    cfg = P.SSIMConfig(L=1.0)
    sets = [(to_dev(r, dev), to_dev(d, dev)), (to_dev(r2, dev), to_dev(d2, dev))]
    eager = [P.msssim_loss_rgb(a, b, cfg) for a, b in sets]
    plan = P.LossPlan(cfg, torch.float32, B, 144, 176, device=dev)
    try:
        for rep in range(6):
            a, b = sets[rep % 2]
            if rep == 4:  # a fresh copy: new input pointers for the same plan
                a, b = a.clone(), b.clone()
            loss, score, grad = plan.run(a, b)
            torch.cuda.synchronize()
            el, es, eg = eager[rep % 2]
            assert torch.equal(loss, el) and torch.equal(score, es) and torch.equal(grad, eg), rep
            # unrelated eager work between replays
            _ = P.ssim(sets[0][0][:, 0].contiguous(), sets[0][1][:, 0].contiguous(), cfg)
            torch.cuda.synchronize()
        lf, sf, gf = plan.run(*sets[0], with_grad=False)
        torch.cuda.synchronize()
        assert gf is None and torch.equal(lf, eager[0][0]) and torch.equal(sf, eager[0][1])
    finally:
        plan.close()


@pytest.mark.parametrize("route", ["segmented", "level_by_level"])
def test_deferred_gradient_equals_the_one_call_form(P, dev, route):
    """Loss and scores from the first call, the gradient from the second,
    equal to ssimx_msssim_loss_rgb's; an upstream scalar (a power of two,
    exact in either product order) scales it."""
    r, d = synth.config4(batch=3, h=100, w=133, stream=4)
    rt, dt = to_dev(r, dev), to_dev(d, dev)
    cfg = P.SSIMConfig(L=1.0, padding="valid" if route == "segmented" else "zero")
    el, es, eg = P.msssim_loss_rgb(rt, dt, cfg)
    loss, score, state = P.ops.msssim_loss_rgb_deferred(rt, dt, cfg)
    assert torch.equal(loss, el) and torch.equal(score, es)
    g1 = P.ops.msssim_loss_rgb_grad(state)
    g2 = P.ops.msssim_loss_rgb_grad(state, torch.tensor(0.25, device=dev))  # the workspace is read, not consumed
    g3 = P.ops.msssim_loss_rgb_grad(state, torch.tensor(-2.0, device=dev), grad_dtype=torch.bfloat16)
    assert torch.equal(g1, eg) and torch.equal(g2, 0.25 * eg)
    assert torch.equal(g3, (-2.0 * eg).bfloat16())


def test_autograd_loss_takes_the_fused_path(P, dev):
    r, d = synth.config4(batch=2, h=96, w=120)
    cfg = P.SSIMConfig(L=1.0)
    rt = to_dev(r, dev)
    dt = to_dev(d, dev).requires_grad_(True)
    loss = P.autograd.ms_ssim_loss_rgb(rt, dt, cfg, n_scales=3, renorm=True)
    (4.0 * loss).backward()  # the upstream 4 is folded into the gradient kernel (exact for a power of two)
    el, _, eg = P.msssim_loss_rgb(rt, dt.detach(), cfg)
    assert torch.equal(loss.detach(), el)
    assert torch.equal(dt.grad, 4.0 * eg)
    # bfloat16 storage: the gradient comes back in bfloat16, scaled before rounding
    rb = rt.bfloat16()
    db = dt.detach().bfloat16().requires_grad_(True)
    lb = P.autograd.ms_ssim_loss_rgb(rb, db, cfg, n_scales=3, renorm=True)
    (0.5 * lb).backward()
    _, _, gb = P.msssim_loss_rgb(rb, db.detach(), cfg, grad_dtype=torch.float32)
    assert db.grad.dtype == torch.bfloat16 and torch.equal(db.grad, (0.5 * gb).bfloat16())
    # with a reference that needs a gradient the composed path serves both planes
    rt2 = to_dev(r, dev).requires_grad_(True)
    dt2 = to_dev(d, dev).requires_grad_(True)
    loss2 = P.autograd.ms_ssim_loss_rgb(rt2, dt2, cfg, n_scales=3, renorm=True)
    loss2.backward()
    assert abs(float(loss2.detach()) - float(el)) <= 1e-6
    rel = float(torch.linalg.vector_norm(dt2.grad - eg) / torch.linalg.vector_norm(eg))
    assert rel <= 1e-5 and rt2.grad is not None
