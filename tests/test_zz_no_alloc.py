"""ssim_pooled_noalloc (the entry point for callers that cannot allocate)
against ssim_pooled, through the C-ABI: equal scores bit for bit on two calls
in a row (the second on a smaller input, so stale scratch from the first call
would show), scores within the pooled tolerance of the FP64 oracle, and the
host-side refusal of a call that needs more scratch than the static buffer."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import synth
from _helpers import SCORE_TOL, device, oparams, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2101_06354_amd as P
    return P


@pytest.fixture(scope="module")
def dev():
    return device()


def _noalloc(P, xt, yt, cfg):
    L = P._lib
    xi, yi, b = P.ops._pair(xt, yt)
    p = cfg.to_c()
    out = torch.full((b,), float("nan"), dtype=torch.float32, device=xt.device)
    st = L.lib.ssim_pooled_noalloc(ctypes.byref(p), ctypes.byref(xi), ctypes.byref(yi), b, out.data_ptr(),
                                   P.ops._stream(xt))
    L.check(st, "ssim_pooled_noalloc")
    return out


@pytest.mark.parametrize("window,k,stride", [("gaussian", 11, 1), ("box", 8, 1), ("gaussian", 7, 3)])
def test_noalloc_equals_ssim_pooled_on_two_calls(P, dev, window, k, stride):
    cfg = P.SSIMConfig(window=window, k=k, stride=stride, sigma=1.5 if k == 11 else 1.0)
    big = synth.config1(frames=6, h=300, w=520)
    small = synth.config1(frames=2, h=97, w=150, stream=1)
    for x, y in (big, small):
        xt, yt = to_dev(x, dev), to_dev(y, dev)
        got = _noalloc(P, xt, yt, cfg)
        want = P.ssim(xt, yt, cfg)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (got, want)
        for f in range(x.shape[0]):
            ref = O.ssim_pooled(x[f], y[f], oparams(cfg))
            assert abs(float(got[f]) - ref) <= SCORE_TOL


def test_noalloc_refuses_calls_beyond_its_scratch(P, dev):
    L = P._lib
    cap = L.lib.ssimx_noalloc_scratch_bytes()
    assert cap == 8 << 20
    # 5 uint32 integral images of one 1080p frame need ~41 MB
    cfg = P.SSIMConfig(window="box", k=8, algo="integral")
    x = torch.zeros((1, 1080, 1920), dtype=torch.uint8, device=dev)
    xi, yi, b = P.ops._pair(x, x)
    need = P.workspace_size(cfg, L.OP_POOLED, L.U8, 1080, 1920, 1)
    assert need > cap
    out = torch.zeros(1, dtype=torch.float32, device=dev)
    p = cfg.to_c()
    assert L.lib.ssim_pooled_noalloc(ctypes.byref(p), ctypes.byref(xi), ctypes.byref(yi), 1, out.data_ptr(),
                                     None) == L.ESCRATCH
    torch.cuda.synchronize()
    assert float(out[0]) == 0.0  # nothing launched
