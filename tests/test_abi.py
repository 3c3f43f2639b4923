"""CPU-only checks of the C-ABI library: it loads, exports every function the
header declares, and its host-side validation rejects bad arguments before
any launch (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssimx.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:ssimx_status|const char\*|int|size_t)\s+([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_2101_06354_amd import _lib
    return _lib


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("ssim_map", "ssim_pooled", "msssim", "ssim_map_backward", "ssim_pooled_backward",
                 "msssim_backward", "ssimx_plan_create", "ssimx_plan_run", "ssimx_autotune"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in _declared() if not hasattr(L.lib, n)]
    assert not missing, missing


def test_struct_layouts_match_c(L):
    assert ctypes.sizeof(L.Params) == 48
    assert ctypes.sizeof(L.Image) == 40
    assert L.Params.C1.offset == 16 and L.Params.algo.offset == 40
    assert L.Image.pitch.offset == 24


def _params(L, **kw):
    d = dict(window=L.WIN_GAUSSIAN, k=11, sigma=1.5, C1=6.5025, C2=58.5225, stride=1, padding=L.PAD_VALID,
             algo=L.ALGO_AUTO)
    d.update(kw)
    return L.Params(**d)


def _shape(L, p, w, h):
    wo, ho = ctypes.c_int(), ctypes.c_int()
    st = L.lib.ssimx_map_shape(ctypes.byref(p), w, h, ctypes.byref(wo), ctypes.byref(ho))
    return st, (ho.value, wo.value)


def test_map_shape_host(L):
    assert _shape(L, _params(L), 1920, 1080) == (L.OK, (1070, 1910))
    assert _shape(L, _params(L, stride=4), 1920, 1080) == (L.OK, (268, 478))
    assert _shape(L, _params(L, window=L.WIN_BOX, k=8), 1920, 1080) == (L.OK, (1073, 1913))
    assert _shape(L, _params(L, window=L.WIN_BOX, k=8, stride=4), 1920, 1080) == (L.OK, (269, 479))
    assert _shape(L, _params(L, padding=L.PAD_REFLECT), 100, 50) == (L.OK, (50, 100))
    assert _shape(L, _params(L), 10, 10)[0] == L.ETOOSMALL


@pytest.mark.parametrize("bad", [dict(k=10), dict(k=0), dict(sigma=0.0), dict(stride=0), dict(C1=-1.0),
                                 dict(padding=7), dict(window=5), dict(k=43), dict(algo=9),
                                 dict(window=1, k=65), dict(C2=float("nan"))])
def test_invalid_params_rejected_on_host(L, bad):
    p = _params(L, **bad)
    assert _shape(L, p, 64, 64)[0] == L.EINVAL


def test_compute_calls_validate_before_launch(L):
    p = _params(L)
    img = L.Image(None, L.U8, 64, 64, 64, 4096)
    ok = L.Image(12345, L.U8, 64, 64, 64, 4096)
    score = ctypes.c_void_p(1)
    # null data pointer
    assert L.lib.ssim_pooled(ctypes.byref(p), ctypes.byref(img), ctypes.byref(ok), 1, score, None, 0, None) == L.EINVAL
    # mismatched sizes
    other = L.Image(12345, L.U8, 65, 64, 65, 4160)
    assert L.lib.ssim_pooled(ctypes.byref(p), ctypes.byref(ok), ctypes.byref(other), 1, score, None, 0,
                             None) == L.EINVAL
    # pitch below width
    badp = L.Image(12345, L.U8, 64, 64, 32, 4096)
    assert L.lib.ssim_pooled(ctypes.byref(p), ctypes.byref(badp), ctypes.byref(badp), 1, score, None, 0,
                             None) == L.EINVAL
    # workspace missing
    assert L.lib.ssim_pooled(ctypes.byref(p), ctypes.byref(ok), ctypes.byref(ok), 1, score, None, 0,
                             None) == L.EWORKSPACE
    # too small for the window
    tiny = L.Image(12345, L.U8, 8, 8, 8, 64)
    assert L.lib.ssim_pooled(ctypes.byref(p), ctypes.byref(tiny), ctypes.byref(tiny), 1, score, None, 0,
                             None) == L.ETOOSMALL
    # bad dtype
    bdt = L.Image(12345, 9, 64, 64, 64, 4096)
    assert L.lib.ssim_pooled(ctypes.byref(p), ctypes.byref(bdt), ctypes.byref(bdt), 1, score, None, 0,
                             None) == L.EDTYPE
    # integral images need an integer plane and valid padding
    pb = _params(L, window=L.WIN_BOX, k=8, algo=L.ALGO_INTEGRAL_IMAGE, padding=L.PAD_ZERO)
    assert L.lib.ssim_pooled(ctypes.byref(pb), ctypes.byref(ok), ctypes.byref(ok), 1, score, None, 0,
                             None) == L.ENOTSUP
    fl = L.Image(12345, L.F32, 64, 64, 64, 4096)
    pb = _params(L, window=L.WIN_BOX, k=8, algo=L.ALGO_INTEGRAL_IMAGE)
    assert L.lib.ssim_pooled(ctypes.byref(pb), ctypes.byref(fl), ctypes.byref(fl), 1, score, None, 0,
                             None) == L.EDTYPE


def test_msssim_scale_validation(L):
    p = _params(L)
    ok = L.Image(12345, L.U8, 256, 256, 256, 65536)
    w = (ctypes.c_float * 5)(0.0448, 0.2856, 0.3001, 0.2363, 0.1333)
    s = ctypes.c_void_p(1)
    # 256 -> 16 at the 5th scale: 16 >= 11 fits; 6 scales would not (8 < 11)
    w6 = (ctypes.c_float * 6)(*([0.2] * 6))
    assert L.lib.msssim(ctypes.byref(p), w6, 6, 0, ctypes.byref(ok), ctypes.byref(ok), 1, s, None, None, 0,
                        None) == L.ETOOSMALL
    assert L.lib.msssim(ctypes.byref(p), w, 0, 0, ctypes.byref(ok), ctypes.byref(ok), 1, s, None, None, 0,
                        None) == L.EINVAL
    assert L.lib.msssim(ctypes.byref(p), w, 5, 0, ctypes.byref(ok), ctypes.byref(ok), 1, s, None, None, 0,
                        None) == L.EWORKSPACE
    # unknown flag bits; normalised weights that sum to zero
    assert L.lib.msssim(ctypes.byref(p), w, 5, 16, ctypes.byref(ok), ctypes.byref(ok), 1, s, None, None, 0,
                        None) == L.EINVAL
    wz = (ctypes.c_float * 2)(1.0, -1.0)
    for fl in (L.MS_RENORM, L.MS_SUM):
        assert L.lib.msssim(ctypes.byref(p), wz, 2, fl, ctypes.byref(ok), ctypes.byref(ok), 1, s, None, None, 0,
                            None) == L.EINVAL
    assert L.lib.msssim(ctypes.byref(p), wz, 2, 0, ctypes.byref(ok), ctypes.byref(ok), 1, s, None, None, 0,
                        None) == L.EWORKSPACE
    assert L.lib.msssim(ctypes.byref(p), w, 5, L.MS_SUM | L.MS_CS_CLAMP, ctypes.byref(ok), ctypes.byref(ok), 1, s,
                        None, None, 0, None) == L.EWORKSPACE


def test_msssim_backward_values_validation(L):
    """The forward-values adjoint: both forward outputs are required, the split
    coarsest term is refused (it is not in cs_out), otherwise the checks of
    msssim_backward apply (here: no workspace)."""
    p = _params(L)
    ok = L.Image(12345, L.U8, 256, 256, 256, 65536)
    w = (ctypes.c_float * 5)(0.0448, 0.2856, 0.3001, 0.2363, 0.1333)
    d = ctypes.c_void_p(1)
    f = L.lib.msssim_backward_values
    args = (ctypes.byref(p), w, 5)
    img = (ctypes.byref(ok), ctypes.byref(ok), 1)
    assert f(*args, 0, *img, None, d, d, d, 256, 65536, None, 0, None) == L.EINVAL
    assert f(*args, 0, *img, d, None, d, d, 256, 65536, None, 0, None) == L.EINVAL
    assert f(*args, L.MS_COARSE_SEPARATE, *img, d, d, d, d, 256, 65536, None, 0, None) == L.ENOTSUP
    assert f(*args, 0, *img, d, d, None, d, 256, 65536, None, 0, None) == L.EINVAL
    assert f(*args, 0, *img, d, d, d, d, 256, 65536, None, 0, None) == L.EWORKSPACE
    assert f(*args, 16, *img, d, d, d, d, 256, 65536, None, 0, None) == L.EINVAL


def test_workspace_size_and_tile_api(L):
    p = _params(L)
    n = ctypes.c_size_t()
    assert L.lib.ssimx_workspace_size(ctypes.byref(p), L.OP_POOLED, L.U8, 1920, 1080, 64, 1, ctypes.byref(n)) == L.OK
    assert n.value > 0
    assert L.lib.ssimx_workspace_size(ctypes.byref(p), L.OP_MSSSIM, L.U8, 1920, 1080, 4, 5, ctypes.byref(n)) == L.OK
    # the pyramid levels dominate: 2 planes * 4 frames * (1/4 + 1/16 + ...) of 1080p in float32
    assert n.value > 2 * 4 * 4 * (960 * 540)
    assert L.lib.ssimx_num_tile_configs() >= 1
    assert L.lib.ssimx_set_tile_override(-1) == L.OK
    assert L.lib.ssimx_set_tile_override(10**6) == L.EINVAL
    assert L.lib.ssimx_strerror(L.EWORKSPACE) == b"workspace missing or too small"
    assert L.lib.ssimx_version() >= 100


def test_plan_create_validates_before_allocating(L):
    pair = L.Pair()
    pair.ref = L.Image(12345, L.U8, 64, 64, 64, 4096)
    pair.dis = L.Image(12345, L.U8, 64, 64, 64, 4096)
    pair.p = _params(L, k=10)  # even Gaussian window
    arr = (L.Pair * 1)(pair)
    h = ctypes.c_void_p()
    assert L.lib.ssimx_plan_create(arr, 1, None, ctypes.byref(h)) == L.EINVAL
    pair.p = _params(L)
    pair.dis = L.Image(12345, L.U16, 64, 64, 64, 4096)
    arr = (L.Pair * 1)(pair)
    assert L.lib.ssimx_plan_create(arr, 1, None, ctypes.byref(h)) == L.EINVAL
    assert L.lib.ssimx_plan_create(arr, 0, None, ctypes.byref(h)) == L.EINVAL
    assert L.lib.ssimx_plan_destroy(None) == L.EINVAL


def _pool(L, kind, p=0.0, o=1.0, r=1.0):
    return L.Pool(kind, p, o, r)


@pytest.mark.parametrize("kind,p,o,r", [(14, 0, 1, 1), (-1, 0, 1, 1), (2, 0.0, 1, 1), (3, -1.0, 1, 1),
                                        (4, -0.5, 1, 1), (6, 101.0, 1, 1), (6, 5.0, 1, 0.0),
                                        (1, float("nan"), 1, 1), (10, 0.0, 1, 1), (11, 2.5, 1, 1),
                                        (13, -3.0, 1, 1)])
def test_pool_parameters_rejected_on_host(L, kind, p, o, r):
    n = ctypes.c_size_t()
    pl = _pool(L, kind, p, o, r)
    assert L.lib.ssimx_pool_workspace_size(ctypes.byref(pl), 64, 64, 1, ctypes.byref(n)) == L.EINVAL
    assert L.lib.ssimx_pool_map(ctypes.byref(pl), 12345, 64, 64, 64, 4096, 1, 12345, 12345, 1 << 20,
                                None) == L.EINVAL


def test_pool_map_validates_before_launch(L):
    pl = _pool(L, L.POOL_COV)
    n = ctypes.c_size_t()
    assert L.lib.ssimx_pool_workspace_size(ctypes.byref(pl), 64, 64, 2, ctypes.byref(n)) == L.OK
    assert n.value > 0
    f = L.lib.ssimx_pool_map
    assert f(ctypes.byref(pl), None, 64, 64, 64, 4096, 1, 12345, 12345, n.value, None) == L.EINVAL
    assert f(ctypes.byref(pl), 12345, 64, 64, 32, 4096, 1, 12345, 12345, n.value, None) == L.EINVAL
    assert f(ctypes.byref(pl), 12345, 64, 64, 64, 100, 2, 12345, 12345, n.value, None) == L.EINVAL
    assert f(ctypes.byref(pl), 12345, 0, 64, 64, 4096, 1, 12345, 12345, n.value, None) == L.ETOOSMALL
    assert f(ctypes.byref(pl), 12345, 64, 64, 64, 4096, 1, 12345, None, 0, None) == L.EWORKSPACE
    big = _pool(L, L.POOL_FIVE_NUMBER)
    assert L.lib.ssimx_pool_workspace_size(ctypes.byref(big), 64, 64, 2, ctypes.byref(n)) == L.OK
    # windowed means: single-row maps, window no longer than the row
    wp = _pool(L, L.POOL_WIN_GM, 8.0)
    assert L.lib.ssimx_pool_workspace_size(ctypes.byref(wp), 300, 1, 2, ctypes.byref(n)) == L.OK
    assert f(ctypes.byref(wp), 12345, 300, 2, 300, 600, 1, 12345, 12345, n.value, None) == L.EINVAL
    assert f(ctypes.byref(wp), 12345, 7, 1, 7, 7, 1, 12345, 12345, n.value, None) == L.ETOOSMALL
    assert f(ctypes.byref(wp), 12345, 300, 1, 300, 300, 2, 12345, None, 0, None) == L.EWORKSPACE


def test_ssim3d_validates_before_launch(L):
    box = _params(L, window=L.WIN_BOX, k=11)
    clip = L.Image(12345, L.U8, 64, 48, 64, 64 * 48)
    s = ctypes.c_void_p(1)
    n = ctypes.c_size_t()

    def call(p, kt, frames=8, m=None, sc=s, ws=None, nb=0):
        return L.lib.ssimx_ssim3d(ctypes.byref(p), kt, ctypes.byref(clip), ctypes.byref(clip), frames, m, 64,
                                  64 * 48, sc, ws, nb, None)

    assert call(_params(L, window=L.WIN_GAUSSIAN, k=11), 3) == L.ENOTSUP
    assert call(_params(L, window=L.WIN_BOX, k=11, stride=2), 3) == L.ENOTSUP
    assert call(_params(L, window=L.WIN_BOX, k=11, padding=L.PAD_ZERO), 3) == L.ENOTSUP
    assert call(_params(L, window=L.WIN_BOX, k=17), 3) == L.ENOTSUP
    assert call(box, 0) == L.EINVAL and call(box, 65) == L.EINVAL
    assert call(box, 9, frames=8) == L.ETOOSMALL
    assert call(box, 3, sc=None) == L.EINVAL          # neither map nor scores
    assert call(box, 3) == L.EWORKSPACE
    wide = L.Image(12345, L.U8, 64, 48, (1 << 26) + 1, ((1 << 26) + 1) * 48)  # row pitch beyond 2^26
    assert L.lib.ssimx_ssim3d(ctypes.byref(box), 3, ctypes.byref(wide), ctypes.byref(clip), 8, None, 64, 64 * 48,
                              s, None, 0, None) == L.EINVAL
    assert L.lib.ssimx_ssim3d_workspace_size(ctypes.byref(box), 3, L.U8, 64, 48, 8, ctypes.byref(n)) == L.OK
    assert n.value > 0
    assert call(box, 3, ws=ctypes.c_void_p(1), nb=n.value - 1) == L.EWORKSPACE
    assert L.lib.ssimx_ssim3d_workspace_size(ctypes.byref(box), 3, L.U8, 10, 48, 8, ctypes.byref(n)) == L.ETOOSMALL
    w = (ctypes.c_float * 3)(0.2, 0.3, 0.5)
    # 48 -> 24 -> 12 rows: three scales hold an 11 x 11 box, four do not
    assert L.lib.ssimx_msssim3d_workspace_size(ctypes.byref(box), 3, 3, L.U8, 64, 48, 8, ctypes.byref(n)) == L.OK
    assert L.lib.ssimx_msssim3d_workspace_size(ctypes.byref(box), 3, 4, L.U8, 64, 48, 8,
                                               ctypes.byref(n)) == L.ETOOSMALL
    assert L.lib.ssimx_msssim3d(ctypes.byref(box), 3, w, 3, 16, ctypes.byref(clip), ctypes.byref(clip), 8, s, None,
                                None, 0, None) == L.EINVAL
    assert L.lib.ssimx_msssim3d(ctypes.byref(box), 3, w, 3, 0, ctypes.byref(clip), ctypes.byref(clip), 8, s, None,
                                None, 0, None) == L.EWORKSPACE


def test_package_fails_loudly_without_the_library(tmp_path):
    """A copy of the package without libssimx.so must not import (no CPU path)."""
    import shutil
    import subprocess
    import sys
    src = os.path.join(ROOT, "paper_2101_06354_amd")
    dst = tmp_path / "paper_2101_06354_amd"
    shutil.copytree(src, dst, ignore=shutil.ignore_patterns("*.so", "_build", "csrc", "__pycache__"))
    env = {k: v for k, v in os.environ.items() if k != "SSIMX_LIBRARY"}  # no other build to fall back on
    r = subprocess.run([sys.executable, "-c", "import paper_2101_06354_amd"], cwd=tmp_path,
                       capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "not built" in r.stderr


def test_host_tensors_are_rejected_not_computed(L):
    import torch
    import paper_2101_06354_amd as P
    x = torch.zeros((1, 32, 32), dtype=torch.uint8)
    with pytest.raises(ValueError, match="device tensors"):
        P.ssim(x, x)
    with pytest.raises(ValueError):
        P.ssim3d(torch.zeros((4, 32, 32), dtype=torch.uint8), torch.zeros((4, 32, 32), dtype=torch.uint8), 2)


# ---------------------------------------------------------------- launch limits
def test_batch_beyond_grid_limit_is_refused_before_launch(L):
    """Frames go on grid.y (65535 at most); the host refuses more with EINVAL
    before any launch (the device pointers here are never dereferenced)."""
    p = _params(L)
    im = L.Image(4096, L.U8, 64, 64, 64, 4096)
    sc, ws = ctypes.c_void_p(8192), ctypes.c_void_p(16384)
    big = 1 << 30
    for batch, want in ((65536, L.EINVAL), (70000, L.EINVAL)):
        assert L.lib.ssim_pooled(ctypes.byref(p), ctypes.byref(im), ctypes.byref(im), batch, sc, ws, big,
                                 None) == want
        assert L.lib.ssim_map(ctypes.byref(p), ctypes.byref(im), ctypes.byref(im), batch, sc, 54, 54 * 54, sc, ws,
                              big, None) == want
        assert L.lib.ssim_pooled_backward(ctypes.byref(p), ctypes.byref(im), ctypes.byref(im), batch, sc, sc, 64,
                                          4096, ws, big, None) == want
        w = (ctypes.c_float * 2)(0.5, 0.5)
        assert L.lib.msssim(ctypes.byref(p), w, 2, 0, ctypes.byref(im), ctypes.byref(im), batch, sc, None, ws, big,
                            None) == want
        n = ctypes.c_size_t()
        assert L.lib.ssimx_workspace_size(ctypes.byref(p), L.OP_POOLED, L.U8, 64, 64, batch, 1,
                                          ctypes.byref(n)) == want
        assert L.lib.ssimx_rgb_to_luma(sc, L.F32, 64, 64, 64, 4096, 3 * 4096, batch, sc, None) == want
        assert L.lib.ssimx_luma_grad_to_rgb(sc, 64, 64, batch, sc, 64, 4096, 3 * 4096, None) == want
        pool = L.Pool(kind=L.POOL_MEAN, p=1.0, o=1.0, r=1.0)
        assert L.lib.ssimx_pool_map(ctypes.byref(pool), sc, 64, 64, 64, 4096, batch, sc, ws, big, None) == want
        assert L.lib.ssimx_pool_workspace_size(ctypes.byref(pool), 64, 64, batch, ctypes.byref(n)) == want
        assert L.lib.ssimx_ssim3d_workspace_size(ctypes.byref(_params(L, window=L.WIN_BOX, k=8)), 3, L.U8, 64, 64,
                                                 batch, ctypes.byref(n)) == want
    # the colour path launches three channel frames per RGB frame
    assert L.lib.ssimx_color_ssim(ctypes.byref(p), 0.125, 0.125, sc, sc, L.U8, 64, 64, 64, 4096, 3 * 4096, 21846,
                                  sc, None, ws, big, None) == L.EINVAL
    n = ctypes.c_size_t()
    assert L.lib.ssimx_color_workspace_size(ctypes.byref(p), 64, 64, 21846, ctypes.byref(n)) == L.EINVAL
    assert L.lib.ssimx_color_workspace_size(ctypes.byref(p), 64, 64, 21845, ctypes.byref(n)) == L.OK
    # the largest accepted batch passes validation (and stops at the workspace check)
    assert L.lib.ssim_pooled(ctypes.byref(p), ctypes.byref(im), ctypes.byref(im), 65535, sc, None, 0,
                             None) == L.EWORKSPACE


def test_plane_element_limit(L):
    p = _params(L)
    sc = ctypes.c_void_p(8192)
    huge = L.Image(4096, L.U8, 1 << 16, 1 << 15, 1 << 16, 1 << 31)  # 2^31 pixels
    assert L.lib.ssim_pooled(ctypes.byref(p), ctypes.byref(huge), ctypes.byref(huge), 1, sc, None, 0,
                             None) == L.EINVAL
    n = ctypes.c_size_t()
    assert L.lib.ssimx_workspace_size(ctypes.byref(p), L.OP_POOLED, L.U8, 1 << 16, 1 << 15, 1, 1,
                                      ctypes.byref(n)) == L.EINVAL
    assert L.lib.ssimx_rgb_to_luma(sc, L.F32, 1 << 16, 1 << 15, 1 << 16, 1 << 31, 3 << 31, 1, sc,
                                   None) == L.EINVAL


def test_integral_image_refuses_16bit_windows(L):
    """uint32 tables cannot hold a 16-bit window sum of squares from k = 2 up
    (k^2 * 65535^2 >= 2^32): ENOTSUP, while the tile-sum algorithm accepts."""
    sc = ctypes.c_void_p(8192)
    im16 = L.Image(4096, L.U16, 64, 64, 64, 4096)
    im8 = L.Image(4096, L.U8, 64, 64, 64, 4096)
    for k in (2, 8, 16):
        pb = _params(L, window=L.WIN_BOX, k=k, algo=L.ALGO_INTEGRAL_IMAGE)
        assert L.lib.ssim_pooled(ctypes.byref(pb), ctypes.byref(im16), ctypes.byref(im16), 1, sc, None, 0,
                                 None) == L.ENOTSUP
        assert L.lib.ssim_pooled(ctypes.byref(pb), ctypes.byref(im8), ctypes.byref(im8), 1, sc, None, 0,
                                 None) == L.EWORKSPACE
        pa = _params(L, window=L.WIN_BOX, k=k, algo=L.ALGO_AUTO)
        assert L.lib.ssim_pooled(ctypes.byref(pa), ctypes.byref(im16), ctypes.byref(im16), 1, sc, None, 0,
                                 None) == L.EWORKSPACE
    p1 = _params(L, window=L.WIN_BOX, k=1, algo=L.ALGO_INTEGRAL_IMAGE)
    assert L.lib.ssim_pooled(ctypes.byref(p1), ctypes.byref(im16), ctypes.byref(im16), 1, sc, None, 0,
                             None) == L.EWORKSPACE


# ---------------------------------------------------------------- tune cache file
def _cache_entries(L, tmp_path, name="dump.json"):
    import json
    out = tmp_path / name
    assert L.lib.ssimx_tune_cache_save(str(out).encode()) == L.OK
    return json.loads(out.read_text())["entries"]


def test_tune_cache_round_trip_and_merge(L, tmp_path):
    v = L.lib.ssimx_version()
    f = tmp_path / "good.json"
    f.write_text('{ "version" : %d ,\n "entries": {"cpu-test|a": 1, "cpu-test|b" :0} }\n' % v)
    assert L.lib.ssimx_tune_cache_load(str(f).encode()) == L.OK
    e = _cache_entries(L, tmp_path)
    assert e["cpu-test|a"] == 1 and e["cpu-test|b"] == 0
    # what save writes loads back unchanged
    again = tmp_path / "dump.json"
    assert L.lib.ssimx_tune_cache_load(str(again).encode()) == L.OK
    assert _cache_entries(L, tmp_path, "dump2.json") == e
    # an empty entries object is valid and changes nothing
    f.write_text('{"version": %d, "entries": {}}' % v)
    assert L.lib.ssimx_tune_cache_load(str(f).encode()) == L.OK
    assert _cache_entries(L, tmp_path, "dump3.json") == e


@pytest.mark.parametrize("text", [
    "",                                                   # empty file
    "{",                                                  # truncated
    '{"version": %(v)d, "entries": {"cpu-bad|x": 1}',     # missing closing brace
    '{"version": %(v)d, "entries": {"cpu-bad|x": 1,}}',   # trailing comma
    '{"version": %(v)d, "entries": {"cpu-bad|x": }}',     # missing value
    '{"version": %(v)d, "entries": {"cpu-bad|x": abc}}',  # non-numeric value
    '{"version": %(v)d, "entries": {"cpu-bad|x": 1.5}}',  # fractional value
    '{"version": %(v)d, "entries": {"cpu-bad|x": -1}}',   # tile index below range
    '{"version": %(v)d, "entries": {"cpu-bad|x": 99}}',   # tile index above range
    '{"version": %(v)d, "entries": {"cpu-bad|x": 1234567890123}}',  # overlong number
    '{"version": %(v)d, "entries": {"cpu-bad|x": 1, "cpu-bad|x": 2}}',  # duplicate key
    '{"version": %(v)d, "entries": {"cpu-bad|\\"x": 1}}',  # escaped quote in a key
    '{"version": %(v)d, "entries": {"cpu-bad|x": 1}} trailing',  # trailing garbage
    '{"version": 1, "entries": {"cpu-bad|x": 1}}',          # another version
    '{"entries": {"cpu-bad|x": 1}}',                        # no version
    '{"version": %(v)d}',                                   # no entries
    '{"version": %(v)d, "entries": {"cpu-bad|x": 1}, "extra": 1}',  # unknown member
    '{"version": %(v)d, "entries": ["cpu-bad|x", 1]}',      # wrong container
    '{"version": %(v)d, "entries": {"cpu-bad|x" 1}}',       # missing colon
    '{"version": %(v)d, "entries": {cpu-bad: 1}}',          # unquoted key
    '{"version": %(v)d, "entries": {"cpu-bad|%(long)s": 1}}',  # key too long
])
def test_tune_cache_rejects_malformed_files(L, tmp_path, text):
    v = L.lib.ssimx_version()
    before = _cache_entries(L, tmp_path, "before.json")
    f = tmp_path / "bad.json"
    f.write_text(text % {"v": v, "long": "k" * 200} if "%(" in text else text)
    assert L.lib.ssimx_tune_cache_load(str(f).encode()) == L.EINVAL
    after = _cache_entries(L, tmp_path, "after.json")
    assert after == before and not any(k.startswith("cpu-bad") for k in after)


def test_tune_cache_rejects_missing_binary_and_oversized_files(L, tmp_path):
    assert L.lib.ssimx_tune_cache_load(str(tmp_path / "absent.json").encode()) == L.EINVAL
    assert L.lib.ssimx_tune_cache_load(None) == L.EINVAL
    v = L.lib.ssimx_version()  # the current version: only the content may be refused
    b = tmp_path / "binary.json"
    b.write_bytes(b'{"version": %d, "entries": {"cpu-bad|\x01": 1}}' % v)
    assert L.lib.ssimx_tune_cache_load(str(b).encode()) == L.EINVAL
    big = tmp_path / "big.json"
    big.write_text('{"version": %d, "entries": {' % v + " " * (1 << 20) + "}}")
    assert L.lib.ssimx_tune_cache_load(str(big).encode()) == L.EINVAL


def test_tune_cache_environment_variable(tmp_path):
    """SSIMX_TUNE_CACHE is loaded once, before the first save/tile choice, in
    a fresh process (the variable is read only once per process)."""
    import subprocess
    import sys
    src = tmp_path / "env.json"
    out = tmp_path / "out.json"
    script = (
        "import sys, json; sys.path.insert(0, %r)\n"
        "from paper_2101_06354_amd import _lib as L\n"
        "v = L.lib.ssimx_version()\n"
        "open(%r, 'w').write('{\"version\": %%d, \"entries\": {\"cpu-env|k\": 2}}' %% v)\n"
        "assert L.lib.ssimx_tune_cache_save(%r.encode()) == L.OK\n"
        "print(json.load(open(%r))['entries'])\n" % (ROOT, str(src), str(out), str(out)))
    env = dict(os.environ, SSIMX_TUNE_CACHE=str(src))
    # the file is written by the child before its first save, so the save sees it
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "'cpu-env|k': 2" in r.stdout


def test_noalloc_entry_refuses_on_the_host(L):
    """ssim_pooled_noalloc validates like ssim_pooled and refuses, before any
    launch, a call whose scratch would exceed its static buffer."""
    p = _params(L)
    sc = ctypes.c_void_p(8192)
    im = L.Image(4096, L.U8, 64, 64, 64, 4096)
    assert L.lib.ssimx_noalloc_scratch_bytes() == 8 << 20
    assert L.lib.ssim_pooled_noalloc(ctypes.byref(p), ctypes.byref(im), ctypes.byref(im), 1, None, None) == L.EINVAL
    assert L.lib.ssim_pooled_noalloc(ctypes.byref(p), ctypes.byref(im), ctypes.byref(im), 65536, sc,
                                     None) == L.EINVAL
    tiny = L.Image(4096, L.U8, 8, 8, 8, 64)
    assert L.lib.ssim_pooled_noalloc(ctypes.byref(p), ctypes.byref(tiny), ctypes.byref(tiny), 1, sc,
                                     None) == L.ETOOSMALL
    # five uint32 integral images of a 1080p frame (~41 MB) exceed the 8 MiB buffer
    big = L.Image(4096, L.U8, 1920, 1080, 1920, 1920 * 1080)
    pb = _params(L, window=L.WIN_BOX, k=8, algo=L.ALGO_INTEGRAL_IMAGE)
    assert L.lib.ssim_pooled_noalloc(ctypes.byref(pb), ctypes.byref(big), ctypes.byref(big), 1, sc,
                                     None) == L.ESCRATCH
    assert L.lib.ssimx_strerror(L.ESCRATCH).decode().startswith("call needs more scratch")


def test_loss_entry_points_validate_on_the_host(L):
    p = _params(L, C1=1e-4, C2=9e-4)
    w = (ctypes.c_float * 3)(0.2, 0.3, 0.5)
    sc = ctypes.c_void_p(8192)
    n = ctypes.c_size_t()
    ok = L.lib.ssimx_msssim_loss_workspace_size(ctypes.byref(p), w, 3, L.MS_RENORM, L.F32, 512, 512, 16,
                                                ctypes.byref(n))
    assert ok == L.OK and n.value > 3 * 16 * 512 * 512 * 4
    assert L.lib.ssimx_msssim_loss_workspace_size(ctypes.byref(p), w, 3, L.MS_RENORM, L.U8, 512, 512, 16,
                                                  ctypes.byref(n)) == L.EDTYPE
    assert L.lib.ssimx_msssim_loss_workspace_size(ctypes.byref(p), w, 3, L.MS_RENORM, L.F32, 512, 512, 65536,
                                                  ctypes.byref(n)) == L.EINVAL
    # 40 x 40 at 3 scales leaves 10 x 10 < 11 at the coarsest
    assert L.lib.ssimx_msssim_loss_workspace_size(ctypes.byref(p), w, 3, L.MS_RENORM, L.F32, 40, 40, 1,
                                                  ctypes.byref(n)) == L.ETOOSMALL

    def call(**kw):
        a = dict(ref=sc, dis=sc, dtype=L.F32, w=64, h=64, pitch=64, cs=4096, bs=3 * 4096, b=2, loss=sc, score=None,
                 grad=sc, gdt=L.F32, gp=64, gcs=4096, gbs=3 * 4096, ws=None, wsb=0)
        a.update(kw)
        return L.lib.ssimx_msssim_loss_rgb(ctypes.byref(p), w, 3, L.MS_RENORM, a["ref"], a["dis"], a["dtype"],
                                           a["w"], a["h"], a["pitch"], a["cs"], a["bs"], a["b"], a["loss"],
                                           a["score"], a["grad"], a["gdt"], a["gp"], a["gcs"], a["gbs"], a["ws"],
                                           a["wsb"], None)
    assert call() == L.EWORKSPACE
    assert call(loss=None) == L.EINVAL
    assert call(dis=None) == L.EINVAL
    assert call(dtype=L.U16) == L.EDTYPE
    assert call(gdt=L.U8) == L.EDTYPE
    assert call(cs=100) == L.EINVAL       # channels overlap
    assert call(gbs=4096) == L.EINVAL     # gradient frames overlap
    assert call(grad=None, gdt=L.U8) == L.EWORKSPACE  # no gradient: its dtype is not looked at
    h = ctypes.c_void_p()
    assert L.lib.ssimx_loss_plan_create(ctypes.byref(p), w, 3, L.MS_RENORM, L.F32, L.U8, 64, 64, 2,
                                        ctypes.byref(h)) == L.EDTYPE
    assert L.lib.ssimx_loss_plan_create(ctypes.byref(p), w, 3, L.MS_RENORM, L.F32, L.F32, 64, 64, 2, None) == L.EINVAL
    assert L.lib.ssimx_loss_plan_run(None, sc, sc, 64, 4096, 3 * 4096, sc, None, None, 0, 0, 0, None) == L.EINVAL
    assert L.lib.ssimx_loss_plan_destroy(None) == L.EINVAL
    # the two-call form: same shape checks; the gradient half checks its own layout
    assert L.lib.ssimx_msssim_loss_rgb_deferred(ctypes.byref(p), w, 3, L.MS_RENORM, sc, sc, L.F32, 64, 64, 64, 4096,
                                                3 * 4096, 2, sc, None, None, 0, None) == L.EWORKSPACE
    assert L.lib.ssimx_msssim_loss_rgb_deferred(ctypes.byref(p), w, 3, L.MS_RENORM, sc, sc, L.F32, 64, 64, 64, 4096,
                                                3 * 4096, 2, None, None, None, 0, None) == L.EINVAL

    def grad(**kw):
        a = dict(grad=sc, gdt=L.F32, gp=64, gcs=4096, gbs=3 * 4096, ws=None, wsb=0, h=64)
        a.update(kw)
        return L.lib.ssimx_msssim_loss_rgb_grad(ctypes.byref(p), w, 3, L.MS_RENORM, L.F32, 64, a["h"], 2, None,
                                                a["grad"], a["gdt"], a["gp"], a["gcs"], a["gbs"], a["ws"], a["wsb"],
                                                None)
    assert grad() == L.EWORKSPACE
    assert grad(grad=None) == L.EINVAL
    assert grad(gdt=L.U16) == L.EDTYPE
    assert grad(gcs=100) == L.EINVAL
    assert grad(h=20) == L.ETOOSMALL
