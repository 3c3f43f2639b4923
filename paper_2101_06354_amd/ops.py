"""Python binding of libssimx: argument marshalling for torch device tensors.

PyTorch supplies device memory (outputs and workspace) and the current HIP
stream only; every step of SSIM / MS-SSIM runs in the library's kernels.
Planes are (H, W) or (B, H, W) tensors whose last dimension is contiguous:
uint8, uint16, float32 or bfloat16.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import torch

from . import _lib as L

MS_WEIGHTS = (0.0448, 0.2856, 0.3001, 0.2363, 0.1333)

_DTYPES = {torch.uint8: L.U8, torch.float32: L.F32, torch.bfloat16: L.BF16}
if hasattr(torch, "uint16"):
    _DTYPES[torch.uint16] = L.U16
_WINDOWS = {"gaussian": L.WIN_GAUSSIAN, "box": L.WIN_BOX}
_PADS = {"valid": L.PAD_VALID, "zero": L.PAD_ZERO, "reflect": L.PAD_REFLECT}
_ALGOS = {"auto": L.ALGO_AUTO, "separable": L.ALGO_SEPARABLE, "integral": L.ALGO_INTEGRAL_IMAGE,
          "integral_image": L.ALGO_INTEGRAL_IMAGE}


@dataclass
class SSIMConfig:
    """Window type, size and sigma, C1 = (K1 L)^2, C2 = (K2 L)^2, stride,
    border handling and (rectangular windows on integer planes) algorithm."""
    window: str = "gaussian"
    k: int = 11
    sigma: float = 1.5
    K1: float = 0.01
    K2: float = 0.03
    L: float = 255.0
    C1: float | None = None
    C2: float | None = None
    stride: int = 1
    padding: str = "valid"
    algo: str = "auto"

    def c1(self) -> float:
        return (self.K1 * self.L) ** 2 if self.C1 is None else float(self.C1)

    def c2(self) -> float:
        return (self.K2 * self.L) ** 2 if self.C2 is None else float(self.C2)

    def to_c(self) -> L.Params:
        try:
            return L.Params(_WINDOWS[self.window], int(self.k), float(self.sigma), self.c1(), self.c2(),
                            int(self.stride), _PADS[self.padding], _ALGOS[self.algo])
        except KeyError as e:
            raise ValueError(f"unknown option {e}") from None


def _cfg(cfg: SSIMConfig | None, kw: dict) -> SSIMConfig:
    if cfg is not None and kw:
        raise ValueError("pass either cfg or keyword options")
    return cfg if cfg is not None else SSIMConfig(**kw)


def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


def _as3(t: torch.Tensor) -> torch.Tensor:
    if t.dim() == 2:
        return t.unsqueeze(0)
    if t.dim() != 3:
        raise ValueError("planes must be (H, W) or (B, H, W)")
    return t


def _image(t: torch.Tensor) -> L.Image:
    if not t.is_cuda:
        raise ValueError("libssimx needs device tensors (no CPU fallback)")
    if t.dtype not in _DTYPES:
        raise TypeError(f"unsupported dtype {t.dtype}")
    t3 = _as3(t)
    if t3.stride(2) != 1:
        raise ValueError("the last dimension must be contiguous")
    b, h, w = t3.shape
    return L.Image(t3.data_ptr(), _DTYPES[t.dtype], w, h, t3.stride(1), t3.stride(0) if b > 1 else t3.stride(1) * h)


def _pair(x: torch.Tensor, y: torch.Tensor):
    if x.shape != y.shape or x.dtype != y.dtype or x.device != y.device:
        raise ValueError("ref and dis must have the same shape, dtype and device")
    return _image(x), _image(y), _as3(x).shape[0]


def map_shape(cfg: SSIMConfig, h: int, w: int) -> tuple[int, int]:
    wo, ho = ctypes.c_int(), ctypes.c_int()
    st = L.lib.ssimx_map_shape(ctypes.byref(cfg.to_c()), w, h, ctypes.byref(wo), ctypes.byref(ho))
    L.check(st, "ssimx_map_shape")
    return ho.value, wo.value


def workspace_size(cfg: SSIMConfig, op: int, dtype: int, h: int, w: int, batch: int, n_scales: int = 1) -> int:
    n = ctypes.c_size_t()
    st = L.lib.ssimx_workspace_size(ctypes.byref(cfg.to_c()), op, dtype, w, h, batch, n_scales, ctypes.byref(n))
    L.check(st, "ssimx_workspace_size")
    return n.value


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(1, nbytes), dtype=torch.uint8, device=device)


def ssim(x: torch.Tensor, y: torch.Tensor, cfg: SSIMConfig | None = None, return_map: bool = False, **kw):
    """Mean SSIM per frame (float32 [B]); with return_map also the float32
    [B, Ho, Wo] quality map."""
    cfg = _cfg(cfg, kw)
    xi, yi, b = _pair(x, y)
    p = cfg.to_c()
    ho, wo = map_shape(cfg, xi.height, xi.width)
    ws = _workspace(workspace_size(cfg, L.OP_MAP, xi.dtype, xi.height, xi.width, b), x.device)
    score = torch.empty(b, dtype=torch.float32, device=x.device)
    if return_map:
        m = torch.empty((b, ho, wo), dtype=torch.float32, device=x.device)
        st = L.lib.ssim_map(ctypes.byref(p), ctypes.byref(xi), ctypes.byref(yi), b, m.data_ptr(), wo, ho * wo,
                            score.data_ptr(), ws.data_ptr(), ws.numel(), _stream(x))
        L.check(st, "ssim_map")
        return score, m
    st = L.lib.ssim_pooled(ctypes.byref(p), ctypes.byref(xi), ctypes.byref(yi), b, score.data_ptr(),
                           ws.data_ptr(), ws.numel(), _stream(x))
    L.check(st, "ssim_pooled")
    return score


def ssim_lw(x: torch.Tensor, y: torch.Tensor, a_s: float, b_s: float, cfg: SSIMConfig | None = None, **kw):
    """Luminance-weighted SSIM per frame (float32 [B]): the map weighted by
    the reference x's local mean (0 below a_s, a ramp of length b_s, then 1),
    summed and divided by the number of map positions."""
    cfg = _cfg(cfg, kw)
    xi, yi, b = _pair(x, y)
    p = cfg.to_c()
    ws = _workspace(workspace_size(cfg, L.OP_POOLED, xi.dtype, xi.height, xi.width, b), x.device)
    score = torch.empty(b, dtype=torch.float32, device=x.device)
    st = L.lib.ssim_pooled_lw(ctypes.byref(p), ctypes.byref(xi), ctypes.byref(yi), b, float(a_s), float(b_s),
                              score.data_ptr(), ws.data_ptr(), ws.numel(), _stream(x))
    L.check(st, "ssim_pooled_lw")
    return score


def _weights(weights, n_scales):
    if len(weights) < n_scales:
        raise ValueError("need one weight per scale")
    return (ctypes.c_float * n_scales)(*[float(v) for v in weights[:n_scales]])


def _ms_flags(renorm: bool, cs_clamp: bool, aggregation: str, coarse_separate: bool = False) -> int:
    if aggregation not in ("product", "sum"):
        raise ValueError(f"aggregation must be 'product' or 'sum', not {aggregation!r}")
    return ((L.MS_RENORM if renorm else 0) | (L.MS_CS_CLAMP if cs_clamp else 0)
            | (L.MS_SUM if aggregation == "sum" else 0) | (L.MS_COARSE_SEPARATE if coarse_separate else 0))


def ms_ssim(x: torch.Tensor, y: torch.Tensor, cfg: SSIMConfig | None = None, weights=MS_WEIGHTS,
            n_scales: int = 5, renorm: bool = False, cs_clamp: bool = False, return_cs: bool = False,
            aggregation: str = "product", coarse_separate: bool = False, return_pyramid: bool = False, **kw):
    """MS-SSIM per frame (float32 [B]); with return_cs also [B, n_scales]
    holding CS_1..CS_{M-1} and S_M.  aggregation="sum" takes the weighted
    average of the same terms with normalised weights instead of the
    weighted product; coarse_separate=True reads the coarsest term as
    mean(l) * mean(cs) instead of mean(l * cs).  return_pyramid=True also
    returns the levels the call built, [(x_j, y_j) for j = 1 .. n_scales-1],
    float32 [B, H_j, W_j] views of its workspace (ssimx_msssim_pyramid_layout)."""
    cfg = _cfg(cfg, kw)
    xi, yi, b = _pair(x, y)
    p = cfg.to_c()
    flags = _ms_flags(renorm, cs_clamp, aggregation, coarse_separate)
    ws = _workspace(workspace_size(cfg, L.OP_MSSSIM, xi.dtype, xi.height, xi.width, b, n_scales), x.device)
    score = torch.empty(b, dtype=torch.float32, device=x.device)
    cs = torch.empty((b, n_scales), dtype=torch.float32, device=x.device) if return_cs else None
    st = L.lib.msssim(ctypes.byref(p), _weights(weights, n_scales), n_scales, flags, ctypes.byref(xi),
                      ctypes.byref(yi), b, score.data_ptr(), cs.data_ptr() if cs is not None else None,
                      ws.data_ptr(), ws.numel(), _stream(x))
    L.check(st, "msssim")
    out = (score, cs) if return_cs else (score,)
    if return_pyramid:
        xo, yo = (ctypes.c_int64 * n_scales)(), (ctypes.c_int64 * n_scales)()
        wj, hj = (ctypes.c_int * n_scales)(), (ctypes.c_int * n_scales)()
        st = L.lib.ssimx_msssim_pyramid_layout(ctypes.byref(p), xi.dtype, xi.width, xi.height, b, n_scales, xo, yo,
                                               wj, hj)
        L.check(st, "ssimx_msssim_pyramid_layout")

        def level(off, j):
            n = b * hj[j] * wj[j] * 4
            return ws[off:off + n].view(torch.float32).reshape(b, hj[j], wj[j])
        out = out + ([(level(xo[j], j), level(yo[j], j)) for j in range(1, n_scales)],)
    return out if len(out) > 1 else out[0]


def ssim_backward(x: torch.Tensor, y: torch.Tensor, grad_score: torch.Tensor, cfg: SSIMConfig | None = None, **kw):
    """d(sum_b grad_score[b] * SSIM_b)/dy, float32 shaped like y."""
    cfg = _cfg(cfg, kw)
    xi, yi, b = _pair(x, y)
    p = cfg.to_c()
    g = grad_score.to(device=x.device, dtype=torch.float32).reshape(b).contiguous()
    out = torch.empty(_as3(y).shape, dtype=torch.float32, device=x.device)
    ws = _workspace(workspace_size(cfg, L.OP_POOLED_BACKWARD, xi.dtype, xi.height, xi.width, b), x.device)
    st = L.lib.ssim_pooled_backward(ctypes.byref(p), ctypes.byref(xi), ctypes.byref(yi), b, g.data_ptr(),
                                    out.data_ptr(), out.stride(1), out.stride(0), ws.data_ptr(), ws.numel(),
                                    _stream(x))
    L.check(st, "ssim_pooled_backward")
    return out.reshape(y.shape)


def ssim_map_backward(x: torch.Tensor, y: torch.Tensor, grad_map: torch.Tensor, cfg: SSIMConfig | None = None,
                      **kw):
    """sum_p grad_map(p) dQ(p)/dy, float32 shaped like y."""
    cfg = _cfg(cfg, kw)
    xi, yi, b = _pair(x, y)
    p = cfg.to_c()
    gm = _as3(grad_map.to(device=x.device, dtype=torch.float32)).contiguous()
    out = torch.empty(_as3(y).shape, dtype=torch.float32, device=x.device)
    ws = _workspace(workspace_size(cfg, L.OP_MAP_BACKWARD, xi.dtype, xi.height, xi.width, b), x.device)
    st = L.lib.ssim_map_backward(ctypes.byref(p), ctypes.byref(xi), ctypes.byref(yi), b, gm.data_ptr(),
                                 gm.stride(1), gm.stride(0), out.data_ptr(), out.stride(1), out.stride(0),
                                 ws.data_ptr(), ws.numel(), _stream(x))
    L.check(st, "ssim_map_backward")
    return out.reshape(y.shape)


def ms_ssim_backward(x: torch.Tensor, y: torch.Tensor, grad_score: torch.Tensor, cfg: SSIMConfig | None = None,
                     weights=MS_WEIGHTS, n_scales: int = 5, renorm: bool = False, cs_clamp: bool = False,
                     aggregation: str = "product", coarse_separate: bool = False, fwd=None, **kw):
    """dL/dy of MS-SSIM.  fwd = (score, cs), the outputs of ms_ssim(..., return_cs=True)
    on the same inputs and options, skips the forward's windowed passes
    (msssim_backward_values); without it they are recomputed."""
    cfg = _cfg(cfg, kw)
    xi, yi, b = _pair(x, y)
    p = cfg.to_c()
    flags = _ms_flags(renorm, cs_clamp, aggregation, coarse_separate)
    g = grad_score.to(device=x.device, dtype=torch.float32).reshape(b).contiguous()
    out = torch.empty(_as3(y).shape, dtype=torch.float32, device=x.device)
    ws = _workspace(workspace_size(cfg, L.OP_MSSSIM_BACKWARD, xi.dtype, xi.height, xi.width, b, n_scales),
                    x.device)
    if fwd is None:
        st = L.lib.msssim_backward(ctypes.byref(p), _weights(weights, n_scales), n_scales, flags, ctypes.byref(xi),
                                   ctypes.byref(yi), b, g.data_ptr(), out.data_ptr(), out.stride(1), out.stride(0),
                                   ws.data_ptr(), ws.numel(), _stream(x))
        L.check(st, "msssim_backward")
    else:
        score, cs = fwd
        score = score.to(device=x.device, dtype=torch.float32).reshape(b).contiguous()
        cs = cs.to(device=x.device, dtype=torch.float32).reshape(b, n_scales).contiguous()
        st = L.lib.msssim_backward_values(ctypes.byref(p), _weights(weights, n_scales), n_scales, flags,
                                          ctypes.byref(xi), ctypes.byref(yi), b, score.data_ptr(), cs.data_ptr(),
                                          g.data_ptr(), out.data_ptr(), out.stride(1), out.stride(0), ws.data_ptr(),
                                          ws.numel(), _stream(x))
        L.check(st, "msssim_backward_values")
    return out.reshape(y.shape)


def box_sums(x: torch.Tensor, y: torch.Tensor, k: int, stride: int = 1, algo: str = "auto") -> torch.Tensor:
    """int32 [5, B, Ho, Wo]: S1x, S1y, S2x, S2y, S12 of every k x k window."""
    xi, yi, b = _pair(x, y)
    cfg = SSIMConfig(window="box", k=k, stride=stride)
    ho, wo = map_shape(cfg, xi.height, xi.width)
    out = torch.empty((5, b, ho, wo), dtype=torch.int32, device=x.device)
    a = _ALGOS[algo]
    nws = 5 * b * (xi.width + 1) * (xi.height + 1) * 4 if a == L.ALGO_INTEGRAL_IMAGE else 0
    ws = _workspace(nws, x.device)
    st = L.lib.ssimx_box_sums(k, stride, a, ctypes.byref(xi), ctypes.byref(yi), b, out.data_ptr(), ws.data_ptr(),
                              ws.numel(), _stream(x))
    L.check(st, "ssimx_box_sums")
    return out


def integral_images(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """The five uint32 integral images as int32 bits [5, B, H+1, W+1]."""
    xi, yi, b = _pair(x, y)
    out = torch.empty((5, b, xi.height + 1, xi.width + 1), dtype=torch.int32, device=x.device)
    st = L.lib.ssimx_integral_images(ctypes.byref(xi), ctypes.byref(yi), b, out.data_ptr(), _stream(x))
    L.check(st, "ssimx_integral_images")
    return out


_POOLS = {"mean": L.POOL_MEAN, "cov": L.POOL_COV, "mean_dev": L.POOL_MEAN_DEV, "minkowski": L.POOL_MINKOWSKI,
          "dist_weighted": L.POOL_DIST_WEIGHTED, "five_number": L.POOL_FIVE_NUMBER, "percentile": L.POOL_PERCENTILE,
          "geometric": L.POOL_GEOMETRIC, "harmonic": L.POOL_HARMONIC, "median": L.POOL_MEDIAN,
          "w_am": L.POOL_WIN_AM, "w_gm": L.POOL_WIN_GM, "w_hm": L.POOL_WIN_HM, "w_cov": L.POOL_WIN_COV}


def pool(qmap: torch.Tensor, kind: str = "cov", p: float = 0.0, o: float = 1.0, r: float = 1.0) -> torch.Tensor:
    """Pooling of quality maps (B, H, W) or (H, W), float32 on the device ->
    float32 [B].  kind: mean | cov | mean_dev (p, o) | minkowski (p) |
    dist_weighted (p) | five_number | percentile (p in percent, r) | geometric
    | harmonic | median | w_am, w_gm, w_hm, w_cov (windows of p values; single
    row maps, see temporal_pool)."""
    m = qmap.unsqueeze(0) if qmap.dim() == 2 else qmap
    if m.dim() != 3 or m.dtype != torch.float32 or not m.is_cuda or m.stride(2) != 1:
        raise ValueError("qmap must be a float32 device tensor (B, H, W) with contiguous rows")
    pl = L.Pool(_POOLS[kind], float(p), float(o), float(r))
    b, h, w = m.shape
    n = ctypes.c_size_t()
    L.check(L.lib.ssimx_pool_workspace_size(ctypes.byref(pl), w, h, b, ctypes.byref(n)), "ssimx_pool_workspace_size")
    ws = _workspace(n.value, m.device)
    out = torch.empty(b, dtype=torch.float32, device=m.device)
    st = L.lib.ssimx_pool_map(ctypes.byref(pl), m.data_ptr(), w, h, m.stride(1), m.stride(0), b, out.data_ptr(),
                              ws.data_ptr(), ws.numel(), _stream(m))
    L.check(st, "ssimx_pool_map")
    return out


def temporal_pool(scores: torch.Tensor, kind: str = "mean", p: float = 0.0, o: float = 1.0,
                  r: float = 1.0) -> torch.Tensor:
    """Temporal pooling of frame scores (B, T) or (T,), float32 on the device
    -> float32 [B]: any pool kind applied to each row of T frame scores (for
    the windowed kinds p is the window length in frames)."""
    s = scores.unsqueeze(0) if scores.dim() == 1 else scores
    if s.dim() != 2:
        raise ValueError("scores must be (B, T) or (T,)")
    return pool(s.unsqueeze(1), kind, p, o, r)


def scaled_pooled_ssim(x: torch.Tensor, y: torch.Tensor, cfg: SSIMConfig | None = None, factor: int = 0,
                       pool: str = "mean", p: float = 0.0, o: float = 1.0, r: float = 1.0, **kw) -> torch.Tensor:
    """Down-sample by factor x factor block averages (0: max(1, ceil(H/256))),
    SSIM map, spatial pooling -> float32 [B]."""
    cfg = _cfg(cfg, kw)
    xi, yi, b = _pair(x, y)
    pc = cfg.to_c()
    pl = L.Pool(_POOLS[pool], float(p), float(o), float(r))
    n = ctypes.c_size_t()
    L.check(L.lib.ssimx_scaled_pooled_workspace_size(ctypes.byref(pc), int(factor), ctypes.byref(pl), xi.dtype,
                                                     xi.width, xi.height, b, ctypes.byref(n)),
            "ssimx_scaled_pooled_workspace_size")
    ws = _workspace(n.value, x.device)
    out = torch.empty(b, dtype=torch.float32, device=x.device)
    st = L.lib.ssimx_scaled_pooled_ssim(ctypes.byref(pc), int(factor), ctypes.byref(pl), ctypes.byref(xi),
                                        ctypes.byref(yi), b, out.data_ptr(), ws.data_ptr(), ws.numel(), _stream(x))
    L.check(st, "ssimx_scaled_pooled_ssim")
    return out


def enhanced_ssim(x: torch.Tensor, y: torch.Tensor, L_: float = 255.0, factor: int = 0) -> torch.Tensor:
    """The paper's Enhanced SSIM: 11x11 rectangular window at stride 5 on the
    pre-scaled luma, CoV pooling -> float32 [B] (0 for identical frames)."""
    cfg = SSIMConfig(window="box", k=11, stride=5, L=L_)
    return scaled_pooled_ssim(x, y, cfg, factor=factor, pool="cov")


def color_ssim(x_rgb: torch.Tensor, y_rgb: torch.Tensor, cfg: SSIMConfig | None = None, alpha: float = 0.125,
               beta: float = 0.125, return_channels: bool = False, **kw):
    """Channel-wise colour SSIM of planar RGB (B, 3, H, W) or (3, H, W):
    (SSIM_Y + alpha SSIM_Cb + beta SSIM_Cr) / (1 + alpha + beta) -> float32 [B]
    (and the per-channel scores [B, 3] with return_channels)."""
    cfg = _cfg(cfg, kw)
    xs = x_rgb.unsqueeze(0) if x_rgb.dim() == 3 else x_rgb
    ys = y_rgb.unsqueeze(0) if y_rgb.dim() == 3 else y_rgb
    if xs.shape != ys.shape or xs.dim() != 4 or xs.shape[1] != 3 or xs.dtype != ys.dtype:
        raise ValueError("x_rgb and y_rgb must be (B, 3, H, W) tensors of one shape and dtype")
    if xs.stride() != ys.stride() or xs.stride(3) != 1 or not xs.is_cuda:
        raise ValueError("planar device tensors with contiguous rows and equal strides expected")
    b, _, h, w = xs.shape
    pc = cfg.to_c()
    n = ctypes.c_size_t()
    L.check(L.lib.ssimx_color_workspace_size(ctypes.byref(pc), w, h, b, ctypes.byref(n)), "ssimx_color_workspace_size")
    ws = _workspace(n.value, xs.device)
    out = torch.empty(b, dtype=torch.float32, device=xs.device)
    ch = torch.empty((b, 3), dtype=torch.float32, device=xs.device)
    st = L.lib.ssimx_color_ssim(ctypes.byref(pc), float(alpha), float(beta), xs.data_ptr(), ys.data_ptr(),
                                _DTYPES[xs.dtype], w, h, xs.stride(2), xs.stride(1), xs.stride(0), b, out.data_ptr(),
                                ch.data_ptr(), ws.data_ptr(), ws.numel(), _stream(xs))
    L.check(st, "ssimx_color_ssim")
    return (out, ch) if return_channels else out


def _clip_pair(x: torch.Tensor, y: torch.Tensor):
    if x.dim() != 3:
        raise ValueError("clips must be (T, H, W) tensors")
    return _pair(x, y)


def ssim3d(x: torch.Tensor, y: torch.Tensor, kt: int, cfg: SSIMConfig | None = None, return_map: bool = False,
           **kw):
    """SSIM-3D of two clips (T, H, W) with the k x k x kt rectangular box:
    float32 [T-kt+1] mean of each map frame; with return_map also the float32
    map [T-kt+1, H-k+1, W-k+1].  The window defaults to the 11 x 11 box."""
    if cfg is None:
        kw.setdefault("window", "box")
    cfg = _cfg(cfg, kw)
    xi, yi, t = _clip_pair(x, y)
    p = cfg.to_c()
    n = ctypes.c_size_t()
    L.check(L.lib.ssimx_ssim3d_workspace_size(ctypes.byref(p), kt, xi.dtype, xi.width, xi.height, t, ctypes.byref(n)),
            "ssimx_ssim3d_workspace_size")
    ws = _workspace(n.value, x.device)
    to, ho, wo = t - kt + 1, xi.height - cfg.k + 1, xi.width - cfg.k + 1
    score = torch.empty(to, dtype=torch.float32, device=x.device)
    m = torch.empty((to, ho, wo), dtype=torch.float32, device=x.device) if return_map else None
    st = L.lib.ssimx_ssim3d(ctypes.byref(p), kt, ctypes.byref(xi), ctypes.byref(yi), t,
                            m.data_ptr() if m is not None else None, wo, ho * wo, score.data_ptr(),
                            ws.data_ptr(), ws.numel(), _stream(x))
    L.check(st, "ssimx_ssim3d")
    return (score, m) if return_map else score


def ms_ssim3d(x: torch.Tensor, y: torch.Tensor, kt: int, cfg: SSIMConfig | None = None, weights=MS_WEIGHTS,
              n_scales: int = 5, renorm: bool = False, cs_clamp: bool = False, aggregation: str = "product",
              return_cs: bool = False, coarse_separate: bool = False, **kw):
    """MS-SSIM-3D of two clips (T, H, W): float32 [T-kt+1] (and, with
    return_cs, [T-kt+1, n_scales] holding CS_1..CS_{M-1} and S_M per map
    frame).  The window defaults to the 11 x 11 box."""
    if cfg is None:
        kw.setdefault("window", "box")
    cfg = _cfg(cfg, kw)
    xi, yi, t = _clip_pair(x, y)
    p = cfg.to_c()
    flags = _ms_flags(renorm, cs_clamp, aggregation, coarse_separate)
    n = ctypes.c_size_t()
    L.check(L.lib.ssimx_msssim3d_workspace_size(ctypes.byref(p), kt, n_scales, xi.dtype, xi.width, xi.height, t,
                                                ctypes.byref(n)), "ssimx_msssim3d_workspace_size")
    ws = _workspace(n.value, x.device)
    to = t - kt + 1
    score = torch.empty(to, dtype=torch.float32, device=x.device)
    cs = torch.empty((to, n_scales), dtype=torch.float32, device=x.device) if return_cs else None
    st = L.lib.ssimx_msssim3d(ctypes.byref(p), kt, _weights(weights, n_scales), n_scales, flags, ctypes.byref(xi),
                              ctypes.byref(yi), t, score.data_ptr(), cs.data_ptr() if cs is not None else None,
                              ws.data_ptr(), ws.numel(), _stream(x))
    L.check(st, "ssimx_msssim3d")
    return (score, cs) if return_cs else score


def rgb_to_luma(rgb: torch.Tensor) -> torch.Tensor:
    """BT.601 luma of planar RGB (B, 3, H, W) or (3, H, W), float32/bfloat16
    -> float32 (B, H, W)."""
    t = rgb.unsqueeze(0) if rgb.dim() == 3 else rgb
    if t.dim() != 4 or t.shape[1] != 3 or t.stride(3) != 1 or not t.is_cuda:
        raise ValueError("rgb must be a device tensor (B, 3, H, W) with contiguous rows")
    dt = {torch.float32: L.F32, torch.bfloat16: L.BF16}.get(t.dtype)
    if dt is None:
        raise TypeError(f"unsupported dtype {t.dtype}")
    b, _, h, w = t.shape
    out = torch.empty((b, h, w), dtype=torch.float32, device=t.device)
    st = L.lib.ssimx_rgb_to_luma(t.data_ptr(), dt, w, h, t.stride(2), t.stride(1), t.stride(0), b, out.data_ptr(),
                                 _stream(t))
    L.check(st, "ssimx_rgb_to_luma")
    return out


def luma_grad_to_rgb(gy: torch.Tensor) -> torch.Tensor:
    """Adjoint of rgb_to_luma: float32 (B, H, W) -> float32 (B, 3, H, W)."""
    g = _as3(gy.to(torch.float32)).contiguous()
    b, h, w = g.shape
    out = torch.empty((b, 3, h, w), dtype=torch.float32, device=g.device)
    st = L.lib.ssimx_luma_grad_to_rgb(g.data_ptr(), w, h, b, out.data_ptr(), out.stride(2), out.stride(1),
                                      out.stride(0), _stream(g))
    L.check(st, "ssimx_luma_grad_to_rgb")
    return out


def autotune(cfg: SSIMConfig, dtype, h: int, w: int, batch: int = 1, device="cuda") -> int:
    best = ctypes.c_int(-1)
    dt = _DTYPES[dtype] if isinstance(dtype, torch.dtype) else int(dtype)
    st = L.lib.ssimx_autotune(ctypes.byref(cfg.to_c()), dt, w, h, batch,
                              torch.cuda.current_stream(torch.device(device)).cuda_stream, ctypes.byref(best))
    L.check(st, "ssimx_autotune")
    return best.value


def tune_cache_save(path: str) -> None:
    L.check(L.lib.ssimx_tune_cache_save(path.encode()), "ssimx_tune_cache_save")


def tune_cache_load(path: str) -> None:
    L.check(L.lib.ssimx_tune_cache_load(path.encode()), "ssimx_tune_cache_load")


def set_tile_override(tile: int) -> None:
    L.check(L.lib.ssimx_set_tile_override(int(tile)), "ssimx_set_tile_override")


def num_tile_configs() -> int:
    return L.lib.ssimx_num_tile_configs()


def _rgb(t: torch.Tensor) -> torch.Tensor:
    t = t.unsqueeze(0) if t.dim() == 3 else t
    if t.dim() != 4 or t.shape[1] != 3 or t.stride(3) != 1 or not t.is_cuda:
        raise ValueError("RGB planes must be a device tensor (B, 3, H, W) with contiguous rows")
    if t.dtype not in (torch.float32, torch.bfloat16):
        raise TypeError(f"unsupported dtype {t.dtype}")
    return t


def msssim_loss_rgb(ref: torch.Tensor, dis: torch.Tensor, cfg: SSIMConfig | None = None, weights=MS_WEIGHTS,
                    n_scales: int = 3, renorm: bool = True, cs_clamp: bool = False, aggregation: str = "product",
                    with_grad: bool = True, grad_dtype=None, coarse_separate: bool = False, **kw):
    """Loss mean_b(1 - MS-SSIM_b) on BT.601 luma of planar RGB (B, 3, H, W)
    float32/bfloat16, in one library call: returns (loss 0-dim float32,
    per-frame MS-SSIM [B], d loss / d dis in grad_dtype (default dis.dtype) or
    None)."""
    cfg = _cfg(cfg, kw)
    r, d = _rgb(ref), _rgb(dis)
    if r.shape != d.shape or r.dtype != d.dtype:
        raise ValueError("ref and dis must have equal shapes and dtypes")
    b, _, h, w = r.shape
    p = cfg.to_c()
    wts = _weights(weights, n_scales)
    flags = _ms_flags(renorm, cs_clamp, aggregation, coarse_separate)
    dt = _DTYPES[r.dtype]
    n = ctypes.c_size_t()
    L.check(L.lib.ssimx_msssim_loss_workspace_size(ctypes.byref(p), wts, n_scales, flags, dt, w, h, b,
                                                   ctypes.byref(n)), "ssimx_msssim_loss_workspace_size")
    ws = _workspace(n.value, r.device)
    loss = torch.empty(1, dtype=torch.float32, device=r.device)
    score = torch.empty(b, dtype=torch.float32, device=r.device)
    gdt = grad_dtype or d.dtype
    grad = torch.empty((b, 3, h, w), dtype=gdt, device=r.device) if with_grad else None
    st = L.lib.ssimx_msssim_loss_rgb(ctypes.byref(p), wts, n_scales, flags, r.data_ptr(), d.data_ptr(), dt, w, h,
                                     r.stride(2), r.stride(1), r.stride(0), b, loss.data_ptr(), score.data_ptr(),
                                     grad.data_ptr() if grad is not None else None, _DTYPES[gdt],
                                     grad.stride(2) if grad is not None else 0,
                                     grad.stride(1) if grad is not None else 0,
                                     grad.stride(0) if grad is not None else 0, ws.data_ptr(), ws.numel(), _stream(r))
    L.check(st, "ssimx_msssim_loss_rgb")
    return loss.reshape(()), score, grad


def msssim_loss_rgb_deferred(ref: torch.Tensor, dis: torch.Tensor, cfg: SSIMConfig | None = None,
                             weights=MS_WEIGHTS, n_scales: int = 3, renorm: bool = True, cs_clamp: bool = False,
                             aggregation: str = "product", coarse_separate: bool = False, **kw):
    """First half of msssim_loss_rgb for callers that learn the upstream
    later: returns (loss, per-frame MS-SSIM, state); state holds the
    workspace with the luma-level gradients for msssim_loss_rgb_grad."""
    cfg = _cfg(cfg, kw)
    r, d = _rgb(ref), _rgb(dis)
    if r.shape != d.shape or r.dtype != d.dtype:
        raise ValueError("ref and dis must have equal shapes and dtypes")
    b, _, h, w = r.shape
    p = cfg.to_c()
    wts = _weights(weights, n_scales)
    flags = _ms_flags(renorm, cs_clamp, aggregation, coarse_separate)
    dt = _DTYPES[r.dtype]
    n = ctypes.c_size_t()
    L.check(L.lib.ssimx_msssim_loss_workspace_size(ctypes.byref(p), wts, n_scales, flags, dt, w, h, b,
                                                   ctypes.byref(n)), "ssimx_msssim_loss_workspace_size")
    ws = _workspace(n.value, r.device)
    loss = torch.empty(1, dtype=torch.float32, device=r.device)
    score = torch.empty(b, dtype=torch.float32, device=r.device)
    st = L.lib.ssimx_msssim_loss_rgb_deferred(ctypes.byref(p), wts, n_scales, flags, r.data_ptr(), d.data_ptr(), dt,
                                              w, h, r.stride(2), r.stride(1), r.stride(0), b, loss.data_ptr(),
                                              score.data_ptr(), ws.data_ptr(), ws.numel(), _stream(r))
    L.check(st, "ssimx_msssim_loss_rgb_deferred")
    return loss.reshape(()), score, (p, wts, n_scales, flags, dt, (b, 3, h, w), ws)


def msssim_loss_rgb_grad(state, upstream: torch.Tensor | None = None, grad_dtype=torch.float32) -> torch.Tensor:
    """d loss / d dis (B, 3, H, W) in grad_dtype, times the device scalar
    `upstream` when given, from msssim_loss_rgb_deferred's state."""
    p, wts, n_scales, flags, dt, shape, ws = state
    b, _, h, w = shape
    grad = torch.empty(shape, dtype=grad_dtype, device=ws.device)
    up = None
    if upstream is not None:
        up = upstream.detach().to(device=ws.device, dtype=torch.float32).reshape(1).contiguous()
    st = L.lib.ssimx_msssim_loss_rgb_grad(ctypes.byref(p), wts, n_scales, flags, dt, w, h, b,
                                          up.data_ptr() if up is not None else None, grad.data_ptr(),
                                          _DTYPES[grad_dtype], grad.stride(2), grad.stride(1), grad.stride(0),
                                          ws.data_ptr(), ws.numel(), _stream(grad))
    L.check(st, "ssimx_msssim_loss_rgb_grad")
    return grad


class LossPlan:
    """The MS-SSIM loss of msssim_loss_rgb for one shape, replayed as one HIP
    graph per run (the plan owns its workspace; inputs and outputs may be new
    tensors on every run).  Runs must be issued on one stream."""

    def __init__(self, cfg: SSIMConfig | None, dtype, batch: int, height: int, width: int, weights=MS_WEIGHTS,
                 n_scales: int = 3, renorm: bool = True, cs_clamp: bool = False, aggregation: str = "product",
                 grad_dtype=None, device=None, coarse_separate: bool = False):
        self.cfg = cfg or SSIMConfig()
        self.dtype, self.grad_dtype = dtype, grad_dtype or dtype
        self.shape = (batch, 3, height, width)
        self.device = torch.device(device or "cuda")
        p = self.cfg.to_c()
        self._h = ctypes.c_void_p()
        st = L.lib.ssimx_loss_plan_create(ctypes.byref(p), _weights(weights, n_scales), n_scales,
                                          _ms_flags(renorm, cs_clamp, aggregation, coarse_separate),
                                          _DTYPES[dtype],
                                          _DTYPES[self.grad_dtype], width, height, batch, ctypes.byref(self._h))
        L.check(st, "ssimx_loss_plan_create")

    def run(self, ref: torch.Tensor, dis: torch.Tensor, with_grad: bool = True):
        """(loss 0-dim, per-frame MS-SSIM [B], gradient or None), as msssim_loss_rgb."""
        r, d = _rgb(ref), _rgb(dis)
        if tuple(r.shape) != self.shape or tuple(d.shape) != self.shape or r.dtype != self.dtype or \
                d.dtype != self.dtype:
            raise ValueError(f"the plan takes {self.shape} {self.dtype} planes")
        b, _, h, w = self.shape
        loss = torch.empty(1, dtype=torch.float32, device=r.device)
        score = torch.empty(b, dtype=torch.float32, device=r.device)
        grad = torch.empty((b, 3, h, w), dtype=self.grad_dtype, device=r.device) if with_grad else None
        st = L.lib.ssimx_loss_plan_run(self._h, r.data_ptr(), d.data_ptr(), r.stride(2), r.stride(1), r.stride(0),
                                       loss.data_ptr(), score.data_ptr(),
                                       grad.data_ptr() if grad is not None else None,
                                       grad.stride(2) if grad is not None else 0,
                                       grad.stride(1) if grad is not None else 0,
                                       grad.stride(0) if grad is not None else 0, _stream(r))
        L.check(st, "ssimx_loss_plan_run")
        return loss.reshape(()), score, grad

    def close(self):
        if self._h:
            torch.cuda.synchronize(self.device)
            L.lib.ssimx_loss_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """Ragged batch of independent pairs: one persistent, graph-captured
    launch per run().  pairs: list of dicts {ref, dis, cfg (SSIMConfig),
    map (optional float32 [Ho, Wo] output)}; the tensors are kept alive by
    the plan."""

    def __init__(self, pairs, device=None):
        self._keep = []
        arr = (L.Pair * len(pairs))()
        dev = None
        for i, pr in enumerate(pairs):
            x, y = pr["ref"], pr["dis"]
            if x.dim() != 2:
                raise ValueError("batch-plan pairs are single (H, W) planes")
            xi, yi, _ = _pair(x, y)
            cfg = pr.get("cfg") or SSIMConfig()
            m = pr.get("map")
            arr[i].ref = xi
            arr[i].dis = yi
            arr[i].p = cfg.to_c()
            arr[i].map_out = m.data_ptr() if m is not None else None
            arr[i].map_pitch = m.stride(0) if m is not None else 0
            self._keep += [x, y, m]
            dev = x.device
        self.device = device or dev
        self.n = len(pairs)
        self._h = ctypes.c_void_p()
        st = L.lib.ssimx_plan_create(arr, self.n, torch.cuda.current_stream(self.device).cuda_stream,
                                     ctypes.byref(self._h))
        L.check(st, "ssimx_plan_create")

    def info(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        L.check(L.lib.ssimx_plan_info(self._h, ctypes.byref(a), ctypes.byref(b)), "ssimx_plan_info")
        return a.value, b.value

    def run(self, out: torch.Tensor | None = None) -> torch.Tensor:
        out = out if out is not None else torch.empty(self.n, dtype=torch.float32, device=self.device)
        st = L.lib.ssimx_plan_run(self._h, out.data_ptr(), torch.cuda.current_stream(self.device).cuda_stream)
        L.check(st, "ssimx_plan_run")
        return out

    def run_unbatched(self, out: torch.Tensor | None = None) -> torch.Tensor:
        out = out if out is not None else torch.empty(self.n, dtype=torch.float32, device=self.device)
        st = L.lib.ssimx_plan_run_unbatched(self._h, out.data_ptr(),
                                            torch.cuda.current_stream(self.device).cuda_stream)
        L.check(st, "ssimx_plan_run_unbatched")
        return out

    def close(self):
        if self._h:
            L.lib.ssimx_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _unused():
    return math
