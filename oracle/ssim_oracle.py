"""FP64 CPU oracle for the SSIM / MS-SSIM hot path.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain, obviously-correct
definition the HIP path is checked against.  Only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product
path (the C-ABI library and its Python binding) never does, and this module
imports nothing from the product package.

Paper: Venkataramanan, Wu, Bovik, Katsavounidis, Shahid, "A Hitchhiker's Guide
to Structural Similarity" (arXiv 2101.06354).  Every function cites the passage
it writes out.  All arithmetic is float64 (integer sums are exact int64).

Readings taken where the paper is silent (each is also listed in the design
notes of the repository):
  * Gaussian taps are sampled at integer offsets from the window centre and the
    1-D taps are normalised to sum to one; the 2-D window is their outer
    product (Background section: the weights "sum to unity").
  * The window W_ij is anchored at its top-left pixel (i, j) (Background).
  * Pooling divides by the number of computed map positions, not by the image
    size (the valid map is smaller than the image).
  * Border handling ('valid' | 'zero' | 'reflect') follows the border column of
    the table of implementation features; 'reflect' is half-sample symmetric
    (x[-1] = x[0]) and the padded ("same") extent is floor((k-1)/2) before and
    ceil((k-1)/2) after.
  * Stride s evaluates windows at (s*i, s*j) from origin (0, 0) (Effect of
    stride subsection).
  * MS-SSIM: 2x2 average pooling with floor of odd sizes; CS_j = mean cs map at
    scales j < M, S_M = mean(l*cs) at the coarsest scale M; score =
    S_M^{w_M} * prod_j CS_j^{w_j}; weights renormalised to sum one only when
    asked (the Daala-fast description).  Negative CS_j with a fractional
    exponent gives NaN unless clamping is asked for.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "SSIMParams", "constants", "window_1d", "window_2d", "pad_image",
    "map_shape", "moments_direct", "moments_separable", "ssim_terms",
    "ssim_map", "ssim_pooled", "box_sums_direct", "integral_images",
    "box_sums_integral", "box_stats", "downsample2x2", "pyramid",
    "msssim", "ssim_map_backward", "ssim_pooled_backward",
    "msssim_backward", "rgb_to_y_bt601", "y_grad_to_rgb_bt601",
    "MS_WEIGHTS", "pool_mean", "pool_cov", "pool_md", "pool_minkowski",
    "pool_distortion_weighted", "pool_five_number", "pool_percentile",
    "scale_factor", "downsample_avg", "scaled_pooled_ssim", "enhanced_ssim",
    "rgb_to_ycbcr_bt709", "color_ssim", "BT709_Y", "BT709_CB", "BT709_CR",
    "box_sums3d", "ssim3d_map", "ssim3d", "msssim3d",
    "pool_geometric", "pool_harmonic", "pool_median", "pool_windowed",
    "lw_weights", "pool_luminance_weighted",
]

# Exponents of the original five-scale MS-SSIM, as used by the configurations
# that reproduce it (Versions of SSIM section, MS-SSIM implementation list).
MS_WEIGHTS = (0.0448, 0.2856, 0.3001, 0.2363, 0.1333)


def constants(K1: float, K2: float, L: float) -> tuple[float, float]:
    """C1 = (K1 L)^2, C2 = (K2 L)^2 (Background section, saturation constants)."""
    return (K1 * L) ** 2, (K2 * L) ** 2


@dataclass
class SSIMParams:
    """The paper's statement of the problem: window type, size and sigma,
    saturation constants, stride and border handling."""
    window: str = "gaussian"          # 'gaussian' | 'box'
    k: int = 11
    sigma: float = 1.5
    C1: float = field(default_factory=lambda: constants(0.01, 0.03, 255.0)[0])
    C2: float = field(default_factory=lambda: constants(0.01, 0.03, 255.0)[1])
    stride: int = 1
    padding: str = "valid"            # 'valid' | 'zero' | 'reflect'

    def check(self) -> None:
        if self.window not in ("gaussian", "box"):
            raise ValueError("window must be 'gaussian' or 'box'")
        if self.k < 1:
            raise ValueError("k must be >= 1")
        if self.window == "gaussian" and (self.k % 2 == 0 or self.sigma <= 0):
            raise ValueError("a Gaussian window needs odd k and sigma > 0")
        if self.stride < 1:
            raise ValueError("stride must be >= 1")
        if self.padding not in ("valid", "zero", "reflect"):
            raise ValueError("padding must be 'valid', 'zero' or 'reflect'")


# --------------------------------------------------------------------------
# Window (Background section; recommended recipe k=11, sigma=1.5)
# --------------------------------------------------------------------------
def window_1d(window: str, k: int, sigma: float = 1.5) -> np.ndarray:
    """1-D taps g_t, t = 0..k-1, summing to one.

    Gaussian: g_t proportional to exp(-(t-c)^2 / (2 sigma^2)), c = (k-1)/2.
    Box: g_t = 1/k, so the 2-D weight is 1/k^2 (Performance-Efficiency
    subsection, rectangular window).
    """
    if window == "box":
        return np.full(k, 1.0 / k, dtype=np.float64)
    c = (k - 1) / 2.0
    t = np.arange(k, dtype=np.float64) - c
    g = np.exp(-(t * t) / (2.0 * sigma * sigma))
    return g / math.fsum(g)


def window_2d(window: str, k: int, sigma: float = 1.5) -> np.ndarray:
    """w(m, n) = g_m g_n; sums to one (Background section)."""
    g = window_1d(window, k, sigma)
    return np.outer(g, g)


# --------------------------------------------------------------------------
# Border handling and output geometry
# --------------------------------------------------------------------------
def pad_image(img: np.ndarray, k: int, padding: str) -> np.ndarray:
    """Extend a 2-D plane for 'zero' or 'reflect' border handling.

    'valid' returns the plane unchanged.  Otherwise floor((k-1)/2) rows/cols
    are added before and ceil((k-1)/2) after, so a stride-1 map has the size of
    the image.  'reflect' is half-sample symmetric (numpy 'symmetric').
    """
    if padding == "valid":
        return img
    before = (k - 1) // 2
    after = (k - 1) - before
    if padding == "zero":
        return np.pad(img, ((before, after), (before, after)), mode="constant")
    if padding == "reflect":
        return np.pad(img, ((before, after), (before, after)), mode="symmetric")
    raise ValueError(padding)


def map_shape(h: int, w: int, k: int, stride: int, padding: str) -> tuple[int, int]:
    """Number of window positions: floor((H' - k)/s) + 1 per axis, H' the
    (padded) extent; 0 when the window does not fit."""
    hp = h if padding == "valid" else h + k - 1
    wp = w if padding == "valid" else w + k - 1
    ho = (hp - k) // stride + 1 if hp >= k else 0
    wo = (wp - k) // stride + 1 if wp >= k else 0
    return ho, wo


# --------------------------------------------------------------------------
# Local statistics (Background section, eqs. local_means .. local_corr)
# --------------------------------------------------------------------------
def moments_direct(x: np.ndarray, y: np.ndarray, w2: np.ndarray, stride: int = 1):
    """Weighted raw moments by the direct O(k^2) sum over every window offset.

    Returns (mu_x, mu_y, E[x^2], E[y^2], E[xy]) at the window anchors
    (s*i, s*j) of already-padded planes.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    k = w2.shape[0]
    ho = (x.shape[0] - k) // stride + 1
    wo = (x.shape[1] - k) // stride + 1
    acc = [np.zeros((ho, wo)) for _ in range(5)]
    for m in range(k):
        for n in range(k):
            xs = x[m:m + stride * (ho - 1) + 1:stride, n:n + stride * (wo - 1) + 1:stride]
            ys = y[m:m + stride * (ho - 1) + 1:stride, n:n + stride * (wo - 1) + 1:stride]
            wmn = w2[m, n]
            acc[0] += wmn * xs
            acc[1] += wmn * ys
            acc[2] += wmn * xs * xs
            acc[3] += wmn * ys * ys
            acc[4] += wmn * xs * ys
    return tuple(acc)


def _filter_rows(a: np.ndarray, g: np.ndarray, stride: int) -> np.ndarray:
    """out[r, j] = sum_n g[n] a[r, s*j + n]."""
    k = g.shape[0]
    wo = (a.shape[1] - k) // stride + 1
    win = np.lib.stride_tricks.sliding_window_view(a, k, axis=1)[:, : stride * (wo - 1) + 1 : stride, :]
    return win @ g


def moments_separable(x: np.ndarray, y: np.ndarray, g: np.ndarray, stride: int = 1):
    """Same five moments with the separable window w = g g^T: a 1-D pass along
    rows, then along columns (valid only for the outer-product window of the
    Background section)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    out = []
    for a in (x, y, x * x, y * y, x * y):
        h = _filter_rows(a, g, stride)
        v = _filter_rows(h.T, g, stride).T
        out.append(v)
    return tuple(out)


def ssim_terms(mu_x, mu_y, exx, eyy, exy, C1: float, C2: float):
    """Luminance, contrast-structure and quality maps.

    sigma^2 = E[I^2] - mu^2, sigma_12 = E[I1 I2] - mu1 mu2 (eqs. local_means ..
    local_corr); l (eq. lum_term); cs with C3 = C2/2; Q = l * cs (Background
    section).
    """
    sxx = exx - mu_x * mu_x
    syy = eyy - mu_y * mu_y
    sxy = exy - mu_x * mu_y
    with np.errstate(divide="ignore", invalid="ignore"):
        l = (2.0 * mu_x * mu_y + C1) / (mu_x * mu_x + mu_y * mu_y + C1)
        cs = (2.0 * sxy + C2) / (sxx + syy + C2)
    return l, cs, l * cs, (sxx, syy, sxy)


def _as_f64(img) -> np.ndarray:
    return np.asarray(img).astype(np.float64)


def ssim_map(x, y, p: SSIMParams | None = None, form: str = "separable") -> dict:
    """SSIM quality map of one plane pair (Background section).

    Box windows on integer planes use exact integer window sums and the
    statistics of the Performance-Efficiency subsection (eqs. mean_from_sum ..
    corr_from_sum); all other cases use weighted float64 moments, either by
    the direct double sum (form='direct') or separably (form='separable').
    Returns a dict with 'map', 'l', 'cs', 'mu_x', 'mu_y', 'sxx', 'syy', 'sxy'.
    """
    p = p or SSIMParams()
    p.check()
    ho, wo = map_shape(x.shape[0], x.shape[1], p.k, p.stride, p.padding)
    if ho < 1 or wo < 1:
        raise ValueError("image smaller than the window")
    integer = np.issubdtype(np.asarray(x).dtype, np.integer) and np.issubdtype(np.asarray(y).dtype, np.integer)
    xp = pad_image(_as_f64(x), p.k, p.padding)
    yp = pad_image(_as_f64(y), p.k, p.padding)
    if p.window == "box" and integer:
        xi = pad_image(np.asarray(x).astype(np.int64), p.k, p.padding)
        yi = pad_image(np.asarray(y).astype(np.int64), p.k, p.padding)
        sums = box_sums_direct(xi, yi, p.k, p.stride)
        mu_x, mu_y, sxx, syy, sxy = box_stats(sums, p.k)
        exx = sxx + mu_x * mu_x
        eyy = syy + mu_y * mu_y
        exy = sxy + mu_x * mu_y
        with np.errstate(divide="ignore", invalid="ignore"):
            l = (2.0 * mu_x * mu_y + p.C1) / (mu_x * mu_x + mu_y * mu_y + p.C1)
            cs = (2.0 * sxy + p.C2) / (sxx + syy + p.C2)
        q = l * cs
    else:
        if form == "direct":
            mom = moments_direct(xp, yp, window_2d(p.window, p.k, p.sigma), p.stride)
        else:
            mom = moments_separable(xp, yp, window_1d(p.window, p.k, p.sigma), p.stride)
        mu_x, mu_y, exx, eyy, exy = mom
        l, cs, q, (sxx, syy, sxy) = ssim_terms(mu_x, mu_y, exx, eyy, exy, p.C1, p.C2)
    assert q.shape == (ho, wo)
    return {"map": q, "l": l, "cs": cs, "mu_x": mu_x, "mu_y": mu_y,
            "sxx": sxx, "syy": syy, "sxy": sxy}


def mean_pool(q: np.ndarray) -> float:
    """Mean SSIM: average of the quality map (Background section), summed
    with correct rounding."""
    return math.fsum(np.asarray(q, dtype=np.float64).ravel().tolist()) / q.size


def ssim_pooled(x, y, p: SSIMParams | None = None) -> float:
    return mean_pool(ssim_map(x, y, p)["map"])


# --------------------------------------------------------------------------
# Rectangular windows: integer sums and integral images
# (Performance-Efficiency subsection, eqs. integral_image_start ..
# corr_from_sum)
# --------------------------------------------------------------------------
def box_sums_direct(x: np.ndarray, y: np.ndarray, k: int, stride: int = 1):
    """Exact int64 window sums S1x, S1y, S2x, S2y, S12 over k x k windows at
    (s*i, s*j), by summing every window offset."""
    x = np.asarray(x).astype(np.int64)
    y = np.asarray(y).astype(np.int64)
    ho = (x.shape[0] - k) // stride + 1
    wo = (x.shape[1] - k) // stride + 1
    acc = [np.zeros((ho, wo), dtype=np.int64) for _ in range(5)]
    for m in range(k):
        for n in range(k):
            xs = x[m:m + stride * (ho - 1) + 1:stride, n:n + stride * (wo - 1) + 1:stride]
            ys = y[m:m + stride * (ho - 1) + 1:stride, n:n + stride * (wo - 1) + 1:stride]
            acc[0] += xs
            acc[1] += ys
            acc[2] += xs * xs
            acc[3] += ys * ys
            acc[4] += xs * ys
    return tuple(acc)


def integral_images(x: np.ndarray, y: np.ndarray):
    """The five summed-area tables of eq. integral_image_start and the four
    equations after it, with the zero first row and column, reduced modulo
    2^32 (uint32).  Shape (H+1, W+1) each; entry (i, j) holds the sum over
    rows < i and cols < j."""
    x = np.asarray(x).astype(np.int64)
    y = np.asarray(y).astype(np.int64)
    out = []
    for a in (x, y, x * x, y * y, x * y):
        s = np.zeros((a.shape[0] + 1, a.shape[1] + 1), dtype=np.int64)
        s[1:, 1:] = a.cumsum(axis=0).cumsum(axis=1)
        out.append((s % (1 << 32)).astype(np.uint32))
    return tuple(out)


def box_sums_integral(sats, k: int, stride: int, ho: int, wo: int):
    """Four-corner window sums (eq. integral_image_end) in modulo-2^32
    arithmetic, returned as int64.  Exact whenever every true window sum is
    below 2^31 (it is for 8- and 10-bit planes with k <= 45)."""
    res = []
    i = np.arange(ho)[:, None] * stride
    j = np.arange(wo)[None, :] * stride
    for s in sats:
        s64 = s.astype(np.int64)
        v = s64[i + k, j + k] + s64[i, j] - s64[i + k, j] - s64[i, j + k]
        res.append(v % (1 << 32))
    return tuple(res)


def box_stats(sums, k: int):
    """Local statistics from window sums (eqs. mean_from_sum .. corr_from_sum),
    with the variance numerators k^2 S2 - S1^2 formed exactly in integers."""
    s1x, s1y, s2x, s2y, s12 = (np.asarray(s, dtype=np.int64) for s in sums)
    kk = k * k
    k4 = float(kk * kk)
    mu_x = s1x.astype(np.float64) / kk
    mu_y = s1y.astype(np.float64) / kk
    sxx = (kk * s2x - s1x * s1x).astype(np.float64) / k4
    syy = (kk * s2y - s1y * s1y).astype(np.float64) / k4
    sxy = (kk * s12 - s1x * s1y).astype(np.float64) / k4
    return mu_x, mu_y, sxx, syy, sxy


# --------------------------------------------------------------------------
# MS-SSIM (Introduction; MS-SSIM implementation list: 2x2 average pooling,
# exponent renormalisation when fewer scales are used)
# --------------------------------------------------------------------------
def downsample2x2(a: np.ndarray) -> np.ndarray:
    """Average of each aligned 2x2 block; an odd last row/column is dropped."""
    a = np.asarray(a, dtype=np.float64)
    h2, w2 = a.shape[0] // 2, a.shape[1] // 2
    a = a[: 2 * h2, : 2 * w2]
    return 0.25 * (a[0::2, 0::2] + a[0::2, 1::2] + a[1::2, 0::2] + a[1::2, 1::2])


def pyramid(a: np.ndarray, n_scales: int) -> list[np.ndarray]:
    lv = [np.asarray(a)]
    for _ in range(n_scales - 1):
        lv.append(downsample2x2(lv[-1]))
    return lv


def _ms_weights(weights, n_scales: int, renorm: bool) -> np.ndarray:
    w = np.asarray(weights[:n_scales], dtype=np.float64)
    if renorm:
        w = w / math.fsum(w.tolist())
    return w


def msssim(x, y, p: SSIMParams | None = None, weights=MS_WEIGHTS, n_scales: int = 5,
           renorm: bool = False, cs_clamp: bool = False, aggregation: str = "product",
           coarse_separate: bool = False) -> dict:
    """Multi-scale SSIM: cs at every scale, luminance at the coarsest only,
    combined as an exponentially weighted product (Introduction; the
    'Product' aggregation of the Versions of SSIM section).

    aggregation="sum" is the 'Sum' aggregation of the same section and of the
    Scikit-Video notes in the Implementations section: the same per-scale
    terms (CS_j for j < M, S_M at the coarsest scale) in a weighted average
    whose weights are the exponents normalised to sum to one (always, so
    `renorm` has no effect; `cs_clamp` has none either, as no power is taken).

    The paper describes the coarsest term without printing it; by default it
    is the mean of l*cs there.  coarse_separate=True takes the other reading,
    mean(l) * mean(cs) at the coarsest scale.

    Returns {'score', 'cs' (list of CS_j, j < M), 's_M', 'weights'}.
    """
    p = p or SSIMParams()
    if aggregation not in ("product", "sum"):
        raise ValueError(f"unknown aggregation {aggregation!r}")
    w = _ms_weights(weights, n_scales, renorm or aggregation == "sum")
    xs = pyramid(_as_f64(x), n_scales)
    ys = pyramid(_as_f64(y), n_scales)
    cs_vals = []
    s_m = None
    for j in range(n_scales):
        r = ssim_map(xs[j], ys[j], p)
        if j < n_scales - 1:
            cs_vals.append(mean_pool(r["cs"]))
        elif coarse_separate:
            s_m = mean_pool(r["l"]) * mean_pool(r["cs"])
        else:
            s_m = mean_pool(r["map"])
    score = _ms_combine(cs_vals, s_m, w, cs_clamp, aggregation)
    return {"score": score, "cs": cs_vals, "s_M": s_m, "weights": w}


def _ms_combine(cs_vals, s_m, w, cs_clamp: bool, aggregation: str) -> float:
    """S_M^{w_M} prod_j CS_j^{w_j}, or sum_j w_j CS_j + w_M S_M ('Sum')."""
    if aggregation == "sum":
        return math.fsum([w[j] * c for j, c in enumerate(cs_vals)] + [w[-1] * s_m])
    score = 1.0
    with np.errstate(invalid="ignore"):
        for j, c in enumerate(cs_vals):
            c = max(c, 0.0) if cs_clamp else c
            score *= float(np.power(c, w[j])) if c >= 0 else float("nan")
        sm = max(s_m, 0.0) if cs_clamp else s_m
        score *= float(np.power(sm, w[-1])) if sm >= 0 else float("nan")
    return score


# --------------------------------------------------------------------------
# Adjoint with respect to the distorted plane y (derivative of the
# Background-section definitions; the paper only mentions MS-SSIM as a
# training objective).
# --------------------------------------------------------------------------
def _unpad_adjoint(gp: np.ndarray, shape, k: int, padding: str) -> np.ndarray:
    """Adjoint of pad_image: drop zero-padded cells, fold reflected cells back
    onto their source pixels."""
    if padding == "valid":
        return gp
    h, w = shape
    before = (k - 1) // 2
    if padding == "zero":
        return gp[before:before + h, before:before + w].copy()

    def src(n, length):
        idx = np.arange(n) - before
        # half-sample symmetric reflection, period 2*length
        idx = np.mod(idx, 2 * length)
        return np.where(idx < length, idx, 2 * length - 1 - idx)

    ri = src(gp.shape[0], h)
    ci = src(gp.shape[1], w)
    tmp = np.zeros((h, gp.shape[1]))
    np.add.at(tmp, ri, gp)
    out = np.zeros((h, w))
    np.add.at(out.T, ci, tmp.T)
    return out


def ssim_map_backward(x, y, grad_map: np.ndarray, p: SSIMParams | None = None,
                      term: str = "ssim") -> np.ndarray:
    """dL/dy for L = sum_p grad_map(p) * T(p), T = Q (term='ssim') or cs
    (term='cs').

    With A1 = 2 mu_x mu_y + C1, B1 = mu_x^2 + mu_y^2 + C1, A2 = 2 s_xy + C2,
    B2 = s_xx + s_yy + C2 and the raw moments mu_y, E[xy], E[y^2]:
      dQ/dmu_y  = cs (2 mu_x - 2 mu_y l)/B1 + l (2 mu_y cs - 2 mu_x)/B2
      dQ/dE[xy] = 2 l / B2,   dQ/dE[y^2] = -Q / B2
      dcs/dmu_y = (2 mu_y cs - 2 mu_x)/B2, dcs/dE[xy] = 2/B2, dcs/dE[y^2] = -cs/B2
    and dL/dy(q) = sum_p w(q - s p) [a(p) + b(p) x(q) + 2 c(p) y(q)], the
    transposed window correlation, followed by the border adjoint.
    """
    p = p or SSIMParams()
    xp = pad_image(_as_f64(x), p.k, p.padding)
    yp = pad_image(_as_f64(y), p.k, p.padding)
    w2 = window_2d(p.window, p.k, p.sigma)
    mu_x, mu_y, exx, eyy, exy = moments_direct(xp, yp, w2, p.stride)
    l, cs, q, (sxx, syy, sxy) = ssim_terms(mu_x, mu_y, exx, eyy, exy, p.C1, p.C2)
    b1 = mu_x * mu_x + mu_y * mu_y + p.C1
    b2 = sxx + syy + p.C2
    g = np.asarray(grad_map, dtype=np.float64)
    if term == "ssim":
        a = g * (cs * (2 * mu_x - 2 * mu_y * l) / b1 + l * (2 * mu_y * cs - 2 * mu_x) / b2)
        b = g * 2 * l / b2
        c = -g * q / b2
    elif term == "cs":
        a = g * (2 * mu_y * cs - 2 * mu_x) / b2
        b = g * 2 / b2
        c = -g * cs / b2
    elif term == "l":
        a = g * (2 * mu_x - 2 * mu_y * l) / b1
        b = np.zeros_like(a)
        c = np.zeros_like(a)
    else:
        raise ValueError(term)
    ho, wo = q.shape
    s = p.stride
    gp = np.zeros_like(yp)
    for m in range(p.k):
        for n in range(p.k):
            sl = (slice(m, m + s * (ho - 1) + 1, s), slice(n, n + s * (wo - 1) + 1, s))
            gp[sl] += w2[m, n] * (a + b * xp[sl] + 2.0 * c * yp[sl])
    return _unpad_adjoint(gp, np.asarray(y).shape, p.k, p.padding)


def ssim_pooled_backward(x, y, grad_score: float = 1.0, p: SSIMParams | None = None) -> np.ndarray:
    """dL/dy for L = grad_score * mean(Q)."""
    p = p or SSIMParams()
    ho, wo = map_shape(np.asarray(x).shape[0], np.asarray(x).shape[1], p.k, p.stride, p.padding)
    g = np.full((ho, wo), grad_score / (ho * wo))
    return ssim_map_backward(x, y, g, p, "ssim")


def _downsample_adjoint(gc: np.ndarray, fine_shape) -> np.ndarray:
    """Transpose of downsample2x2: each coarse value sends 1/4 to its four
    parents; a dropped odd row/column receives zero."""
    out = np.zeros(fine_shape)
    h2, w2 = gc.shape
    q = 0.25 * gc
    out[0:2 * h2:2, 0:2 * w2:2] += q
    out[0:2 * h2:2, 1:2 * w2:2] += q
    out[1:2 * h2:2, 0:2 * w2:2] += q
    out[1:2 * h2:2, 1:2 * w2:2] += q
    return out


def msssim_backward(x, y, grad_score: float = 1.0, p: SSIMParams | None = None,
                    weights=MS_WEIGHTS, n_scales: int = 5, renorm: bool = False,
                    cs_clamp: bool = False, aggregation: str = "product",
                    coarse_separate: bool = False) -> np.ndarray:
    """dL/dy for L = grad_score * MS-SSIM(x, y), by the chain rule through the
    weighted product (or, for the 'Sum' aggregation, the weighted average) and
    the 2x2 pyramid, coarse to fine."""
    p = p or SSIMParams()
    fwd = msssim(x, y, p, weights, n_scales, renorm, cs_clamp, aggregation, coarse_separate)
    w = fwd["weights"]
    ms = fwd["score"]
    xs = pyramid(_as_f64(x), n_scales)
    ys = pyramid(_as_f64(y), n_scales)
    g_next = None
    for j in range(n_scales - 1, -1, -1):
        ho, wo = map_shape(xs[j].shape[0], xs[j].shape[1], p.k, p.stride, p.padding)
        if j == n_scales - 1:
            val, term = fwd["s_M"], "ssim"
        else:
            val, term = fwd["cs"][j], "cs"
        if aggregation == "sum":
            dval = grad_score * w[j]
        elif cs_clamp and val <= 0:
            dval = 0.0
        else:
            dval = grad_score * ms * w[j] / val
        if j == n_scales - 1 and coarse_separate:
            # S_M = mean(l) mean(cs): dS_M = mean(cs) dmean(l) + mean(l) dmean(cs)
            r = ssim_map(xs[j], ys[j], p)
            lm, cm = mean_pool(r["l"]), mean_pool(r["cs"])
            gj = (ssim_map_backward(xs[j], ys[j], np.full((ho, wo), dval * cm / (ho * wo)), p, "l")
                  + ssim_map_backward(xs[j], ys[j], np.full((ho, wo), dval * lm / (ho * wo)), p, "cs"))
        else:
            gm = np.full((ho, wo), dval / (ho * wo))
            gj = ssim_map_backward(xs[j], ys[j], gm, p, term)
        if g_next is not None:
            gj = gj + _downsample_adjoint(g_next, xs[j].shape)
        g_next = gj
    return g_next


# --------------------------------------------------------------------------
# Colour to luma for the differentiable-loss workload.  The paper prints the
# BT.709 matrix (Channel-wise SSIM subsection); the training workload uses
# BT.601 luma weights.
# --------------------------------------------------------------------------
BT601 = (0.299, 0.587, 0.114)


def rgb_to_y_bt601(rgb: np.ndarray) -> np.ndarray:
    """Y = 0.299 R + 0.587 G + 0.114 B over a leading channel axis of 3."""
    rgb = np.asarray(rgb, dtype=np.float64)
    return BT601[0] * rgb[0] + BT601[1] * rgb[1] + BT601[2] * rgb[2]


def y_grad_to_rgb_bt601(gy: np.ndarray) -> np.ndarray:
    gy = np.asarray(gy, dtype=np.float64)
    return np.stack([BT601[0] * gy, BT601[1] * gy, BT601[2] * gy])


# --------------------------------------------------------------------------
# Spatial pooling of a quality map (Spatial and Temporal Aggregation section).
# q is the map of one frame; n = number of map positions.  Readings:
#   * standard deviations are population ones (divide by n), as the mean-
#     deviation equation with p = 2 makes them;
#   * the mean-deviation Minkowski distance uses |Q - mu|^p;
#   * distortion-weighted pooling with all weights zero (every Q = 1) gives 1;
#   * quartiles and the median are linear interpolation between the two
#     nearest order statistics at rank (n - 1) q;
#   * percentile pooling divides the m = ceil(p_s n / 100) smallest values by
#     r_s (ties at the cut do not change the result).
# --------------------------------------------------------------------------
def pool_mean(q: np.ndarray) -> float:
    """Arithmetic mean of the map (the baseline pooling)."""
    return mean_pool(q)


def lw_weights(mu1: np.ndarray, a_s: float, b_s: float) -> np.ndarray:
    """Luminance weights of the Luminance-Weighted Pooling subsection: 0 where
    the reference's local mean mu1 lies below a_s, (mu1 - a_s)/b_s on
    [a_s, a_s + b_s), 1 from a_s + b_s on (b_s = 0: a step at a_s)."""
    mu1 = np.asarray(mu1, dtype=np.float64)
    w = np.ones_like(mu1)
    w[mu1 < a_s] = 0.0
    if b_s > 0:
        mid = (mu1 >= a_s) & (mu1 < a_s + b_s)
        w[mid] = (mu1[mid] - a_s) / b_s
    return w


def pool_luminance_weighted(x, y, p: SSIMParams | None = None, a_s: float = 0.0, b_s: float = 0.0) -> float:
    """S_LW = (1/MN) sum_x w_LW(mu1(x)) Q(x): the weighted sum divided by the
    number of map positions, not by the sum of the weights (Luminance-Weighted
    Pooling subsection); mu1 is the reference's windowed mean."""
    r = ssim_map(x, y, p)
    wq = lw_weights(r["mu_x"], a_s, b_s) * r["map"]
    return math.fsum(wq.ravel().tolist()) / wq.size


def pool_cov(q: np.ndarray) -> float:
    """Coefficient of variation sigma_Q / mu_Q (the CoV equation of the
    Spatial and Temporal Aggregation section, after the MOVIE index)."""
    v = np.asarray(q, dtype=np.float64).ravel()
    mu = math.fsum(v) / v.size
    var = math.fsum((v - mu) ** 2) / v.size
    return math.sqrt(var) / mu


def pool_md(q: np.ndarray, p: float, o: float) -> float:
    """Mean-deviation pooling: (((1/n) sum |Q - mu|^p)^(1/p))^o."""
    v = np.asarray(q, dtype=np.float64).ravel()
    mu = math.fsum(v) / v.size
    d = math.fsum(np.abs(v - mu) ** p) / v.size
    return (d ** (1.0 / p)) ** o


def pool_minkowski(q: np.ndarray, p: float) -> float:
    """Minkowski pooling of the dissimilarity: (1/n) sum (1 - Q)^p."""
    v = np.asarray(q, dtype=np.float64).ravel()
    return math.fsum((1.0 - v) ** p) / v.size


def pool_distortion_weighted(q: np.ndarray, p: float) -> float:
    """Distortion-weighted pooling: sum (1-Q)^p Q / sum (1-Q)^p."""
    v = np.asarray(q, dtype=np.float64).ravel()
    w = (1.0 - v) ** p
    den = math.fsum(w)
    if den == 0.0:
        return 1.0
    return math.fsum(w * v) / den


def _percentile_linear(sorted_v: np.ndarray, frac: float) -> float:
    h = (sorted_v.size - 1) * frac
    lo = int(math.floor(h))
    hi = min(lo + 1, sorted_v.size - 1)
    return float(sorted_v[lo] + (h - lo) * (sorted_v[hi] - sorted_v[lo]))


# Moment-based and windowed pooling (Moment-Based Pooling subsection and the
# windowed means after the CoV equation).  The paper applies them to the
# series of frame scores (temporal pooling); every pooling above applies to
# such a series too (a 1 x T map).  Readings: the geometric mean of values
# with a zero is 0 and with a negative value NaN; the harmonic mean of values
# with a zero is 0; windows of w consecutive values lie inside the series (T -
# w + 1 of them) and their local values are averaged with equal weights.
def pool_geometric(q: np.ndarray) -> float:
    """Geometric mean exp((1/n) sum log Q)."""
    v = np.asarray(q, dtype=np.float64).ravel()
    if np.any(v < 0) or np.any(np.isnan(v)):
        return float("nan")
    if np.any(v == 0):
        return 0.0
    return math.exp(math.fsum(np.log(v)) / v.size)


def pool_harmonic(q: np.ndarray) -> float:
    """Harmonic mean n / sum (1/Q)."""
    v = np.asarray(q, dtype=np.float64).ravel()
    if np.any(v == 0):
        return 0.0
    return v.size / math.fsum(1.0 / v)


def pool_median(q: np.ndarray) -> float:
    """Sample median (mean of the two middle values for even n)."""
    s = np.sort(np.asarray(q, dtype=np.float64).ravel())
    return _percentile_linear(s, 0.5)


_WINDOW_MEANS = {"am": pool_mean, "gm": pool_geometric, "hm": pool_harmonic, "cov": pool_cov}


def pool_windowed(q: np.ndarray, w: int, mean: str) -> float:
    """Windowed pooling W-AM / W-GM / W-HM / W-CoV: the mean over every window
    of w consecutive values of the window's AM, GM, HM or CoV."""
    v = np.asarray(q, dtype=np.float64).ravel()
    if not 1 <= w <= v.size:
        raise ValueError("window length must be in 1..n")
    f = _WINDOW_MEANS[mean]
    return math.fsum(f(v[t:t + w]) for t in range(v.size - w + 1)) / (v.size - w + 1)


def pool_five_number(q: np.ndarray) -> float:
    """Five-number summary: (min + Q1 + median + Q3 + max) / 5."""
    s = np.sort(np.asarray(q, dtype=np.float64).ravel())
    parts = [s[0], _percentile_linear(s, 0.25), _percentile_linear(s, 0.5), _percentile_linear(s, 0.75), s[-1]]
    return math.fsum(parts) / 5.0


def pool_percentile(q: np.ndarray, p_s: float, r_s: float) -> float:
    """Percentile pooling: the lowest p_s percent of the map divided by r_s,
    then the mean."""
    s = np.sort(np.asarray(q, dtype=np.float64).ravel())
    m = int(math.ceil(p_s * s.size / 100.0))
    return (math.fsum(s[:m] / r_s) + math.fsum(s[m:])) / s.size


# --------------------------------------------------------------------------
# Pre-scaling and the "Enhanced SSIM" composition.
#   * the down-sampling transform of the Transforming-across-Scales
#     subsection: Z = max(1, ceil(H / 256)), an f x f block average with
#     decimation by f (odd remainders dropped, as for the 2x2 pyramid);
#   * Enhanced SSIM (closing recommendation of the aggregation section):
#     luma, rectangular 11x11 windows, stride 5, pre-scaling, CoV pooling.
#     The rule that infers the factor from D/H is not printed; the factor is
#     an argument and defaults to Z.
# --------------------------------------------------------------------------
def scale_factor(h: int) -> int:
    """Z = max(1, ceil(H / 256)) of the Transforming-across-Scales subsection."""
    return max(1, -(-int(h) // 256))


def downsample_avg(a: np.ndarray, f: int) -> np.ndarray:
    """f x f block means over the aligned blocks that fit (decimation by f)."""
    a = _as_f64(a)
    if f == 1:
        return a.copy()
    h, w = a.shape[0] // f, a.shape[1] // f
    return a[:h * f, :w * f].reshape(h, f, w, f).mean(axis=(1, 3))


_POOLERS = {
    "mean": lambda q, p, o, r: pool_mean(q),
    "cov": lambda q, p, o, r: pool_cov(q),
    "mean_dev": lambda q, p, o, r: pool_md(q, p, o),
    "minkowski": lambda q, p, o, r: pool_minkowski(q, p),
    "dist_weighted": lambda q, p, o, r: pool_distortion_weighted(q, p),
    "five_number": lambda q, p, o, r: pool_five_number(q),
    "percentile": lambda q, p, o, r: pool_percentile(q, p, r),
}


def scaled_pooled_ssim(x, y, p: SSIMParams | None = None, factor: int = 1, pool: str = "mean",
                       pp: float = 0.0, po: float = 1.0, pr: float = 1.0) -> float:
    """Down-sample by `factor`, take the SSIM map with parameters p, pool it."""
    xs, ys = downsample_avg(x, factor), downsample_avg(y, factor)
    q = ssim_map(xs, ys, p)["map"]
    return _POOLERS[pool](q, pp, po, pr)


def enhanced_ssim(x, y, factor: int | None = None, L: float = 255.0) -> float:
    """Enhanced SSIM: 11x11 rectangular window at stride 5 on the pre-scaled
    luma, pooled by the coefficient of variation."""
    C1, C2 = constants(0.01, 0.03, L)
    p = SSIMParams(window="box", k=11, C1=C1, C2=C2, stride=5)
    f = scale_factor(np.asarray(x).shape[0]) if factor is None else factor
    return scaled_pooled_ssim(x, y, p, f, "cov")


# --------------------------------------------------------------------------
# Channel-wise colour SSIM (Channel-wise SSIM subsection): YCbCr by the BT.709
# transform printed there, the pooled SSIM of each channel, and the weighted
# average (f(Y) + alpha f(Cb) + beta f(Cr)) / (1 + alpha + beta).  Reading:
# the same window and C1, C2 serve all three channels.
# --------------------------------------------------------------------------
BT709_Y = (0.213, 0.715, 0.072)
BT709_CB, BT709_CR = 0.539, 0.635


def rgb_to_ycbcr_bt709(rgb: np.ndarray) -> np.ndarray:
    """(3, H, W) RGB -> (3, H, W) Y, Cb = 0.539 (B - Y), Cr = 0.635 (R - Y)."""
    rgb = np.asarray(rgb, dtype=np.float64)
    y = BT709_Y[0] * rgb[0] + BT709_Y[1] * rgb[1] + BT709_Y[2] * rgb[2]
    return np.stack([y, BT709_CB * (rgb[2] - y), BT709_CR * (rgb[0] - y)])


def color_ssim(x_rgb, y_rgb, p: SSIMParams | None = None, alpha: float = 0.125, beta: float = 0.125) -> dict:
    """Per-channel pooled SSIM and their weighted average; alpha = beta =
    0.125 gives the 0.8 / 0.1 / 0.1 weighting of the FFMPEG / Daala form."""
    xs, ys = rgb_to_ycbcr_bt709(x_rgb), rgb_to_ycbcr_bt709(y_rgb)
    s = [ssim_pooled(xs[c], ys[c], p) for c in range(3)]
    return {"channels": s, "score": (s[0] + alpha * s[1] + beta * s[2]) / (1.0 + alpha + beta)}


# --------------------------------------------------------------------------
# SSIM-3D and MS-SSIM-3D (Spatio-Temporal SSIM subsection).  SSIM whose mean,
# variance and covariance are taken over k x k x kt spatio-temporal boxes with
# equal weights; MS-SSIM-3D applies it at every scale of a spatial pyramid
# (each frame down-sampled on its own, the temporal extent unchanged).
#
# Readings: the box (t, i, j) covers frames t .. t+kt-1, rows i .. i+k-1 and
# columns j .. j+k-1 (top-left anchoring as for 2-D windows; the paper's
# trailing-window sums differ only in the index of the output); boxes lie
# inside the clip in all three axes, so a clip of T frames gives T-kt+1 map
# frames; each map frame is pooled by its mean, and MS-SSIM-3D combines the
# per-scale means of the same map frame as MS-SSIM does.
# --------------------------------------------------------------------------
def box_sums3d(x, y, k: int, kt: int):
    """Window sums S1x, S1y, S2x, S2y, S12 over every k x k x kt box, by
    adding every (frame, row, column) offset of the box: exact int64 for
    integer clips, float64 otherwise.  x, y: [T, H, W]."""
    integer = np.issubdtype(np.asarray(x).dtype, np.integer) and np.issubdtype(np.asarray(y).dtype, np.integer)
    dt = np.int64 if integer else np.float64
    x = np.asarray(x).astype(dt)
    y = np.asarray(y).astype(dt)
    T, H, W = x.shape
    to, ho, wo = T - kt + 1, H - k + 1, W - k + 1
    if to < 1 or ho < 1 or wo < 1:
        raise ValueError("clip smaller than the box")
    acc = [np.zeros((to, ho, wo), dtype=dt) for _ in range(5)]
    for o in range(kt):
        for m in range(k):
            for n in range(k):
                xs = x[o:o + to, m:m + ho, n:n + wo]
                ys = y[o:o + to, m:m + ho, n:n + wo]
                acc[0] += xs
                acc[1] += ys
                acc[2] += xs * xs
                acc[3] += ys * ys
                acc[4] += xs * ys
    return tuple(acc)


def ssim3d_map(x, y, p: SSIMParams | None = None, kt: int = 1) -> dict:
    """SSIM-3D map [T-kt+1, H-k+1, W-k+1] of two clips [T, H, W] with the
    rectangular k x k x kt box (p.window must be 'box', stride 1, valid).
    Statistics from the window sums as in eqs. mean_from_sum .. corr_from_sum
    with N = k*k*kt samples; the numerators N S2 - S1^2 are exact integers for
    integer clips."""
    p = p or SSIMParams(window="box", k=11)
    p.check()
    if p.window != "box" or p.stride != 1 or p.padding != "valid":
        raise ValueError("SSIM-3D uses a rectangular box, stride 1, valid borders")
    if kt < 1:
        raise ValueError("kt must be positive")
    s1x, s1y, s2x, s2y, s12 = box_sums3d(x, y, p.k, kt)
    n = p.k * p.k * kt
    n2 = float(n) * float(n)
    mu_x = s1x.astype(np.float64) / n
    mu_y = s1y.astype(np.float64) / n
    sxx = (n * s2x - s1x * s1x).astype(np.float64) / n2
    syy = (n * s2y - s1y * s1y).astype(np.float64) / n2
    sxy = (n * s12 - s1x * s1y).astype(np.float64) / n2
    with np.errstate(divide="ignore", invalid="ignore"):
        l = (2.0 * mu_x * mu_y + p.C1) / (mu_x * mu_x + mu_y * mu_y + p.C1)
        cs = (2.0 * sxy + p.C2) / (sxx + syy + p.C2)
    return {"map": l * cs, "l": l, "cs": cs, "mu_x": mu_x, "mu_y": mu_y, "sxx": sxx, "syy": syy, "sxy": sxy}


def ssim3d(x, y, p: SSIMParams | None = None, kt: int = 1) -> np.ndarray:
    """Mean of every SSIM-3D map frame, float64 [T-kt+1]."""
    m = ssim3d_map(x, y, p, kt)["map"]
    return np.array([mean_pool(m[t]) for t in range(m.shape[0])])


def msssim3d(x, y, p: SSIMParams | None = None, kt: int = 1, weights=MS_WEIGHTS, n_scales: int = 5,
             renorm: bool = False, cs_clamp: bool = False, aggregation: str = "product",
             coarse_separate: bool = False) -> dict:
    """MS-SSIM-3D per map frame: every frame of both clips is reduced by the
    2x2 pyramid of MS-SSIM; at each scale the SSIM-3D maps give CS_j(t) (mean
    cs, j < M) and S_M(t) (mean l*cs at the coarsest scale), combined per map
    frame t as in msssim.  Returns {'score' [T-kt+1], 'cs' [T-kt+1, M-1],
    's_M' [T-kt+1]}."""
    p = p or SSIMParams(window="box", k=11)
    if aggregation not in ("product", "sum"):
        raise ValueError(f"unknown aggregation {aggregation!r}")
    w = _ms_weights(weights, n_scales, renorm or aggregation == "sum")
    xf = _as_f64(x)
    yf = _as_f64(y)
    xs = [np.stack(v) for v in zip(*[pyramid(f, n_scales) for f in xf])]
    ys = [np.stack(v) for v in zip(*[pyramid(f, n_scales) for f in yf])]
    to = xf.shape[0] - kt + 1
    cs = np.zeros((to, n_scales - 1))
    s_m = np.zeros(to)
    for j in range(n_scales):
        r = ssim3d_map(xs[j], ys[j], p, kt)
        for t in range(to):
            if j < n_scales - 1:
                cs[t, j] = mean_pool(r["cs"][t])
            elif coarse_separate:
                s_m[t] = mean_pool(r["l"][t]) * mean_pool(r["cs"][t])
            else:
                s_m[t] = mean_pool(r["map"][t])
    score = np.array([_ms_combine(list(cs[t]), s_m[t], w, cs_clamp, aggregation) for t in range(to)])
    return {"score": score, "cs": cs, "s_M": s_m, "weights": w}
