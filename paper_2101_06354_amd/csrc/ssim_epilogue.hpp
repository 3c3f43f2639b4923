// Per-position SSIM terms from local statistics, in the sum/difference basis
// u = x + y, v = x - y used by the float kernels.
//
// With mu_x = (mu_u + mu_v)/2 and mu_y = (mu_u - mu_v)/2 the Background-section
// terms become
//   2 mu_x mu_y          = (mu_u^2 - mu_v^2) / 2
//   mu_x^2 + mu_y^2      = (mu_u^2 + mu_v^2) / 2
//   2 sigma_xy           = (var_u - var_v) / 2
//   sigma_x^2+sigma_y^2  = (var_u + var_v) / 2
// so the numerator and denominator of l (and of cs) differ by exactly
// mu_v^2 (and var_v).  Writing D1 = B1 - A1 and D2 = B2 - A2,
//   Q = A1 A2 / (B1 B2) = 1 - (D1 A2 + D2 B1) / (B1 B2),   cs = 1 - D2 / B2,
// so the division only scales a correction term: a reciprocal estimate
// (about 1 ulp) then costs at most a few ulp of 1 - Q, and when x == y the
// correction is exactly 0 (D1 = D2 = 0), so Q == 1.0f exactly.  Swapping x and
// y only flips the sign of v, which D1, D2, A and B do not see, so Q is
// bitwise symmetric.
#pragma once

#include <hip/hip_runtime.h>

namespace ssimx {

struct SsimTerms {
  float A1, B1, A2, B2;
  float D1, D2;  // B1 - A1 and B2 - A2, formed without cancellation
};

__device__ __forceinline__ SsimTerms ssim_terms_uv(float mean_u, float mean_v, float var_u, float var_v, float C1,
                                                   float C2) {
  SsimTerms t;
  const float P = (0.5f * mean_u) * mean_u;
  const float R = (0.5f * mean_v) * mean_v;
  t.A1 = (P - R) + C1;
  t.B1 = (P + R) + C1;
  t.A2 = 0.5f * (var_u - var_v) + C2;
  t.B2 = 0.5f * (var_u + var_v) + C2;
  t.D1 = 2.f * R;
  t.D2 = var_v;
  return t;
}

// mode 0: Q = l*cs ; mode 1: cs ; mode 3: l
__device__ __forceinline__ float ssim_value(const SsimTerms& t, int mode) {
  if (mode == 1) return fmaf(-t.D2, __builtin_amdgcn_rcpf(t.B2), 1.f);
  if (mode == 3) return fmaf(-t.D1, __builtin_amdgcn_rcpf(t.B1), 1.f);
  const float n = fmaf(t.D1, t.A2, t.D2 * t.B1);
  return fmaf(-n, __builtin_amdgcn_rcpf(t.B1 * t.B2), 1.f);
}

// The same Q (mode 0), cs (mode 1) or l (mode 3) straight from the u, v
// statistics, with the numerator and denominator of l and of cs both doubled
// (a ratio does not change): with a = mu_u^2, b = mu_v^2,
//   B1 = a + b + 2 C1,  A1 = B1 - 2 b,  B2 = var_u + 2 C2 + var_v,  A2 = B2 - 2 var_v,
//   1 - Q = 2 (b A2 + var_v B1) / (B1 B2),
// which needs neither A1 nor the halvings.  x == y still gives b = var_v = 0
// and Q == 1.0f exactly, and swapping x and y leaves b and var_v unchanged.
// c1x2 = 2 C1, c2x2 = 2 C2.
// The same from s = var_u + 2 C2 (a caller may accumulate the variance of u
// on top of 2 C2 and so skip the addition).
template <int MODE>
__device__ __forceinline__ float ssim_value_uv_s(float mean_u, float mean_v, float s, float var_v, float c1x2) {
  const float b = mean_v * mean_v;
  if constexpr (MODE == 1) return fmaf(-2.f * var_v, __builtin_amdgcn_rcpf(s + var_v), 1.f);
  const float B1 = fmaf(mean_u, mean_u, b) + c1x2;
  if constexpr (MODE == 3) return fmaf(-2.f * b, __builtin_amdgcn_rcpf(B1), 1.f);
  const float B2 = s + var_v, A2 = s - var_v;
  const float n = fmaf(b, A2, var_v * B1);
  return fmaf(n, -2.f * __builtin_amdgcn_rcpf(B1 * B2), 1.f);
}

template <int MODE>
__device__ __forceinline__ float ssim_value_uv_m(float mean_u, float mean_v, float var_u, float var_v, float c1x2,
                                                 float c2x2) {
  return ssim_value_uv_s<MODE>(mean_u, mean_v, var_u + c2x2, var_v, c1x2);
}

__device__ __forceinline__ float ssim_value_uv(float mean_u, float mean_v, float var_u, float var_v, float c1x2,
                                               float c2x2, int mode) {
  if (mode == 1) return ssim_value_uv_m<1>(mean_u, mean_v, var_u, var_v, c1x2, c2x2);
  if (mode == 3) return ssim_value_uv_m<3>(mean_u, mean_v, var_u, var_v, c1x2, c2x2);
  return ssim_value_uv_m<0>(mean_u, mean_v, var_u, var_v, c1x2, c2x2);
}

// Same terms from exact integer window sums of a k x k rectangular window
// (the statistics of the integral-image method): every numerator below is an
// exact integer and is rounded to float once.
__device__ __forceinline__ SsimTerms ssim_terms_box(int64_t sx, int64_t sy, int64_t sxx, int64_t syy, int64_t sxy,
                                                    int64_t kk, float k4, float C1, float C2) {
  const int64_t nxx = kk * sxx - sx * sx;
  const int64_t nyy = kk * syy - sy * sy;
  const int64_t nxy = kk * sxy - sx * sy;
  SsimTerms t;
  t.A1 = (float)(2 * sx * sy) / k4 + C1;
  t.B1 = (float)(sx * sx + sy * sy) / k4 + C1;
  t.A2 = (float)(2 * nxy) / k4 + C2;
  t.B2 = (float)(nxx + nyy) / k4 + C2;
  const int64_t dxy = sx - sy;
  t.D1 = (float)(dxy * dxy) / k4;                // (mu_x - mu_y)^2
  t.D2 = (float)(nxx + nyy - 2 * nxy) / k4;      // variance of x - y
  return t;
}

}  // namespace ssimx
