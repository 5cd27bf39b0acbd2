// asinh gray-scale stretch y = b * asinh(v / a) and its backward
// (Sec. 2.2.6: per-pixel gray-scale maps ahead of neural networks).
// Element-wise and HBM-bound: 8 B/px forward (read v, write y), 12 B/px
// backward (read v and dL/dy, write dL/dv).  The parameter gradients are
// binary64 block partials reduced in a fixed order by one workgroup.
#include <mutex>

#include "ipp_internal.h"
#include "kernels.h"

namespace ipp {

// Scratch of the allocation-free backward: the binary64 block partials of
// the two parameter gradients.  One copy per GPU, held until the process
// ends.  In host code `scratch` names a host-side stand-in, never the
// device memory: kernels are given the address from asinh_scratch().
static __device__ __align__(256) double scratch[2 * kAsinhMaxBlocks];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t asinh_scratch(int device, double** ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) hipSetDevice(cur);
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = (double*)p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

// Elements i (float4 groups when every pointer is 16-byte aligned), two
// groups per thread and step, so that several loads are in flight.
template <typename Fn>
__device__ __forceinline__ void for_elements(int64_t n, bool vec, Fn fn) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t i0 = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  int64_t done = 0;
  if (vec) {
    const int64_t n4 = n >> 2;
    for (int64_t i = i0; i < n4; i += 2 * stride) {
      fn(i, true);
      if (i + stride < n4) fn(i + stride, true);
    }
    done = n4 << 2;
  }
  for (int64_t i = done + i0; i < n; i += stride) fn(i, false);
}

// b * asinh(t) in binary32: for |t| < 1/4 the Maclaurin series of asinh
// through t^11 (the first term left out is below 3e-10 relative),
// otherwise ln 2 * log2(|t| + sqrt(t^2 + 1)) with the hardware base-2
// logarithm (its argument is then above 1.28, so the result keeps a
// relative error of a few 1e-7), and log2|t| + 1 where t^2 would overflow.
__device__ __forceinline__ float stretch(float x, float inv_a, float b) {
  const float t = x * inv_a;
  const float at = fabsf(t);
  const float t2 = at * at;
  float p = -63.0f / 2816.0f;
  p = fmaf(p, t2, 35.0f / 1152.0f);
  p = fmaf(p, t2, -5.0f / 112.0f);
  p = fmaf(p, t2, 3.0f / 40.0f);
  p = fmaf(p, t2, -1.0f / 6.0f);
  const float ser = fmaf(at * t2, p, at);
  const float u = at + sqrtf(fmaf(at, at, 1.0f));
  const float lg = at > 1e18f ? __builtin_amdgcn_logf(at) + 1.0f
                              : __builtin_amdgcn_logf(u);
  const float big = 0.693147180559945f * lg;
  return b * copysignf(at < 0.25f ? ser : big, t);
}

// Parameters read on the device: (a, b) = ab[0..1].  A non-positive or
// non-finite a, or a non-finite b, makes every output NaN (the host cannot
// check values it never sees).
__device__ __forceinline__ bool device_params(const double* ab, double* a,
                                              double* b) {
  *a = ab[0];
  *b = ab[1];
  return *a > 0.0 && isfinite(*a) && isfinite(*b);
}

__global__ __launch_bounds__(kBlock) void k_asinh_fwd(const float* v,
                                                      float* y, int64_t n,
                                                      float inv_a, float b,
                                                      const double* ab) {
  if (ab) {
    double ad, bd;
    const bool ok = device_params(ab, &ad, &bd);
    inv_a = ok ? (float)(1.0 / ad) : __builtin_nanf("");
    b = ok ? (float)bd : __builtin_nanf("");
  }
  const bool vec = (((uintptr_t)v | (uintptr_t)y) & 15) == 0;
  for_elements(n, vec, [&](int64_t i, bool four) {
    if (four) {
      float4 x = ((const float4*)v)[i];
      x.x = stretch(x.x, inv_a, b);
      x.y = stretch(x.y, inv_a, b);
      x.z = stretch(x.z, inv_a, b);
      x.w = stretch(x.w, inv_a, b);
      ((float4*)y)[i] = x;
    } else {
      y[i] = stretch(v[i], inv_a, b);
    }
  });
}

// ln(1 + y) for y >= 0 in binary64: 1 + y = m 2^e with m in [sqrt(1/2),
// sqrt(2)), ln(1 + y) = e ln 2 + 2 atanh(f / (2 + f)) with f = m - 1 (f = y
// itself when e = 0, so small y keep every digit), and the series
// atanh(s) = s + s^3/3 + ... + s^21/21 for |s| <= 0.1716 (the first term left
// out is below 2e-18 relative).  ln 2 is split in two parts (Cody and
// Waite's argument-reduction split: a 30-bit leading part, so that e times
// it is exact, and the remainder).
__device__ __forceinline__ double log1p_pos(double y) {
  const double u = 1.0 + y;
  int e;
  double m = frexp(u, &e);                 // m in [1/2, 1)
  if (m < 0.70710678118654752) {
    m *= 2.0;
    e -= 1;
  }
  const double f = e == 0 ? y : m - 1.0;
  const double s = f / (2.0 + f);
  const double s2 = s * s;
  double q = 1.0 / 21.0;
  q = fma(q, s2, 1.0 / 19.0);
  q = fma(q, s2, 1.0 / 17.0);
  q = fma(q, s2, 1.0 / 15.0);
  q = fma(q, s2, 1.0 / 13.0);
  q = fma(q, s2, 1.0 / 11.0);
  q = fma(q, s2, 1.0 / 9.0);
  q = fma(q, s2, 1.0 / 7.0);
  q = fma(q, s2, 1.0 / 5.0);
  q = fma(q, s2, 1.0 / 3.0);
  const double at2 = 2.0 * fma(s * s2, q, s);     // 2 atanh(s)
  const double ed = (double)e;
  const double ln2_hi = 6.93147180369123816490e-01;   // 30 leading bits
  const double ln2_lo = 1.90821492927058770002e-10;   // ln 2 - ln2_hi
  return fma(ed, ln2_hi, fma(ed, ln2_lo, at2));
}

// One element of the backward.  With r = sqrt(a^2 + v^2) and
// w = 1 / (r (a + r)) (one division):
//   dy/dv = b / r = b (a + r) w,
//   dy/da = -b v / (a r) = -(b / a) v (a + r) w,
//   asinh(v / a) = sign(v) log1p(t + t^2 a / (a + r)), t = |v| / a, and
//   a / (a + r) = a r w (the log1p form of asinh, with sqrt(1 + t^2) = r/a).
__device__ __forceinline__ void asinh_bwd_one(float x, float g, double a,
                                              double inv_a, double b,
                                              double mb_inv_a, bool want_ab,
                                              float* dv, double& pa,
                                              double& pb) {
  if (!want_ab) {
    const float af = (float)a, bf = (float)b;
    *dv = g * (bf / sqrtf(af * af + x * x));
    return;
  }
  const double xd = (double)x, gd = (double)g;
  const double r = sqrt(fma(xd, xd, a * a));
  const double ar = a + r;
  const double w = 1.0 / (r * ar);
  *dv = g * (float)(b * ar * w);
  pa = fma(gd, mb_inv_a * xd * ar * w, pa);
  const double t = fabs(xd) * inv_a;
  const double as = log1p_pos(fma(t * t, a * r * w, t));
  pb = fma(gd, copysign(as, xd), pb);
}

__global__ __launch_bounds__(kBlock) void k_asinh_bwd(const float* v,
                                                      const float* dy,
                                                      float* dv, int64_t n,
                                                      double a, double b,
                                                      const double* ab,
                                                      double* partial) {
  __shared__ double red[kWaves];
  if (ab && !device_params(ab, &a, &b)) a = b = __builtin_nan("");
  const double inv_a = 1.0 / a, mb_inv_a = -b / a;
  const bool want_ab = partial != nullptr;
  double pa = 0.0, pb = 0.0;
  const bool vec =
      (((uintptr_t)v | (uintptr_t)dy | (uintptr_t)dv) & 15) == 0;
  for_elements(n, vec, [&](int64_t i, bool four) {
    if (four) {
      const float4 x = ((const float4*)v)[i];
      const float4 g = ((const float4*)dy)[i];
      float4 o;
      asinh_bwd_one(x.x, g.x, a, inv_a, b, mb_inv_a, want_ab, &o.x, pa, pb);
      asinh_bwd_one(x.y, g.y, a, inv_a, b, mb_inv_a, want_ab, &o.y, pa, pb);
      asinh_bwd_one(x.z, g.z, a, inv_a, b, mb_inv_a, want_ab, &o.z, pa, pb);
      asinh_bwd_one(x.w, g.w, a, inv_a, b, mb_inv_a, want_ab, &o.w, pa, pb);
      if (dv) ((float4*)dv)[i] = o;
    } else {
      float o;
      asinh_bwd_one(v[i], dy[i], a, inv_a, b, mb_inv_a, want_ab, &o, pa, pb);
      if (dv) dv[i] = o;
    }
  });
  if (!want_ab) return;
  pa = block_sum(pa, red);
  pb = block_sum(pb, red);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = pa;
    partial[2 * blockIdx.x + 1] = pb;
  }
}

__global__ __launch_bounds__(kBlock) void k_asinh_bwd_final(
    const double* partial, int nb, double* out) {
  __shared__ double red[kWaves];
  double pa = 0.0, pb = 0.0;
  for (int i = threadIdx.x; i < nb; i += kBlock) {
    pa += partial[2 * i];
    pb += partial[2 * i + 1];
  }
  pa = block_sum(pa, red);
  pb = block_sum(pb, red);
  if (threadIdx.x == 0) {
    out[0] = pa;
    out[1] = pb;
  }
}

}  // namespace ipp
