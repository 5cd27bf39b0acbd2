// asinh gray-scale stretch y = b * asinh(v / a) and its backward
// (Sec. 2.2.6: per-pixel gray-scale maps ahead of neural networks).
// Element-wise and HBM-bound: 8 B/px forward (read v, write y), 12 B/px
// backward (read v and dL/dy, write dL/dv).  The parameter gradients are
// binary64 block partials reduced in a fixed order by one workgroup.
#include "ipp_internal.h"
#include "kernels.h"

namespace ipp {

__global__ __launch_bounds__(kBlock) void k_asinh_fwd(const float* v,
                                                      float* y, int64_t n,
                                                      float inv_a, float b) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    y[i] = b * asinhf(v[i] * inv_a);
}

__global__ __launch_bounds__(kBlock) void k_asinh_bwd(const float* v,
                                                      const float* dy,
                                                      float* dv, int64_t n,
                                                      double a, double b,
                                                      double* partial) {
  __shared__ double red[kWaves];
  const float af = (float)a, bf = (float)b;
  double pa = 0.0, pb = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const float x = v[i], g = dy[i];
    if (dv) dv[i] = g * (bf / sqrtf(af * af + x * x));
    if (partial) {
      const double xd = (double)x, gd = (double)g;
      const double r = sqrt(a * a + xd * xd);
      pa += gd * (-b * xd / (a * r));
      pb += gd * asinh(xd / a);
    }
  }
  if (!partial) return;
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
