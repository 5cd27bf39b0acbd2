// Stamp convolution and image subtraction (Sec. 2.2.4, Eq. 8-10): the
// template R is convolved with a spatially varying kernel
//   K(u, v) = sum_n a_n(x, y) exp(-(u^2 + v^2) / (2 sigma_k^2)) u^i v^j
// and the difference D = (I + B) - R (x) K is written.  As in the paper's
// GPU design, the image is cut into stamps (21 x 21 by default) and one
// workgroup handles one stamp: the stamp's kernel (a_n and B evaluated at
// the stamp centre) is built in binary64 and kept in LDS as binary32, the
// template tile with its (2 hw)-pixel margin is staged in LDS (zero outside
// the frame), and each output pixel sums its (2hw+1)^2 products in binary32
// per kernel row, the rows in binary64: the error stays below
// (2hw + 2) 2^-24 of sum |K| |R|.  One HBM read of I and R and one write
// of D per pixel (12 B/px); the tile re-reads its margin from L2.
#include "ipp_internal.h"
#include "kernels.h"

namespace ipp {

namespace {
__device__ __forceinline__ double norm_c(double x, int n) {
  return n > 1 ? (2.0 * x - (double)(n - 1)) / (double)(n - 1) : 0.0;
}

// sum c_pq xn^p yn^q over p = 0..d, q = 0..d-p, in that order
__device__ double poly2(const double* c, int d, double xn, double yn) {
  double tot = 0.0;
  int k = 0;
  double xp = 1.0;
  for (int p = 0; p <= d; ++p) {
    double yq = 1.0;
    for (int q = 0; q <= d - p; ++q) {
      tot += c[k++] * xp * yq;
      yq *= yn;
    }
    xp *= xn;
  }
  return tot;
}
}  // namespace

__global__ __launch_bounds__(kBlock) void k_subtract(
    const SubFrame* frames, int nframes, SubBasis bs, int64_t total_stamps) {
  __shared__ double a_s[kSubMaxBasis];
  __shared__ double b_s;
  __shared__ float ker[(2 * kSubMaxHw + 1) * (2 * kSubMaxHw + 1)];
  __shared__ float tile[(kSubMaxStamp + 2 * kSubMaxHw) *
                        (kSubMaxStamp + 2 * kSubMaxHw)];
  const int hw = bs.hw, kw = 2 * hw + 1, S = bs.stamp;
  const int tw = S + 2 * hw;
  for (int64_t st = blockIdx.x; st < total_stamps; st += gridDim.x) {
    // frame of this stamp (frames are few: a linear search)
    int f = 0;
    while (f + 1 < nframes && frames[f + 1].stamp0 <= st) ++f;
    const SubFrame fr = frames[f];
    const int64_t ls = st - fr.stamp0;
    const int sy = (int)(ls / fr.nsx), sx = (int)(ls % fr.nsx);
    const int x0 = sx * S, y0 = sy * S;
    const int x1 = min(x0 + S, fr.w), y1 = min(y0 + S, fr.h);
    const double xc = (double)(x0 + x1 - 1) / 2.0;
    const double yc = (double)(y0 + y1 - 1) / 2.0;
    const double xn = norm_c(xc, fr.w), yn = norm_c(yc, fr.h);
    const int ns = (bs.spatial_order + 1) * (bs.spatial_order + 2) / 2;
    __syncthreads();                 // the previous stamp is done with LDS
    for (int n = threadIdx.x; n < bs.nbasis; n += kBlock)
      a_s[n] = poly2(fr.coef + (int64_t)n * ns, bs.spatial_order, xn, yn);
    if (threadIdx.x == 0)
      b_s = poly2(fr.coef + (int64_t)bs.nbasis * ns, bs.bkg_order, xn, yn);
    // template tile with its margin, zero outside the frame
    for (int e = threadIdx.x; e < tw * tw; e += kBlock) {
      const int ty = e / tw, tx = e - ty * tw;
      const int gy = y0 - hw + ty, gx = x0 - hw + tx;
      float r = 0.0f;
      if (gy >= 0 && gy < fr.h && gx >= 0 && gx < fr.w)
        r = fr.R[(int64_t)gy * fr.pitchR + gx];
      tile[e] = r;
    }
    __syncthreads();
    // the stamp's kernel in binary64, kept as binary32
    for (int t = threadIdx.x; t < kw * kw; t += kBlock) {
      const int v = t / kw - hw, u = t % kw - hw;
      const double du = (double)u, dv = (double)v;
      double k = 0.0;
      int n = 0;
      for (int g = 0; g < bs.ngauss; ++g) {
        const double s = bs.sigma[g];
        const double e = exp(-(du * du + dv * dv) / (2.0 * s * s));
        double ui = 1.0;
        for (int i = 0; i <= bs.order[g]; ++i) {
          double vj = 1.0;
          for (int j = 0; j <= bs.order[g] - i; ++j) {
            k += a_s[n++] * (e * ui * vj);
            vj *= dv;
          }
          ui *= du;
        }
      }
      ker[t] = (float)k;
    }
    __syncthreads();
    const double B = b_s;
    const int ow = x1 - x0, oh = y1 - y0;
    for (int o = threadIdx.x; o < ow * oh; o += kBlock) {
      const int ly = o / ow, lx = o - ly * ow;
      // R(x - u, y - v) = tile[ly + hw - v][lx + hw - u]
      double acc = 0.0;
      for (int vv = 0; vv < kw; ++vv) {          // vv = v + hw
        const float* trow = tile + (ly + 2 * hw - vv) * tw + lx + 2 * hw;
        const float* krow = ker + vv * kw;
        float rs = 0.0f;
        for (int uu = 0; uu < kw; ++uu)          // uu = u + hw
          rs = fmaf(krow[uu], trow[-uu], rs);
        acc += (double)rs;
      }
      const int64_t gy = y0 + ly, gx = x0 + lx;
      const double I = (double)fr.I[gy * fr.pitchI + gx];
      fr.D[gy * fr.w + gx] = (float)((I + B) - acc);
    }
  }
}

}  // namespace ipp
