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

// LDS layout of one stamp (dynamic shared memory, sized by the host with
// sub_lds_bytes): the stamp's a_n and B (and one pad, so that what follows
// is 16-byte aligned), the kernel (rows padded to a multiple of 4 floats)
// and the template tile with its margin (rows padded so that every
// thread's row segment is whole float4s).
constexpr int kSubHead = kSubMaxBasis + 2;
static_assert((kSubHead * sizeof(double)) % 16 == 0, "float4 alignment");
constexpr int kSubOut = 4;           // adjacent outputs per thread
__host__ __device__ int sub_groups(int stamp) {
  return (stamp + kSubOut - 1) / kSubOut;
}
__host__ __device__ int sub_kstride(int hw) { return (2 * hw + 1 + 3) & ~3; }
__host__ __device__ int sub_nr(int hw) {
  return (2 * hw + kSubOut + 3) / 4;
}
__host__ __device__ int sub_tstride(int stamp, int hw) {
  return kSubOut * (sub_groups(stamp) - 1) + 4 * sub_nr(hw);
}
size_t sub_lds_bytes(int stamp, int hw) {
  const int kw = 2 * hw + 1, th = stamp + 2 * hw;
  return sizeof(double) * kSubHead +
         sizeof(float) * ((size_t)kw * sub_kstride(hw) +
                          (size_t)th * sub_tstride(stamp, hw));
}
int sub_threads(int stamp) {
  const int t = stamp * sub_groups(stamp);
  return ((t + kWave - 1) / kWave) * kWave;
}

// One workgroup per stamp (two wavefronts for the default 21-pixel
// stamps); each thread computes kSubOut adjacent outputs of one row, with
// its template row segment (2 HW + kSubOut values) and the kernel row in
// registers: per kernel row kSubOut (2 HW + 1) FMAs for about HW + 2
// float4 LDS reads.  Each output sums a kernel row's products in binary32, taps
// in order, and the rows in binary64, rows in order.
template <int HW>
__global__ __launch_bounds__(kBlock) void k_subtract_t(
    const SubFrame* frames, int nframes, SubBasis bs, int64_t total_stamps) {
  constexpr int KW = 2 * HW + 1;
  constexpr int NR = (2 * HW + kSubOut + 3) / 4;  // float4s of a segment
  constexpr int KR = (KW + 3) / 4;            // float4s of a kernel row
  extern __shared__ __align__(16) unsigned char sub_lds[];
  double* a_s = (double*)sub_lds;             // a_n, then B at kSubMaxBasis
  float* ker = (float*)(a_s + kSubHead);
  const int S = bs.stamp, G = sub_groups(S);
  const int ks = sub_kstride(HW), ts = sub_tstride(S, HW);
  float* tile = ker + KW * ks;
  const int th = S + 2 * HW;
  const int t = threadIdx.x, nt = blockDim.x;
  const int ly = t / G, lx0 = kSubOut * (t - (t / G) * G);
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
    for (int n = t; n < bs.nbasis; n += nt)
      a_s[n] = poly2(fr.coef + (int64_t)n * ns, bs.spatial_order, xn, yn);
    if (t == 0)
      a_s[kSubMaxBasis] =
          poly2(fr.coef + (int64_t)bs.nbasis * ns, bs.bkg_order, xn, yn);
    // template tile with its margin, zero outside the frame (and in the
    // row padding)
    for (int e = t; e < th * ts; e += nt) {
      const int ty = e / ts, tx = e - ty * ts;
      const int gy = y0 - HW + ty, gx = x0 - HW + tx;
      float r = 0.0f;
      if (gy >= 0 && gy < fr.h && gx >= 0 && gx < fr.w && tx < S + 2 * HW)
        r = fr.R[(int64_t)gy * fr.pitchR + gx];
      tile[e] = r;
    }
    __syncthreads();
    // the stamp's kernel in binary64, kept as binary32 (row padding 0)
    for (int e = t; e < KW * ks; e += nt) {
      const int vv = e / ks, uu = e - vv * ks;
      float kv = 0.0f;
      if (uu < KW) {
        const double du = (double)(uu - HW), dv = (double)(vv - HW);
        double k = 0.0;
        int n = 0;
        for (int g = 0; g < bs.ngauss; ++g) {
          const double sg = bs.sigma[g];
          const double ex = exp(-(du * du + dv * dv) / (2.0 * sg * sg));
          double ui = 1.0;
          for (int i = 0; i <= bs.order[g]; ++i) {
            double vj = 1.0;
            for (int j = 0; j <= bs.order[g] - i; ++j) {
              k += a_s[n++] * (ex * ui * vj);
              vj *= dv;
            }
            ui *= du;
          }
        }
        kv = (float)k;
      }
      ker[e] = kv;
    }
    __syncthreads();
    const int ow = x1 - x0, oh = y1 - y0;
    if (ly < oh && lx0 < ow) {
      double acc[kSubOut];
#pragma unroll
      for (int i = 0; i < kSubOut; ++i) acc[i] = 0.0;
      for (int vv = 0; vv < KW; ++vv) {          // vv = v + HW
        // R(x - u, y - v) = tile[ly + 2HW - vv][lx + 2HW - uu]
        float r[4 * NR];
        const float4* trow =
            (const float4*)(tile + (ly + 2 * HW - vv) * ts + lx0);
#pragma unroll
        for (int q = 0; q < NR; ++q) {
          const float4 a = trow[q];
          r[4 * q] = a.x; r[4 * q + 1] = a.y;
          r[4 * q + 2] = a.z; r[4 * q + 3] = a.w;
        }
        float kr[4 * KR];
        const float4* krow = (const float4*)(ker + vv * ks);
#pragma unroll
        for (int q = 0; q < KR; ++q) {
          const float4 a = krow[q];
          kr[4 * q] = a.x; kr[4 * q + 1] = a.y;
          kr[4 * q + 2] = a.z; kr[4 * q + 3] = a.w;
        }
#pragma unroll
        for (int i = 0; i < kSubOut; ++i) {
          float rs = 0.0f;
#pragma unroll
          for (int uu = 0; uu < KW; ++uu)        // uu = u + HW
            rs = fmaf(kr[uu], r[i + 2 * HW - uu], rs);
          acc[i] += (double)rs;
        }
      }
      const double B = a_s[kSubMaxBasis];
      const int64_t gy = y0 + ly;
#pragma unroll
      for (int i = 0; i < kSubOut; ++i) {
        const int lx = lx0 + i;
        if (lx < ow) {
          const int64_t gx = x0 + lx;
          const double I = (double)fr.I[gy * fr.pitchI + gx];
          fr.D[gy * fr.w + gx] = (float)((I + B) - acc[i]);
        }
      }
    }
  }
}

#define IPP_SUB_INST(H)                                                  \
  template __global__ void k_subtract_t<H>(const SubFrame*, int, SubBasis, \
                                           int64_t);
IPP_SUB_INST(1) IPP_SUB_INST(2) IPP_SUB_INST(3) IPP_SUB_INST(4)
IPP_SUB_INST(5) IPP_SUB_INST(6) IPP_SUB_INST(7) IPP_SUB_INST(8)
IPP_SUB_INST(9) IPP_SUB_INST(10) IPP_SUB_INST(11) IPP_SUB_INST(12)
IPP_SUB_INST(13) IPP_SUB_INST(14) IPP_SUB_INST(15)
#undef IPP_SUB_INST

}  // namespace ipp
