// Gray-scale transformations (Sec. 2.2.6): the zscale display range of a
// frame, point maps (linear, logarithmic, exponential, power law) over a
// value range, and histogram equalization (pixel counts per gray level,
// their cumulative distribution, and an interpolating map onto it).
//
// zscale follows the display-range estimate of SAOimage DS9 and IRAF:
// sort a grid sample of the frame, fit a straight line to the sorted values
// against their index with iterative rejection of outlying samples (each
// rejection widened to its neighbours), and evaluate the line, with its
// slope divided by a contrast factor, at the ends of the index range
// through the median.
#include "ipp_internal.h"
#include "kernels.h"

namespace ipp {

namespace {

// Frame of a flat row index, given each frame's first row (ascending).
__device__ __forceinline__ int gray_frame_of(const GrayFrame* fr, int n,
                                             int row) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (fr[mid].row0 <= row) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Rows [r0, r1) of the batch handled by this block: contiguous ranges, so
// that a block meets few frame changes.
__device__ __forceinline__ void block_rows(int total_rows, int* r0, int* r1) {
  const int per = (total_rows + gridDim.x - 1) / gridDim.x;
  *r0 = min(total_rows, (int)blockIdx.x * per);
  *r1 = min(total_rows, *r0 + per);
}

// ln(1 + u) for u >= 0 in binary32, from w = fl(1 + u): ln(w) u / (w - 1)
// (Goldberg, "What every computer scientist should know about
// floating-point arithmetic", 1991, Thm. 4), with the hardware log2.
__device__ __forceinline__ float log1p_g(float u) {
  const float w = 1.0f + u;
  if (w == 1.0f) return u;
  return 0.69314718f * __builtin_amdgcn_logf(w) * (u / (w - 1.0f));
}

// e^t - 1 in binary32 from u = fl(e^t): (u - 1) t / ln(u) (W. Kahan's
// identity), with the hardware exp2 and log2.
__device__ __forceinline__ float expm1_k(float t) {
  const float u = __builtin_amdgcn_exp2f(t * 1.44269504f);
  if (u == 1.0f) return t;
  const float lu = 0.69314718f * __builtin_amdgcn_logf(u);
  return (u - 1.0f) * (t / lu);
}

struct MapConst {
  int kind;
  float a;          // the map's parameter
  float c;          // LOG: 1 / ln(1 + a); EXP: 1 / (a - 1)
  float lna;        // EXP: ln a
};

// Gray level of one pixel: x = (v - lo) / (hi - lo) in binary64, clipped
// to [0, 1], then the map in binary32.
__device__ __forceinline__ float map_pixel(float v, double lo, double inv,
                                           bool step, const MapConst& m) {
  if (!isfinite(v)) return __builtin_nanf("");
  double xd = step ? ((double)v <= lo ? 0.0 : 1.0) : ((double)v - lo) * inv;
  xd = fmin(fmax(xd, 0.0), 1.0);
  const float x = (float)xd;
  switch (m.kind) {
    case IPP_MAP_LOG:
      return log1p_g(m.a * x) * m.c;
    case IPP_MAP_EXP:
      return expm1_k(x * m.lna) * m.c;
    case IPP_MAP_POWER: {
      if (xd <= 0.0) return 0.0f;
      // log2 of the binary64 x through its exponent (x may be below the
      // binary32 normal range)
      int e;
      const double mant = frexp(xd, &e);              // [0.5, 1)
      const float l2 = (float)e + __builtin_amdgcn_logf((float)mant);
      return __builtin_amdgcn_exp2f(m.a * l2);
    }
    default:
      return x;
  }
}

// Row y of frame F: fn(v, out_row, x) with v a float4 of columns x..x+3
// (aligned rows) or a float of column x.  Two groups per thread are loaded
// before either is used, so that both loads are in flight together.
template <typename Fn>
__device__ __forceinline__ void row_elements(const GrayFrame& F, int y,
                                             bool vec, Fn fn) {
  const float* in = F.pix + (int64_t)y * F.pitch;
  float* out = F.out ? F.out + (int64_t)y * F.w : nullptr;
  int x0 = 0;
  if (vec) {
    const int n4 = F.w >> 2;
    const float4* in4 = (const float4*)in;
    int i = threadIdx.x;
    for (; i + kBlock < n4; i += 2 * kBlock) {
      const float4 a = in4[i], b = in4[i + kBlock];
      fn(a, out, 4 * i);
      fn(b, out, 4 * (i + kBlock));
    }
    if (i < n4) fn(in4[i], out, 4 * i);
    x0 = n4 << 2;
  }
  for (int x = x0 + threadIdx.x; x < F.w; x += kBlock) fn(in[x], out, x);
}

__device__ __forceinline__ bool row_vec(const GrayFrame& F) {
  return ((F.pitch | F.w) & 3) == 0 && ((uintptr_t)F.pix & 15) == 0 &&
         (!F.out || ((uintptr_t)F.out & 15) == 0);
}

}  // namespace

// ---------------------------------------------------------------------
// zscale: one workgroup per frame.
// ---------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_zscale(const GrayFrame* frames,
                                                   double contrast,
                                                   double krej, int max_iter,
                                                   double* z1z2,
                                                   double* info) {
  __shared__ float sv[kZMax];
  __shared__ uint8_t bad[kZMax];
  __shared__ uint8_t rej[kZMax];
  __shared__ double redd[kWaves];
  __shared__ int redi[kWaves];
  const int f = blockIdx.x;
  const GrayFrame F = frames[f];
  const int t = threadIdx.x;
  const int ns = F.sy * F.sx;          // <= kZMax, checked on the host
  // ---- the grid sample; non-finite values and padding sort last --------
  int nfin = 0;
  for (int e = t; e < kZMax; e += kBlock) {
    float v = __builtin_inff();
    if (e < ns) {
      const int i = e / F.sx, j = e - (e / F.sx) * F.sx;
      const float x =
          F.pix[(int64_t)i * F.s * F.pitch + (int64_t)j * F.s];
      if (isfinite(x)) {
        v = x;
        ++nfin;
      }
    }
    sv[e] = v;
    bad[e] = 0;
  }
  const int n = block_sum(nfin, redi);
  // ---- bitonic sort, ascending -------------------------------------------
  for (int k = 2; k <= kZMax; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      __syncthreads();
      for (int e = t; e < kZMax / 2; e += kBlock) {
        const int lo = 2 * e - (e & (j - 1));        // index bit of j clear
        const int hi = lo + j;
        const bool up = (lo & k) == 0;
        const float a = sv[lo], b = sv[hi];
        if ((a > b) == up) {
          sv[lo] = b;
          sv[hi] = a;
        }
      }
    }
  }
  __syncthreads();
  if (n == 0) {
    if (t == 0) {
      z1z2[2 * f] = 0.0;
      z1z2[2 * f + 1] = 0.0;
      if (info) {
        info[4 * f] = 0.0;
        info[4 * f + 1] = 0.0;
        info[4 * f + 2] = 0.0;
        info[4 * f + 3] = 0.0;
      }
    }
    return;
  }
  // median of the sorted sample (Eq. 1)
  const double med = (n & 1) ? (double)sv[(n - 1) / 2]
                             : ((double)sv[n / 2 - 1] + (double)sv[n / 2]) /
                                   2.0;
  const int minpix = max(5, n / 2);
  const int half = max(1, n / 100) / 2;
  int kept = n, last = n + 1, fits = 0;
  double b = 0.0;
  while (fits < max_iter && kept < last && kept >= minpix) {
    // ---- least-squares line over the kept samples ---------------------
    double sx = 0.0, sxx = 0.0, sy = 0.0, sxy = 0.0;
    for (int e = t; e < n; e += kBlock) {
      if (bad[e]) continue;
      const double i = (double)e, v = (double)sv[e];
      sx += i;
      sxx += i * i;
      sy += v;
      sxy += i * v;
    }
    sx = block_sum(sx, redd);
    sxx = block_sum(sxx, redd);
    sy = block_sum(sy, redd);
    sxy = block_sum(sxy, redd);
    const double nk = (double)kept;
    const double den = nk * sxx - sx * sx;
    b = den != 0.0 ? (nk * sxy - sx * sy) / den : 0.0;
    const double a = (sy - b * sx) / nk;
    ++fits;
    // ---- scale: ddof-0 deviation of the kept residuals ----------------
    double s1 = 0.0;
    for (int e = t; e < n; e += kBlock)
      if (!bad[e]) s1 += (double)sv[e] - (a + b * (double)e);
    const double mu = block_sum(s1, redd) / nk;
    double s2 = 0.0;
    for (int e = t; e < n; e += kBlock) {
      if (bad[e]) continue;
      const double d = ((double)sv[e] - (a + b * (double)e)) - mu;
      s2 += d * d;
    }
    const double thr = krej * sqrt(block_sum(s2, redd) / nk);
    // ---- reject, widen each rejection, count --------------------------
    for (int e = t; e < n; e += kBlock)
      rej[e] = fabs((double)sv[e] - (a + b * (double)e)) > thr;
    __syncthreads();
    int nk2 = 0;
    for (int e = t; e < n; e += kBlock) {
      bool out = bad[e];
      const int j0 = max(0, e - half), j1 = min(n - 1, e + half);
      for (int j = j0; j <= j1 && !out; ++j) out = rej[j];
      bad[e] = out;
      nk2 += !out;
    }
    last = kept;
    kept = block_sum(nk2, redi);
  }
  if (t == 0) {
    double z1 = (double)sv[0], z2 = (double)sv[n - 1];
    if (kept >= minpix) {
      const double slope = contrast > 0.0 ? b / contrast : b;
      const int c = (n - 1) / 2;
      z1 = fmax(z1, med - (double)c * slope);
      z2 = fmin(z2, med + (double)(n - 1 - c) * slope);
    }
    z1z2[2 * f] = z1;
    z1z2[2 * f + 1] = z2;
    if (info) {
      info[4 * f] = (double)n;
      info[4 * f + 1] = (double)kept;
      info[4 * f + 2] = (double)fits;
      info[4 * f + 3] = b;
    }
  }
}

// ---------------------------------------------------------------------
// Point map of every frame over [lohi[2f], lohi[2f+1]].
// ---------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_gray_map(
    const GrayFrame* frames, int nframes, int total_rows, int kind, float a,
    float c, float lna, const double* lohi) {
  const MapConst m = {kind, a, c, lna};
  for (int row = blockIdx.x; row < total_rows; row += gridDim.x) {
    const int f = gray_frame_of(frames, nframes, row);
    const GrayFrame F = frames[f];
    const int y = row - F.row0;
    const double lo = lohi[2 * f], hi = lohi[2 * f + 1];
    const bool step = !(hi > lo);
    const double inv = step ? 0.0 : 1.0 / (hi - lo);
    row_elements(F, y, row_vec(F), [&](auto v, float* out, int x) {
      if constexpr (sizeof(v) == sizeof(float4)) {
        float4 o;
        o.x = map_pixel(v.x, lo, inv, step, m);
        o.y = map_pixel(v.y, lo, inv, step, m);
        o.z = map_pixel(v.z, lo, inv, step, m);
        o.w = map_pixel(v.w, lo, inv, step, m);
        *(float4*)(out + x) = o;
      } else {
        out[x] = map_pixel(v, lo, inv, step, m);
      }
    });
  }
}

// ---------------------------------------------------------------------
// Histogram equalization.
// ---------------------------------------------------------------------
// Smallest and largest finite value of every frame, as ordered keys in
// mm[f] (min, starts at ~0) and mm[nframes + f] (max, starts at 0).
__global__ __launch_bounds__(kBlock) void k_eq_minmax(const GrayFrame* frames,
                                                      int nframes,
                                                      int total_rows,
                                                      uint32_t* mm) {
  __shared__ uint32_t red[kWaves];
  int r0, r1;
  block_rows(total_rows, &r0, &r1);
  if (r0 >= r1) return;
  int f = gray_frame_of(frames, nframes, r0);
  uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
  for (int row = r0; row < r1; ++row) {
    while (f + 1 < nframes && frames[f + 1].row0 <= row) {
      // frame change: flush this frame's partial range
      const uint32_t bmin = block_min(kmin, red);
      const uint32_t bmax = block_max(kmax, red);
      if (threadIdx.x == 0 && bmin <= bmax) {
        atomicMin(&mm[f], bmin);
        atomicMax(&mm[nframes + f], bmax);
      }
      kmin = 0xFFFFFFFFu;
      kmax = 0u;
      ++f;
    }
    const GrayFrame F = frames[f];
    auto take = [&](float v) {
      if (isfinite(v)) {
        const uint32_t k = f2key(v + 0.0f);
        kmin = min(kmin, k);
        kmax = max(kmax, k);
      }
    };
    row_elements(F, row - F.row0, row_vec(F), [&](auto v, float*, int) {
      if constexpr (sizeof(v) == sizeof(float4)) {
        take(v.x); take(v.y); take(v.z); take(v.w);
      } else {
        take(v);
      }
    });
  }
  const uint32_t bmin = block_min(kmin, red);
  const uint32_t bmax = block_max(kmax, red);
  if (threadIdx.x == 0 && bmin <= bmax) {
    atomicMin(&mm[f], bmin);
    atomicMax(&mm[nframes + f], bmax);
  }
}

// Bin of a finite value: floor(((v - lo) / (hi - lo)) * nbins), the top
// value in the last bin (binary64, division as written).  t = (v - lo) *
// (nbins / (hi - lo)) is within a few units in the last place (< 4e-12 for
// t <= 4096) of the value the written form floors, so where t is more than
// 1e-9 from an integer its floor is the bin; values nearer a bin edge take
// the division.
__device__ __forceinline__ int eq_bin(float v, double lo, double range,
                                      double scale, int nbins) {
  const double d = (double)v - lo;
  const double t = d * scale;
  const double ft = floor(t);
  const double fr = t - ft;
  int k = (int)ft;
  if (fr < 1e-9 || fr > 1.0 - 1e-9)
    k = (int)floor((d / range) * (double)nbins);
  return min(k, nbins - 1);
}

// Per-block LDS histograms in two copies (lane parity picks the copy, the
// copies of a bin sit in adjacent banks), so that the many lanes whose sky
// values fall in the same few bins collide half as often; each lane merges
// equal bins among its four values before adding.
__global__ __launch_bounds__(kBlock) void k_eq_hist(const GrayFrame* frames,
                                                    int nframes,
                                                    int total_rows, int nbins,
                                                    const uint32_t* mm,
                                                    uint32_t* counts) {
  __shared__ uint32_t h[2 * kMaxBins];
  int r0, r1;
  block_rows(total_rows, &r0, &r1);
  if (r0 >= r1) return;
  const uint32_t rep = threadIdx.x & 1u;
  for (int i = threadIdx.x; i < 2 * nbins; i += kBlock) h[i] = 0;
  __syncthreads();
  int f = gray_frame_of(frames, nframes, r0);
  auto flush = [&](int fr) {
    __syncthreads();
    for (int i = threadIdx.x; i < nbins; i += kBlock) {
      const uint32_t c = h[2 * i] + h[2 * i + 1];
      if (c) atomicAdd(&counts[(size_t)fr * nbins + i], c);
      h[2 * i] = 0;
      h[2 * i + 1] = 0;
    }
    __syncthreads();
  };
  int64_t held = 0;                        // pixels counted since a flush
  for (int row = r0; row < r1; ++row) {
    while (f + 1 < nframes && frames[f + 1].row0 <= row) {
      flush(f);
      held = 0;
      ++f;
    }
    const GrayFrame F = frames[f];
    if (held + F.w > (int64_t)1 << 31) {     // keep the 32-bit counters exact
      flush(f);
      held = 0;
    }
    held += F.w;
    const uint32_t kl = mm[f], kh = mm[nframes + f];
    if (kl > kh) continue;                 // no finite value in the frame
    const double lo = (double)key2f(kl), hi = (double)key2f(kh);
    const double range = hi - lo;
    const double scale = range > 0.0 ? (double)nbins / range : 0.0;
    auto bin = [&](float v) -> int {       // -1: not finite
      if (!isfinite(v)) return -1;
      return range > 0.0 ? eq_bin(v, lo, range, scale, nbins) : 0;
    };
    auto add = [&](int k, uint32_t c) {
      if (k >= 0) atomicAdd(&h[2 * k + rep], c);
    };
    row_elements(F, row - F.row0, row_vec(F), [&](auto v, float*, int) {
      if constexpr (sizeof(v) == sizeof(float4)) {
        const int k0 = bin(v.x), k1 = bin(v.y);
        const int k2 = bin(v.z), k3 = bin(v.w);
        // runs of equal bins among the four
        uint32_t c = 1;
        if (k1 == k0) ++c; else { add(k0, c); c = 1; }
        if (k2 == k1) ++c; else { add(k1, c); c = 1; }
        if (k3 == k2) ++c; else { add(k2, c); c = 1; }
        add(k3, c);
      } else {
        add(bin(v), 1u);
      }
    });
  }
  flush(f);
}

// cdf[f][k] = (pixels of frame f in bins 0..k) / (its finite pixels): one
// workgroup per frame, kMaxBins / kBlock consecutive bins per thread.
__global__ __launch_bounds__(kBlock) void k_eq_cdf(const uint32_t* counts,
                                                   int nbins, double* cdf) {
  __shared__ int red[kWaves];
  constexpr int kPer = kMaxBins / kBlock;
  const int f = blockIdx.x;
  const uint32_t* c = counts + (size_t)f * nbins;
  double* out = cdf + (size_t)f * nbins;
  const int b0 = threadIdx.x * kPer;
  int own = 0;
  for (int i = 0; i < kPer; ++i)
    if (b0 + i < nbins) own += (int)c[b0 + i];
  int total;
  const int before = block_exclusive_scan(own, red, &total);
  if (total == 0) return;
  int run = before;
  for (int i = 0; i < kPer; ++i) {
    if (b0 + i >= nbins) break;
    run += (int)c[b0 + i];
    out[b0 + i] = (double)run / (double)total;
  }
}

// y = the interpolation of (centre_k, cdf_k) at v, held at the ends.  Each
// block maps a contiguous range of rows; the cdf of the frame being mapped
// is staged in LDS in binary32 (values in [0, 1]: 6e-8 absolute).  The
// position of v among the centres, t = (v - lo) / w - 1/2, is taken in
// binary64 (v - lo exactly); the interpolation is continuous, so the
// interval a value on a centre falls in does not change y.
__global__ __launch_bounds__(kBlock) void k_eq_map(const GrayFrame* frames,
                                                   int nframes,
                                                   int total_rows, int nbins,
                                                   const uint32_t* mm,
                                                   const double* cdf) {
  __shared__ float T[kMaxBins];
  int r0, r1;
  block_rows(total_rows, &r0, &r1);
  if (r0 >= r1) return;
  int f = -1;
  double lo = 0.0, inv_w = 0.0;
  bool span = false;
  for (int row = r0; row < r1; ++row) {
    int nf = f < 0 ? gray_frame_of(frames, nframes, row) : f;
    while (nf + 1 < nframes && frames[nf + 1].row0 <= row) ++nf;
    if (nf != f) {
      // a new frame: its value range and cdf
      f = nf;
      const uint32_t kl = mm[f], kh = mm[nframes + f];
      const double l = kl <= kh ? (double)key2f(kl) : 0.0;
      const double h = kl <= kh ? (double)key2f(kh) : 0.0;
      lo = l;
      span = h > l;
      inv_w = span ? (double)nbins / (h - l) : 0.0;
      __syncthreads();
      if (span)
        for (int k = threadIdx.x; k < nbins; k += kBlock)
          T[k] = (float)cdf[(size_t)f * nbins + k];
      __syncthreads();
    }
    const GrayFrame F = frames[f];
    auto eq = [&](float vf) -> float {
      if (!isfinite(vf)) return __builtin_nanf("");
      if (!span) return 1.0f;
      const double t = ((double)vf - lo) * inv_w - 0.5;
      if (t < 0.0) return T[0];
      const int j = (int)t;
      if (j >= nbins - 1) return T[nbins - 1];
      const float fr = (float)(t - (double)j);
      const float y0 = T[j];
      return y0 + (T[j + 1] - y0) * fr;
    };
    row_elements(F, row - F.row0, row_vec(F), [&](auto v, float* out, int x) {
      if constexpr (sizeof(v) == sizeof(float4)) {
        float4 o;
        o.x = eq(v.x); o.y = eq(v.y); o.z = eq(v.z); o.w = eq(v.w);
        *(float4*)(out + x) = o;
      } else {
        out[x] = eq(v);
      }
    });
  }
}

}  // namespace ipp
