// Aperture photometry with a local sky annulus (Sec. 2.2.5: per-object
// aperture photometry).  One 256-thread workgroup per source: every window
// pixel gets its exact circle/pixel overlap weights in binary64, the annulus
// values are sorted in LDS (bitonic), and the k-sigma clipping of the sky
// then works on contiguous ranges of the sorted values.
#include "ipp_internal.h"
#include "kernels.h"
#include "phot_geom.h"

namespace ipp {

namespace {
constexpr int kSortMax = 1024;     // annulus pixels (r_out <= 16)
constexpr int kPixPerThread = 5;   // window pixels per thread (34 x 34)
}  // namespace

__global__ __launch_bounds__(kBlock) void k_aperture(Work wk, ipp_params p,
                                                     ipp_sources src,
                                                     double* sky_lohi) {
  __shared__ double sbuf[kSortMax];
  __shared__ double dred[kWaves];
  __shared__ int ired[kWaves];
  __shared__ int cnt_s;
  const int t = threadIdx.x;
  long long nrows = src.capacity;
  if (src.n_total && *src.n_total < nrows) nrows = *src.n_total;
  const double R = p.r_ap > p.r_out ? p.r_ap : p.r_out;
  for (long long row = blockIdx.x; row < nrows; row += gridDim.x) {
    const int f = src.frame[row];
    const double cx = src.x[row], cy = src.y[row];
    const bool fok = f >= 0 && f < wk.nframes;
    const FrameDev fr = wk.frames[fok ? f : 0];
    uint32_t flags = 0;
    if (!fok || !(isfinite(cx) && isfinite(cy)) || fabs(cx) > 1e9 ||
        fabs(cy) > 1e9) {
      if (t == 0) {
        src.flux_ap[row] = __builtin_nan("");
        src.sky[row] = __builtin_nan("");
        src.area_ap[row] = 0.0;
        src.area_ann[row] = 0.0;
        src.flags[row] |= IPP_SRC_APERTURE_OFF_EDGE | IPP_SRC_NO_SKY;
        if (sky_lohi) { sky_lohi[2 * row] = 0.0; sky_lohi[2 * row + 1] = -1.0; }
      }
      continue;
    }
    const int xa = (int)ceil(cx - R - 0.5), xb = (int)floor(cx + R + 0.5);
    const int ya = (int)ceil(cy - R - 0.5), yb = (int)floor(cy + R + 0.5);
    const int nwx = xb - xa + 1, npx = nwx * (yb - ya + 1);
    if (t == 0) cnt_s = 0;
    __syncthreads();
    double pv[kPixPerThread], pwa[kPixPerThread], pwn[kPixPerThread];
    uint32_t okm = 0, annm = 0;
    double a_ap = 0.0, raw = 0.0;
#pragma unroll
    for (int k = 0; k < kPixPerThread; ++k) {
      pv[k] = 0.0; pwa[k] = 0.0; pwn[k] = 0.0;
      const int e = t + k * kBlock;
      if (e >= npx) continue;
      const int px = xa + e % nwx, py = ya + e / nwx;
      const bool in_ap = touches(cx, cy, p.r_ap, px, py);
      const bool in_ann = touches(cx, cy, p.r_out, px, py) &&
                          !within(cx, cy, p.r_in, px, py);
      if (!(in_ap || in_ann)) continue;
      bool ok = px >= 0 && px < fr.w && py >= 0 && py < fr.h;
      double v = 0.0;
      if (ok) {
        const float I = fr.pix[(int64_t)py * fr.pitch + px];
        ok = isfinite(I);
        v = (double)I - (double)fr.bkg[(int64_t)py * fr.w + px];
      }
      if (!ok) {
        if (in_ap) flags |= IPP_SRC_APERTURE_OFF_EDGE;
        if (in_ann) flags |= IPP_SRC_ANNULUS_OFF_EDGE;
        continue;
      }
      okm |= 1u << k;
      pv[k] = v;
      if (in_ap) {
        const double wa = overlap(cx, cy, p.r_ap, px, py);
        pwa[k] = wa;
        a_ap += wa;
        raw += wa * v;
      }
      if (in_ann) {
        pwn[k] = overlap(cx, cy, p.r_out, px, py) -
                 overlap(cx, cy, p.r_in, px, py);
        annm |= 1u << k;
        const int slot = atomicAdd(&cnt_s, 1);
        if (slot < kSortMax) sbuf[slot] = v;
      }
    }
    __syncthreads();
    int nann = cnt_s;
    if (nann > kSortMax) nann = kSortMax;      // not reachable for r <= 16
    int ns = 64;
    while (ns < nann) ns <<= 1;
    for (int i = nann + t; i < ns; i += kBlock) sbuf[i] = __builtin_inf();
    __syncthreads();
    // bitonic sort of sbuf[0, ns)
    for (int kk = 2; kk <= ns; kk <<= 1) {
      for (int j = kk >> 1; j > 0; j >>= 1) {
        for (int i = t; i < ns; i += kBlock) {
          const int l = i ^ j;
          if (l > i) {
            const double a = sbuf[i], b = sbuf[l];
            const bool up = (i & kk) == 0;
            if ((a > b) == up) { sbuf[i] = b; sbuf[l] = a; }
          }
        }
        __syncthreads();
      }
    }
    // k-sigma clipping on the sorted range [a, b)
    int a = 0, b = nann;
    for (int it = 0; it < p.sky_clip_iters; ++it) {
      const int n = b - a;
      if (n == 0) break;
      double med = (n & 1) ? sbuf[a + (n - 1) / 2]
                           : (sbuf[a + n / 2 - 1] + sbuf[a + n / 2]) / 2.0;
      double s1 = 0.0;
      for (int i = a + t; i < b; i += kBlock) s1 += sbuf[i];
      s1 = block_sum(s1, dred);
      const double mean = s1 / (double)n;
      double s2 = 0.0;
      for (int i = a + t; i < b; i += kBlock) {
        const double d = sbuf[i] - mean;
        s2 += d * d;
      }
      s2 = block_sum(s2, dred);
      const double sd = sqrt(s2 / (double)n);
      const double lo = med - p.sky_clip_sigma * sd;
      const double hi = med + p.sky_clip_sigma * sd;
      int cl = 0, ch = 0;
      for (int i = a + t; i < b; i += kBlock) {
        cl += sbuf[i] < lo;
        ch += sbuf[i] > hi;
      }
      cl = block_sum(cl, ired);
      ch = block_sum(ch, ired);
      if (cl == 0 && ch == 0) break;
      a += cl;
      b -= ch;
    }
    double vlo = 0.0, vhi = -1.0;
    if (b > a) { vlo = sbuf[a]; vhi = sbuf[b - 1]; }
    // weighted sky over the surviving annulus pixels
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int k = 0; k < kPixPerThread; ++k) {
      if (((annm >> k) & 1u) && pv[k] >= vlo && pv[k] <= vhi) {
        num += pwn[k] * pv[k];
        den += pwn[k];
      }
    }
    num = block_sum(num, dred);
    den = block_sum(den, dred);
    a_ap = block_sum(a_ap, dred);
    raw = block_sum(raw, dred);
    for (int o = kWave / 2; o > 0; o >>= 1) flags |= __shfl_xor(flags, o, kWave);
    if ((t & (kWave - 1)) == 0) ired[t / kWave] = (int)flags;
    __syncthreads();
    if (t == 0) {
      uint32_t fl = (uint32_t)(ired[0] | ired[1] | ired[2] | ired[3]);
      double sky = 0.0;
      if (den > 0.0) sky = num / den; else fl |= IPP_SRC_NO_SKY;
      src.flux_ap[row] = raw - sky * a_ap;
      src.sky[row] = sky;
      src.area_ap[row] = a_ap;
      src.area_ann[row] = den;
      src.flags[row] |= fl;
      if (sky_lohi) { sky_lohi[2 * row] = vlo; sky_lohi[2 * row + 1] = vhi; }
    }
    __syncthreads();
  }
}

}  // namespace ipp
