// Background mesh: sigma-clipped statistics of every region (Sec. 2.2.2,
// Eq. 1-4 and the clipping loop), then invalid-node fill, median filter and
// natural-spline tables per frame.
//
// k_mesh_stats: one 256-thread workgroup per region.  The region's pixels
// stay in registers as order-preserving uint32 keys of their float32 values.
// Every set the clipping loop visits is a key interval of the region's
// finite, unmasked pixels, so each median is an order statistic of that one
// multiset.  A 2048-bin histogram is built once over a robust key range
// (the inter-quartile range of a 256-pixel sample, widened by four IQRs on
// each side; everything outside falls into an end bin), so the middle order
// statistics land in bins of a few keys: both are found by one gather of
// their bins and an exact rank count.  Dense or end bins are narrowed with
// a second histogram.  Means and deviations are binary64 block sums in a
// fixed order, taken about the median.
#include "ipp_internal.h"
#include "kernels.h"

namespace ipp {

namespace {

constexpr int kBins = 2048;       // bin 0: below the range, kBins-1: above
constexpr int kGather = 256;

struct MeshLds {
  uint32_t c1[kBins + 1];     // level-1 exclusive prefix counts
  uint32_t h2[kBins];         // narrowing histogram; sample buffer first
  uint32_t list[kGather];     // gathered keys
  uint32_t sel[4];            // query results / counters
  uint32_t ured[kWaves];
  int ired[kWaves];
  double dred[2 * kWaves];
};

struct Bins {
  uint32_t kmin, kmax, klo, khi;
  int sh;
};

__device__ __forceinline__ int bin_of(uint32_t k, const Bins& b) {
  if (k < b.klo) return 0;
  if (k > b.khi) return kBins - 1;
  return 1 + (int)((k - b.klo) >> b.sh);
}

// Key range [lo, hi] of level-1 bin j (only asked for non-empty bins).
__device__ __forceinline__ void bin_range(int j, const Bins& b, uint64_t* lo,
                                          uint64_t* hi) {
  if (j == 0) {
    *lo = b.kmin;
    *hi = (uint64_t)b.klo - 1;
  } else if (j == kBins - 1) {
    *lo = (uint64_t)b.khi + 1;
    *hi = b.kmax;
  } else {
    *lo = (uint64_t)b.klo + ((uint64_t)(j - 1) << b.sh);
    const uint64_t h = *lo + ((1ull << b.sh) - 1);
    *hi = h < b.khi ? h : b.khi;
  }
}

// Largest j with c1[j] <= r: the non-empty bin holding rank r.
__device__ __forceinline__ int rank_bin(const uint32_t* c1, int r) {
  int lo = 0, hi = kBins - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int)c1[mid] <= r) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__device__ __forceinline__ void block_sum2(T& a, T& b, T* red) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) {
    red[w] = a;
    red[kWaves + w] = b;
  }
  __syncthreads();
  a = (red[0] + red[1]) + (red[2] + red[3]);
  b = (red[4] + red[5]) + (red[6] + red[7]);
}

// Block-wide exclusive scan of kBins counters held in h (8 per thread):
// finds the bin containing rank `r` (0-based).  Writes (bin, prefix, count)
// into out[0..2] in LDS.
__device__ void find_rank_bin(const uint32_t* h, int r, uint32_t* out,
                              int* ired) {
  const int t = threadIdx.x;
  uint32_t loc[8];
  int s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) { loc[i] = h[t * 8 + i]; s += (int)loc[i]; }
  int total;
  int ex = block_exclusive_scan(s, ired, &total);
  if (r >= ex && r < ex + s) {
    int acc = ex;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (r >= acc && r < acc + (int)loc[i]) {
        out[0] = (uint32_t)(t * 8 + i);
        out[1] = (uint32_t)acc;
        out[2] = loc[i];
      }
      acc += (int)loc[i];
    }
  }
  __syncthreads();
}

// Gathers the keys of [lo, hi] (cnt of them, cnt <= kGather) and returns
// the keys of within-range ranks w0 and w1 in L.sel[0], L.sel[1].
template <int PPT>
__device__ void gather_select(const uint32_t (&key)[PPT], uint64_t lo,
                              uint64_t hi, int cnt, int w0, int w1,
                              MeshLds& L) {
  __syncthreads();
  if (threadIdx.x == 0) L.sel[3] = 0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const uint32_t v = key[k];
    if (v != kSentinel && v >= lo && v <= hi) {
      const uint32_t slot = atomicAdd(&L.sel[3], 1u);
      L.list[slot] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < cnt) {
    const uint32_t me = L.list[threadIdx.x];
    int less = 0;
    for (int i = 0; i < cnt; ++i) {
      const uint32_t o = L.list[i];
      less += (o < me) || (o == me && i < (int)threadIdx.x);
    }
    if (less == w0) L.sel[0] = me;
    if (less == w1) L.sel[1] = me;
  }
  __syncthreads();
}

// Key of rank `rank`, narrowing the level-1 bin that holds it with second
// histograms until at most kGather keys remain.
template <int PPT>
__device__ uint32_t select_narrow(const uint32_t (&key)[PPT], int rank,
                                  const Bins& B, MeshLds& L) {
  const int j = rank_bin(L.c1, rank);
  uint64_t lo, hi;
  bin_range(j, B, &lo, &hi);
  int base = (int)L.c1[j];
  int cnt = (int)(L.c1[j + 1] - L.c1[j]);
  for (int level = 0; level < 5; ++level) {
    if (lo == hi) return (uint32_t)lo;
    if (cnt <= kGather) {
      gather_select<PPT>(key, lo, hi, cnt, rank - base, rank - base, L);
      const uint32_t res = L.sel[0];
      __syncthreads();
      return res;
    }
    const uint32_t range = (uint32_t)(hi - lo);
    const int bits = 32 - __clz(range);
    const int sh = bits > 11 ? bits - 11 : 0;
    for (int i = threadIdx.x; i < kBins; i += kBlock) L.h2[i] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const uint32_t v = key[k];
      if (v != kSentinel && v >= lo && v <= hi)
        atomicAdd(&L.h2[(uint32_t)(v - lo) >> sh], 1u);
    }
    __syncthreads();
    find_rank_bin(L.h2, rank - base, L.sel, L.ired);
    const uint32_t b = L.sel[0];
    const int pre = (int)L.sel[1];
    cnt = (int)L.sel[2];
    __syncthreads();
    lo = lo + ((uint64_t)b << sh);
    const uint64_t nhi = lo + ((1ull << sh) - 1);
    hi = nhi < hi ? nhi : hi;
    base += pre;
  }
  return (uint32_t)lo;  // not reached: the key range is exhausted by then
}

// Keys of ranks r0 and r1 = r0 or r0 + 1.
template <int PPT>
__device__ void select_pair(const uint32_t (&key)[PPT], int r0, int r1,
                            const Bins& B, MeshLds& L, uint32_t* k0,
                            uint32_t* k1) {
  const int j0 = rank_bin(L.c1, r0), j1 = rank_bin(L.c1, r1);
  const int base = (int)L.c1[j0];
  const int cnt = (int)(L.c1[j1 + 1] - L.c1[j0]);
  if (cnt <= kGather) {
    uint64_t lo, hi, lo1, hi1;
    bin_range(j0, B, &lo, &hi);
    bin_range(j1, B, &lo1, &hi1);
    gather_select<PPT>(key, lo, hi1, cnt, r0 - base, r1 - base, L);
    *k0 = L.sel[0];
    *k1 = L.sel[1];
    __syncthreads();
    return;
  }
  *k0 = select_narrow<PPT>(key, r0, B, L);
  *k1 = r1 == r0 ? *k0 : select_narrow<PPT>(key, r1, B, L);
}

// Smallest key whose float value is >= lo / largest with value <= hi.
__device__ __forceinline__ uint32_t key_ceil(double lo) {
  float f = (float)lo;
  uint32_t k = f2key(f);
  if ((double)f < lo) k += 1;
  return k;
}
__device__ __forceinline__ uint32_t key_floor(double hi) {
  float f = (float)hi;
  uint32_t k = f2key(f);
  if ((double)f > hi) k -= 1;
  // hi = -0.0 admits +0.0 (no pixel value is -0.0 after normalisation)
  if (k == 0x7FFFFFFFu) k = 0x80000000u;
  return k;
}

}  // namespace

template <int PPT>
__global__ __launch_bounds__(kBlock) void k_mesh_stats(Work wk,
                                                       ipp_params p) {
  __shared__ MeshLds L;
  const int t = threadIdx.x;
  const int region = blockIdx.x;
  const int f = find_frame(wk.frames, wk.nframes, region, &FrameDev::node0);
  const FrameDev fr = wk.frames[f];
  const int local = region - fr.node0;
  const int rj = local / fr.nx, ri = local - rj * fr.nx;
  const int y0 = rj * p.mesh_h, x0 = ri * p.mesh_w;
  const int th = min(p.mesh_h, fr.h - y0), tw = min(p.mesh_w, fr.w - x0);
  const int P = th * tw;

  // ---- load the region as keys -------------------------------------
  uint32_t key[PPT];
  int r = t / tw, c = t - (t / tw) * tw;
  const int qr = kBlock / tw, qc = kBlock - (kBlock / tw) * tw;
  int nloc = 0;
  uint32_t kmin_l = kSentinel, kmax_l = 0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    uint32_t kk = kSentinel;
    if (k * kBlock + t < P) {
      const int64_t o = (int64_t)(y0 + r) * fr.pitch + (x0 + c);
      float v = fr.pix[o];
      bool ok = isfinite(v);
      if (fr.mask && fr.mask[o]) ok = false;
      if (ok) {
        v = v + 0.0f;                       // -0 -> +0
        kk = f2key(v);
        ++nloc;
        kmin_l = min(kmin_l, kk);
        kmax_l = max(kmax_l, kk);
      }
    }
    key[k] = kk;
    r += qr; c += qc;
    if (c >= tw) { c -= tw; ++r; }
  }
  // one sample key per thread, spread over the rows of the region
  L.h2[t] = key[(t >> 4) & (PPT - 1)];
  const int n0 = block_sum(nloc, L.ired);
  const uint32_t kmin = block_min(kmin_l, L.ured);
  const uint32_t kmax = block_max(kmax_l, L.ured);

  double out_bkg = __builtin_nan(""), out_rms = __builtin_nan("");
  int out_n = 0;
  if (n0 > 0) {
    // ---- robust range from the sample's quartiles --------------------
    if (t < kWave) {
      uint32_t sv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) sv[i] = L.h2[t * 4 + i];
      // bitonic sort of 256 keys, 4 per lane (sentinels last)
#pragma unroll
      for (int kk = 2; kk <= 256; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
          if (j < 4) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int l = i ^ j;
              if (l > i) {
                const bool up = ((t * 4 + i) & kk) == 0;
                const uint32_t a = sv[i], b = sv[l];
                const bool sw = up ? (a > b) : (a < b);
                sv[i] = sw ? b : a;
                sv[l] = sw ? a : b;
              }
            }
          } else {
            const int lm = j / 4;
            const bool lower = (t & lm) == 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const bool up = ((t * 4 + i) & kk) == 0;
              const uint32_t o = __shfl_xor(sv[i], lm, kWave);
              const uint32_t mn = sv[i] < o ? sv[i] : o;
              const uint32_t mx = sv[i] < o ? o : sv[i];
              sv[i] = (lower == up) ? mn : mx;
            }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) L.list[t * 4 + i] = sv[i];
    }
    __syncthreads();
    Bins B;
    B.kmin = kmin;
    B.kmax = kmax;
    B.klo = kmin;
    B.khi = kmax;
    {
      int ns = 0;                          // valid samples: not sentinels
      int lo_b = 0, hi_b = kGather;
      while (lo_b < hi_b) {
        const int mid = (lo_b + hi_b) >> 1;
        if (L.list[mid] != kSentinel) lo_b = mid + 1; else hi_b = mid;
      }
      ns = lo_b;
      if (ns >= 16) {
        const double a = (double)key2f(L.list[ns / 4]);
        const double b = (double)key2f(L.list[(3 * ns) / 4]);
        const double iqr = b - a;
        if (iqr > 0.0) {
          const uint32_t klo = key_ceil(a - 4.0 * iqr);
          const uint32_t khi = key_floor(b + 4.0 * iqr);
          B.klo = klo > kmin ? klo : kmin;
          B.khi = khi < kmax ? khi : kmax;
          if (B.klo > B.khi) { B.klo = kmin; B.khi = kmax; }
        }
      }
    }
    {
      const uint32_t range = B.khi - B.klo;
      int sh = 0;
      while ((range >> sh) >= (uint32_t)(kBins - 2)) ++sh;
      B.sh = sh;
    }
    // ---- level-1 histogram ----------------------------------------
    for (int i = t; i < kBins; i += kBlock) L.h2[i] = 0;
    __syncthreads();
    int nlow = 0, nhigh = 0;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const uint32_t v = key[k];
      if (v == kSentinel) continue;
      const int b = bin_of(v, B);
      if (b == 0) ++nlow;
      else if (b == kBins - 1) ++nhigh;
      else atomicAdd(&L.h2[b], 1u);
    }
    nlow = wave_sum(nlow);
    nhigh = wave_sum(nhigh);
    if ((t & (kWave - 1)) == 0) {
      if (nlow) atomicAdd(&L.h2[0], (uint32_t)nlow);
      if (nhigh) atomicAdd(&L.h2[kBins - 1], (uint32_t)nhigh);
    }
    __syncthreads();
    {
      uint32_t loc[8];
      int s = 0;
#pragma unroll
      for (int i = 0; i < 8; ++i) { loc[i] = L.h2[t * 8 + i]; s += loc[i]; }
      int total;
      int ex = block_exclusive_scan(s, L.ired, &total);
#pragma unroll
      for (int i = 0; i < 8; ++i) { L.c1[t * 8 + i] = ex; ex += loc[i]; }
      if (t == kBlock - 1) L.c1[kBins] = ex;
      __syncthreads();
    }

    // ---- clipping loop on key intervals [klo, khi] of the region -----
    uint32_t klo = 0, khi = kSentinel - 1;
    int below = 0, nS = n0;
    double med = 0, mean = 0, sd = 0;
    bool have = false;
    for (int it = 0; it <= p.clip_iters; ++it) {
      // median (Eq. 1) of the current set: ranks below + (nS-1)/2, nS/2
      const int r0 = below + (nS - 1) / 2, r1 = below + nS / 2;
      uint32_t k0, k1;
      select_pair<PPT>(key, r0, r1, B, L, &k0, &k1);
      med = (r1 == r0) ? (double)key2f(k0)
                       : ((double)key2f(k0) + (double)key2f(k1)) / 2.0;
      // mean and population sigma, summed about the median
      double s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const uint32_t v = key[k];
        if (v != kSentinel && v >= klo && v <= khi) {
          const double d = (double)key2f(v) - med;
          s1 += d;
          s2 += d * d;
        }
      }
      block_sum2(s1, s2, L.dred);
      const double dm = s1 / (double)nS;
      mean = med + dm;
      const double var = s2 / (double)nS - dm * dm;
      sd = sqrt(var > 0.0 ? var : 0.0);
      have = true;
      if (it == p.clip_iters) break;
      // reject outside median +- k sigma
      const double lo = med - p.clip_sigma * sd;
      const double hi = med + p.clip_sigma * sd;
      uint32_t nlo = key_ceil(lo), nhi = key_floor(hi);
      nlo = nlo > klo ? nlo : klo;
      nhi = nhi < khi ? nhi : khi;
      int packed = 0;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const uint32_t v = key[k];
        if (v != kSentinel) {
          packed += (v < nlo) << 16;
          packed += (v >= nlo && v <= nhi);
        }
      }
      packed = block_sum(packed, L.ired);
      const int cb = packed >> 16, cin = packed & 0xFFFF;
      if (cin == nS) break;          // nothing rejected: data stabilised
      klo = nlo; khi = nhi; below = cb; nS = cin;
      have = false;
      if (nS == 0) break;
    }
    if (have && nS > 0) {
      out_n = nS;
      out_rms = sd;
      switch (p.estimator) {
        case IPP_EST_MEDIAN: out_bkg = med; break;
        case IPP_EST_MEAN: out_bkg = mean; break;
        case IPP_EST_MODE:
          out_bkg = p.median_factor * med - p.mean_factor * mean; break;
        default: out_bkg = 2.5 * med - 1.5 * mean; break;
      }
    }
  }
  if (t == 0) {
    wk.m_bkg[region] = out_bkg;
    wk.m_rms[region] = out_rms;
    wk.m_n[region] = out_n;
    if (fr.o_bkg_raw) fr.o_bkg_raw[local] = out_bkg;
    if (fr.o_rms_raw) fr.o_rms_raw[local] = out_rms;
    if (fr.o_n) fr.o_n[local] = out_n;
  }
}

// ---------------------------------------------------------------------
// k_mesh_stats_w: one wavefront per region for regions of at most 64 * PPL
// pixels (no workgroup barriers).  Same selection scheme as k_mesh_stats,
// with wave-level histograms of 16-bit counts (two per LDS word), ballot
// counts, and one fused pass per clipping step that counts the new set and
// sums its moments about a fixed shift c0 (the sample median).
namespace {

constexpr int kWBins = 2048;       // level-1 bins: 32 per lane
constexpr int kWSub = 1024;        // narrowing bins: 16 per lane
constexpr int kWGather = 256;

static_assert(kWBins == kBins, "wave bins share the block bin layout");

struct WaveLds {
  uint32_t h[kWBins / 2];
  uint32_t h2[kWSub / 2];
  uint32_t list[kWGather];
  uint32_t nlist;
  uint32_t sel[2];
};

__device__ __forceinline__ void wsync() {
  // wavefront scope: the wave's own LDS operations are performed in
  // order, so these order the code without waiting on memory
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// All ones if byte i of m is non-zero (a masked pixel), else 0.
__device__ __forceinline__ uint32_t byte_flag(uint32_t m, int i) {
  return (uint32_t)(-(int)((m >> (8 * i)) & 0xFFu) >> 31);
}

// Pixel value as held in registers: -0 folded onto +0, and the canonical
// quiet NaN for an excluded pixel (`bad` all ones) or a non-finite value.
constexpr uint32_t kNanBits = 0x7FC00000u;
constexpr uint32_t kBadKey = 0xFFC00000u;   // its key: above every finite key
__device__ __forceinline__ float pix_val(float v, uint32_t bad) {
  const uint32_t u = __float_as_uint(v + 0.0f);
  const uint32_t nf = (uint32_t)((int)(0x7F7FFFFFu - (u & 0x7FFFFFFFu)) >> 31);
  const uint32_t m = nf | bad;
  return __uint_as_float((m & kNanBits) | (~m & u));
}
__device__ __forceinline__ uint32_t pix_key(float v, uint32_t bad) {
  return f2key(pix_val(v, bad));
}

// Float bounds of a key interval [lo, hi] of pixel keys: v >= flo && v <= fhi
// holds exactly for the finite values whose key lies in [lo, hi] (no value
// is -0, so the key of -0 as an upper bound excludes +0).
__device__ __forceinline__ float key_lo_f(uint32_t lo) { return key2f(lo); }
__device__ __forceinline__ float key_hi_f(uint32_t hi) {
  return hi == 0x7FFFFFFFu ? -__uint_as_float(1u) : key2f(hi);
}

// Loads a th x tw region (row-major, four consecutive columns per group,
// PPL / 4 groups per lane) as keys.  Branch-free: rows and columns past the
// region re-read its last row or column and become sentinels.  VEC: the
// groups are 16-byte aligned float4s.  The scalar form converts every four
// groups before loading more, to bound the values in flight.
template <int PPL, bool VEC, bool MASK>
__device__ __forceinline__ void load_region(float (&key)[PPL],
                                            const float* base,
                                            const uint8_t* mbase,
                                            int64_t pitch, int th, int tw) {
  const int lane = lane_id();
  const int q4 = (tw + 3) >> 2;
  int r = lane / q4, c = lane - (lane / q4) * q4;
  const int dr = kWave / q4, dc = kWave - (kWave / q4) * q4;
#pragma unroll
  for (int k = 0; k < PPL / 4; ++k) {
    const int64_t o = (int64_t)min(r, th - 1) * pitch;
    const uint32_t out = (uint32_t)((th - 1 - r) >> 31);
    if (VEC) {
      const float4 v = *(const float4*)(base + o + 4 * c);
      uint32_t mk = 0;
      if (MASK) mk = *(const uint32_t*)(mbase + o + 4 * c);
      key[4 * k + 0] = pix_val(v.x, out | byte_flag(mk, 0));
      key[4 * k + 1] = pix_val(v.y, out | byte_flag(mk, 1));
      key[4 * k + 2] = pix_val(v.z, out | byte_flag(mk, 2));
      key[4 * k + 3] = pix_val(v.w, out | byte_flag(mk, 3));
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int cc = 4 * c + j;
        const int64_t oj = o + min(cc, tw - 1);
        uint32_t mk = 0;
        if (MASK) mk = mbase[oj];
        key[4 * k + j] = pix_val(base[oj], out | byte_flag(mk, 0) |
                                               (uint32_t)((tw - 1 - cc) >> 31));
      }
      if ((k & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    r += dr; c += dc;
    if (c >= q4) { c -= q4; ++r; }
  }
}

// An opaque copy of a key: stops the compiler from reusing per-pixel
// values of an earlier pass (which would keep a second PPL registers alive).
__device__ __forceinline__ uint32_t fresh(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}
__device__ __forceinline__ float fresh(float v) {
  asm volatile("" : "+v"(v));
  return v;
}

__device__ __forceinline__ uint32_t count16(const uint32_t* h, int b) {
  return (h[b >> 1] >> ((b & 1) << 4)) & 0xFFFFu;
}

__device__ __forceinline__ int wave_incl_scan(int x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int u = __shfl_up(x, o, kWave);
    if (lane >= o) x += u;
  }
  return x;
}

__device__ __forceinline__ int rl(int v, int lane) {
  return __builtin_amdgcn_readlane(v, lane);
}

// Wave-uniform copies (SGPR) of values every lane already agrees on.
__device__ __forceinline__ int uni(int v) {
  return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ uint32_t uni(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ double uni(double v) {
  const uint64_t u = __double_as_longlong(v);
  const uint32_t lo = uni((uint32_t)u), hi = uni((uint32_t)(u >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Exclusive prefix (over lanes) of the totals of the BPL consecutive
// 16-bit bins each lane owns.
template <int BPL>
__device__ __forceinline__ int lane_base_of(const uint32_t* h) {
  const int lane = lane_id();
  int s = 0;
#pragma unroll
  for (int i = 0; i < BPL / 2; ++i) {
    const uint32_t w = h[lane * (BPL / 2) + i];
    s += (int)(w & 0xFFFFu) + (int)(w >> 16);
  }
  return wave_incl_scan(s) - s;
}

// Bin of a 64*BPL-bin histogram holding rank rr; *before = keys in lower
// bins, *cnt = keys in the bin.
template <int BPL>
__device__ __forceinline__ int wave_find(const uint32_t* h, int base, int rr,
                                         int* before, int* cnt) {
  const int lane = lane_id();
  const uint64_t m = __ballot(base <= rr);
  const int L = 63 - __builtin_clzll(m);
  const int c = lane < BPL ? (int)count16(h, L * BPL + lane) : 0;
  const int incl = wave_incl_scan(c);
  const int r = rr - rl(base, L);
  const uint64_t m2 = __ballot(lane < BPL && incl > r);
  const int j = __builtin_ctzll(m2);
  *before = rl(base, L) + rl(incl - c, j);
  *cnt = rl(c, j);
  return L * BPL + j;
}

// Keys of [lo, hi] (cnt of them, cnt <= kWGather) gathered into LDS; the
// keys of within-range ranks w0 and w1 are returned.
template <int PPL>
__device__ __forceinline__ void wave_gather_select(
    const float (&val)[PPL], uint32_t lo, uint32_t hi, int cnt, int w0,
    int w1, WaveLds& L, uint32_t* k0, uint32_t* k1) {
  const int lane = lane_id();
  const float flo = key_lo_f(lo), fhi = key_hi_f(hi);
  if (lane == 0) L.nlist = 0;
  wsync();
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const float v = val[k];
    if (v >= flo && v <= fhi) {
      const uint32_t slot = atomicAdd(&L.nlist, 1u);
      if (slot < (uint32_t)kWGather) L.list[slot] = f2key(fresh(v));
    }
  }
  wsync();
  for (int i = lane; i < cnt; i += kWave) {
    const uint32_t me = L.list[i];
    int less = 0;
    for (int q = 0; q < cnt; ++q) {
      const uint32_t o = L.list[q];
      less += (o < me) || (o == me && q < i);
    }
    if (less == w0) L.sel[0] = me;
    if (less == w1) L.sel[1] = me;
  }
  wsync();
  *k0 = uni(L.sel[0]);
  *k1 = uni(L.sel[1]);
  wsync();
}

// Key of rank r inside level-1 bin [lo, hi] (base keys below it, cnt in
// it), narrowing with 1024-bin histograms until a gather suffices.
template <int PPL>
__device__ __forceinline__ uint32_t wave_narrow(const float (&key)[PPL],
                                                int r, uint32_t lo,
                                                uint32_t hi, int base, int cnt,
                                                WaveLds& L) {
  const int lane = lane_id();
  for (int level = 0; level < 6; ++level) {
    if (lo == hi) return lo;
    if (cnt <= kWGather) {
      uint32_t a, b;
      wave_gather_select<PPL>(key, lo, hi, cnt, r - base, r - base, L, &a,
                              &b);
      return a;
    }
    const uint32_t range = (uint32_t)(hi - lo);
    const int bits = 32 - __clz(range);
    const int sh = bits > 10 ? bits - 10 : 0;
#pragma unroll
    for (int i = 0; i < kWSub / 2 / kWave; ++i) L.h2[lane + i * kWave] = 0;
    wsync();
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const uint32_t v = f2key(fresh(key[k]));
      const bool in = v >= lo && v <= hi;
      const uint32_t b = in ? (v - lo) >> sh : 0u;
      atomicAdd(&L.h2[b >> 1], (uint32_t)in << ((b & 1) << 4));
    }
    wsync();
    const int sbase = lane_base_of<kWSub / kWave>(L.h2);
    int pre, c;
    const int b = wave_find<kWSub / kWave>(L.h2, sbase, r - base, &pre, &c);
    wsync();
    const uint64_t nlo = (uint64_t)lo + ((uint64_t)b << sh);
    const uint64_t nhi = nlo + ((1ull << sh) - 1);
    lo = (uint32_t)nlo;
    hi = nhi < hi ? (uint32_t)nhi : hi;
    base += pre;
    cnt = c;
  }
  return lo;  // not reached: 32 key bits are exhausted by then
}

}  // namespace

template <int PPL>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(PPL == 64 ? 4 : 6))) void k_mesh_stats_w(Work wk,
                                                         ipp_params p) {
  __shared__ WaveLds Lall[kWaves];
  const int lane = lane_id();
  // wave index made provably uniform: geometry then lives in SGPRs
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int region = blockIdx.x * kWaves + wv;
  if (region >= wk.total_nodes) return;        // whole wavefront leaves
  WaveLds& L = Lall[wv];
  const int f = find_frame(wk.frames, wk.nframes, region, &FrameDev::node0);
  const FrameDev fr = wk.frames[f];
  const int local = region - fr.node0;
  const int rj = local / fr.nx, ri = local - rj * fr.nx;
  const int y0 = rj * p.mesh_h, x0 = ri * p.mesh_w;
  const int th = min(p.mesh_h, fr.h - y0), tw = min(p.mesh_w, fr.w - x0);
  const int P = th * tw;

  // ---- load the region as keys (sentinel: excluded pixel) ------------
  // Branch-free: rows past the region re-read its last row and are turned
  // into sentinels arithmetically, so no per-element lane masks stay live.
  float key[PPL];
  const float* base = fr.pix + (int64_t)y0 * fr.pitch + x0;
  const uint8_t* mbase = fr.mask ? fr.mask + (int64_t)y0 * fr.pitch + x0
                                 : nullptr;
  const bool vec4 = (tw & 3) == 0 && (fr.pitch & 3) == 0 && (x0 & 3) == 0 &&
                    ((uintptr_t)fr.pix & 15) == 0 &&
                    (!fr.mask || ((uintptr_t)fr.mask & 3) == 0);
  if (vec4) {
    if (mbase) load_region<PPL, true, true>(key, base, mbase, fr.pitch, th, tw);
    else load_region<PPL, true, false>(key, base, mbase, fr.pitch, th, tw);
  } else {
    if (mbase) load_region<PPL, false, true>(key, base, mbase, fr.pitch, th, tw);
    else load_region<PPL, false, false>(key, base, mbase, fr.pitch, th, tw);
  }
  // one sample pixel per lane, spread over the rows and columns
  uint32_t smp;
  {
    const int r = (lane * th) >> 6, c = (lane * 37 + 11) % tw;
    const int64_t o = (int64_t)r * fr.pitch + c;
    smp = pix_key(base[o], mbase ? byte_flag(mbase[o], 0) : 0u);
  }
  double out_bkg = __builtin_nan(""), out_rms = __builtin_nan("");
  int out_n = 0;
  {
    // ---- sample quartiles: histogram range and moment shift ----------
#pragma unroll
    for (int kk = 2; kk <= kWave; kk <<= 1) {
#pragma unroll
      for (int j = kk >> 1; j > 0; j >>= 1) {
        const uint32_t o = __shfl_xor(smp, j, kWave);
        const bool up = (lane & kk) == 0;
        const bool lower = (lane & j) == 0;
        const uint32_t mn = smp < o ? smp : o;
        const uint32_t mx = smp < o ? o : smp;
        smp = (lower == up) ? mn : mx;
      }
    }
    const int ns = __popcll(__ballot(smp < kBadKey));
    // end bins reach over every finite key
    Bins B;
    B.kmin = 0;
    B.kmax = kBadKey - 1;
    B.klo = 0;
    B.khi = kBadKey - 1;
    float c0f = 0.0f;
    if (ns > 0) {
      c0f = key2f((uint32_t)rl((int)smp, ns / 2));
      B.klo = (uint32_t)rl((int)smp, 0);
      B.khi = (uint32_t)rl((int)smp, ns - 1);
    }
    if (ns >= 16) {
      const double a = (double)key2f((uint32_t)rl((int)smp, ns / 4));
      const double b = (double)key2f((uint32_t)rl((int)smp, (3 * ns) / 4));
      const double iqr = b - a;
      if (iqr > 0.0) {
        B.klo = key_ceil(a - 4.0 * iqr);
        B.khi = key_floor(b + 4.0 * iqr);
        if (B.khi >= kBadKey) B.khi = kBadKey - 1;
        if (B.klo > B.khi) B.klo = B.khi;
      }
    }
    {
      const uint32_t range = B.khi - B.klo;
      int sh = 0;
      while ((range >> sh) >= (uint32_t)(kWBins - 2)) ++sh;
      B.sh = sh;
    }
    const double c0 = (double)c0f;

    // ---- level-1 histogram, and the moments of the full set ---------
#pragma unroll
    for (int i = 0; i < kWBins / 2 / kWave; ++i) L.h[lane + i * kWave] = 0;
    wsync();
    double s1 = 0.0, s2 = 0.0;
    int n0 = 0;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      // branch-free: excluded pixels land in the top bin and are taken out
      // below
      const float fv = fresh(key[k]);
      const uint32_t v = f2key(fv);
      uint32_t b = 1 + ((v - B.klo) >> B.sh);
      b = v > B.khi ? kWBins - 1 : b;
      b = v < B.klo ? 0 : b;
      atomicAdd(&L.h[b >> 1], 1u << ((b & 1) << 4));
      const bool ok = fv == fv;
      n0 += __popcll(__builtin_amdgcn_ballot_w64(ok));
      const double d = (double)(ok ? fv : c0f) - c0;
      s1 += d;
      s2 = fma(d, d, s2);
    }
    n0 = uni(n0);
    s1 = uni(wave_sum(s1));
    s2 = uni(wave_sum(s2));
    wsync();
    if (lane == 0)
      atomicSub(&L.h[kWBins / 2 - 1], (uint32_t)(kWave * PPL - n0) << 16);
    wsync();
    const int lbase = lane_base_of<kWBins / kWave>(L.h);

    auto select = [&](int r0, int r1, uint32_t* k0, uint32_t* k1) {
      int pre0, c0n, pre1, c1n;
      const int j0 = wave_find<kWBins / kWave>(L.h, lbase, r0, &pre0, &c0n);
      int j1 = j0;
      pre1 = pre0;
      c1n = c0n;
      if (r1 != r0 && r1 >= pre0 + c0n)
        j1 = wave_find<kWBins / kWave>(L.h, lbase, r1, &pre1, &c1n);
      const int cnt = pre1 + c1n - pre0;
      uint64_t lo0w, hi0w, lo1w, hi1w;          // all within [kmin, kmax]
      bin_range(j0, B, &lo0w, &hi0w);           // kWBins == kBins
      bin_range(j1, B, &lo1w, &hi1w);
      const uint32_t lo0 = (uint32_t)lo0w, hi0 = (uint32_t)hi0w;
      const uint32_t lo1 = (uint32_t)lo1w, hi1 = (uint32_t)hi1w;
      if (cnt <= kWGather) {
        wave_gather_select<PPL>(key, lo0, hi1, cnt, r0 - pre0, r1 - pre0, L,
                                k0, k1);
      } else {
        *k0 = wave_narrow<PPL>(key, r0, lo0, hi0, pre0, c0n, L);
        *k1 = r1 == r0 ? *k0
                       : wave_narrow<PPL>(key, r1, lo1, hi1, pre1, c1n, L);
      }
    };

    // ---- clipping loop on key intervals [klo, khi] -------------------
    uint32_t klo = 0, khi = kSentinel - 1;
    int below = 0, nS = n0;
    double med = 0, mean = 0, sd = 0;
    bool have = false;
    // float bounds of the current set (every finite value at the start)
    float pflo = -__builtin_inff(), pfhi = __builtin_inff();
    for (int it = 0; n0 > 0 && it <= p.clip_iters; ++it) {
      const int r0 = below + (nS - 1) / 2, r1 = below + nS / 2;
      uint32_t k0, k1;
      select(r0, r1, &k0, &k1);
      med = (r1 == r0) ? (double)key2f(k0)
                       : ((double)key2f(k0) + (double)key2f(k1)) / 2.0;
      const double dm = s1 / (double)nS;
      mean = c0 + dm;
      const double var = s2 / (double)nS - dm * dm;
      sd = sqrt(var > 0.0 ? var : 0.0);
      have = true;
      if (it == p.clip_iters) break;
      const double lo = med - p.clip_sigma * sd;
      const double hi = med + p.clip_sigma * sd;
      uint32_t nlo = key_ceil(lo), nhi = key_floor(hi);
      nlo = nlo > klo ? nlo : klo;
      nhi = nhi < khi ? nhi : khi;
      // float bounds of the key interval (a NaN value fails both tests)
      const float flo = key_lo_f(nlo), fhi = key_hi_f(nhi);
      // The new set is the current one less its values outside
      // [flo, fhi]: only those are visited (a register whose pixels all
      // stay is skipped by the whole wave) and their moments subtracted.
      int nrem = 0, nremlo = 0;
      double q1 = 0.0, q2 = 0.0;
#pragma unroll
      for (int k = 0; k < PPL; ++k) {
        const float v = fresh(key[k]);
        const bool was = v >= pflo && v <= pfhi;
        const bool lo_ = v < flo;
        const uint64_t gm = __builtin_amdgcn_ballot_w64(was & (lo_ | (v > fhi)));
        if (gm) {
          nrem += __popcll(gm);
          nremlo += __popcll(__builtin_amdgcn_ballot_w64(was & lo_));
          const bool gone = (gm >> lane) & 1ull;
          const double d = gone ? (double)v - c0 : 0.0;
          q1 += d;
          q2 = fma(d, d, q2);
        }
      }
      // summed before the exit test, so that the per-pixel terms are not
      // deferred past it and kept alive
      const int cin = nS - uni(nrem);
      const int cb = below + uni(nremlo);
      q1 = uni(wave_sum(q1));
      q2 = uni(wave_sum(q2));
      if (cin == nS) break;          // nothing rejected: data stabilised
      double t1 = s1 - q1, t2 = s2 - q2;
      if (q2 > 16384.0 * t2) {
        // the removed values dominated the sums: the survivors' moments
        // are summed afresh, so that no cancellation reaches them
        t1 = 0.0;
        t2 = 0.0;
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
          const float v = fresh(key[k]);
          const bool in = v >= flo && v <= fhi;
          const double d = (double)(in ? v : c0f) - c0;
          t1 += d;
          t2 = fma(d, d, t2);
        }
        t1 = uni(wave_sum(t1));
        t2 = uni(wave_sum(t2));
      }
      pflo = flo;
      pfhi = fhi;
      klo = nlo; khi = nhi; below = cb; nS = cin;
      s1 = t1;
      s2 = t2;
      have = false;
      if (nS == 0) break;
    }
    if (have && nS > 0) {
      out_n = nS;
      out_rms = sd;
      switch (p.estimator) {
        case IPP_EST_MEDIAN: out_bkg = med; break;
        case IPP_EST_MEAN: out_bkg = mean; break;
        case IPP_EST_MODE:
          out_bkg = p.median_factor * med - p.mean_factor * mean; break;
        default: out_bkg = 2.5 * med - 1.5 * mean; break;
      }
    }
  }
  if (lane == 0) {
    wk.m_bkg[region] = out_bkg;
    wk.m_rms[region] = out_rms;
    wk.m_n[region] = out_n;
    if (fr.o_bkg_raw) fr.o_bkg_raw[local] = out_bkg;
    if (fr.o_rms_raw) fr.o_rms_raw[local] = out_rms;
    if (fr.o_n) fr.o_n[local] = out_n;
  }
}

// ---------------------------------------------------------------------
// Per-frame finish: fill invalid nodes, median filter, spline tables.
// ---------------------------------------------------------------------
namespace {

// Median (Eq. 1) of the valid entries of a window held in registers: the
// order statistics of rank (n-1)/2 and n/2 found by rank counting, fully
// unrolled so nothing is indexed dynamically.
template <int MAXN>
__device__ __forceinline__ double median_window(const double (&v)[MAXN],
                                                uint64_t valid, int n) {
  const int k1 = (n - 1) / 2, k2 = n / 2;
  double m1 = 0.0, m2 = 0.0;
#pragma unroll
  for (int i = 0; i < MAXN; ++i) {
    if (!((valid >> i) & 1ull)) continue;
    int lt = 0, le = 0;
#pragma unroll
    for (int j = 0; j < MAXN; ++j) {
      if ((valid >> j) & 1ull) {
        lt += v[j] < v[i];
        le += v[j] <= v[i];
      }
    }
    if (lt <= k1 && k1 < le) m1 = v[i];
    if (lt <= k2 && k2 < le) m2 = v[i];
  }
  return (n & 1) ? m1 : (m1 + m2) / 2.0;
}

// Second derivatives of the natural cubic spline along one mesh line:
// values f[base + k*stride], k < n, on node_coord(k, m, len); Thomas
// algorithm with scratch cp/dp at the same strided positions.  The loads
// of each sweep are issued in chunks ahead of the dependent recurrence.
__device__ void natural_line(const double* f, double* M, double* cp,
                             double* dp, int base, int stride, int n, int m,
                             int len) {
  constexpr int CH = 8;
  M[base] = 0.0;
  M[base + (n - 1) * stride] = 0.0;
  if (n < 3) {
    for (int k = 0; k < n; ++k) M[base + k * stride] = 0.0;
    return;
  }
  double cprev = 0.0, dprev = 0.0;
  for (int i0 = 1; i0 <= n - 2; i0 += CH) {
    double fl[CH + 2];
#pragma unroll
    for (int u = 0; u < CH + 2; ++u) {
      const int i = i0 - 1 + u;
      fl[u] = i < n ? f[base + i * stride] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = i0 + u;
      if (i > n - 2) break;
      const double t0 = node_coord(i - 1, m, len), t1 = node_coord(i, m, len);
      const double t2 = node_coord(i + 1, m, len);
      const double h0 = t1 - t0, h1 = t2 - t1;
      const double a = (i > 1) ? h0 : 0.0;
      const double b = 2.0 * (h0 + h1);
      const double d = 6.0 * ((fl[u + 2] - fl[u + 1]) / h1 -
                              (fl[u + 1] - fl[u]) / h0);
      const double den = b - a * cprev;
      cprev = h1 / den;
      dprev = (d - a * dprev) / den;
      cp[base + i * stride] = cprev;
      dp[base + i * stride] = dprev;
    }
  }
  double nxt = dprev;                          // M[n-2]
  M[base + (n - 2) * stride] = nxt;
  for (int i1 = n - 3; i1 >= 1; i1 -= CH) {
    double dl[CH], cl[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = i1 - u;
      dl[u] = i >= 1 ? dp[base + i * stride] : 0.0;
      cl[u] = i >= 1 ? cp[base + i * stride] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = i1 - u;
      if (i < 1) break;
      nxt = dl[u] - cl[u] * nxt;
      M[base + i * stride] = nxt;
    }
  }
}

}  // namespace

// Invalid-node fill (one workgroup per frame).
__global__ __launch_bounds__(kBlock) void k_mesh_fill(Work wk, ipp_params p) {
  __shared__ int ired[kWaves];
  const int f = blockIdx.x;
  const FrameDev fr = wk.frames[f];
  const int ny = fr.ny, nx = fr.nx, N = ny * nx, b0 = fr.node0;
  uint32_t flags = 0;

  // validity and fallbacks
  int nv = 0, n1 = 0;
  for (int i = threadIdx.x; i < N; i += kBlock) {
    nv += wk.m_n[b0 + i] >= p.min_valid;
    n1 += wk.m_n[b0 + i] >= 1;
  }
  nv = block_sum(nv, ired);
  n1 = block_sum(n1, ired);
  int thr = p.min_valid;
  if (nv == 0) { flags |= IPP_FRAME_NO_VALID_MESH; thr = 1; }
  const bool empty = (n1 == 0);
  if (empty) flags |= IPP_FRAME_EMPTY_MESH;

  for (int i = threadIdx.x; i < N; i += kBlock) {
    const bool known = !empty && wk.m_n[b0 + i] >= thr;
    wk.f_pass[b0 + i] = known ? 0 : (empty ? 0 : -1);
    wk.f_bkg[b0 + i] = known ? wk.m_bkg[b0 + i] : 0.0;
    wk.f_rms[b0 + i] = known ? wk.m_rms[b0 + i] : 0.0;
  }
  __syncthreads();
  // Jacobi fill passes: a node unknown before pass q takes the mean of its
  // neighbours known before pass q (summed in raster order)
  for (int pass = 1; pass <= N; ++pass) {
    int todo = 0;
    for (int i = threadIdx.x; i < N; i += kBlock) {
      if (wk.f_pass[b0 + i] >= 0) continue;
      const int j = i / nx, ii = i - j * nx;
      double sb = 0.0, sr = 0.0;
      int cnt = 0;
      for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
          const int jj = j + dj, i2 = ii + di;
          if ((dj | di) == 0 || jj < 0 || jj >= ny || i2 < 0 || i2 >= nx)
            continue;
          const int q = b0 + jj * nx + i2;
          const int kp = wk.f_pass[q];
          if (kp >= 0 && kp < pass) {
            sb += wk.f_bkg[q];
            sr += wk.f_rms[q];
            ++cnt;
          }
        }
      if (cnt) {
        wk.f_bkg[b0 + i] = sb / cnt;
        wk.f_rms[b0 + i] = sr / cnt;
        wk.f_pass[b0 + i] = pass;
      } else {
        todo = 1;
      }
    }
    todo = block_sum(todo, ired);
    __syncthreads();
    if (todo == 0) break;
  }
  if (threadIdx.x == 0 && wk.frame_flags) wk.frame_flags[f] = flags;
}

// Median filter (window (2F+1)^2 at most), one thread per node of the batch.
template <int F>
__global__ __launch_bounds__(kBlock) void k_mesh_filter(Work wk,
                                                        ipp_params p) {
  constexpr int S = 2 * F + 1, MAXN = S * S;
  const int node = blockIdx.x * kBlock + threadIdx.x;
  if (node >= wk.total_nodes) return;
  const int f = find_frame(wk.frames, wk.nframes, node, &FrameDev::node0);
  const FrameDev& fr = wk.frames[f];
  const int nx = fr.nx, ny = fr.ny, b0 = fr.node0, i = node - b0;
  const int fh = p.filter_h / 2, fw = p.filter_w / 2;
  const int j = i / nx, ii = i - j * nx;
  double vb[MAXN], vr[MAXN];
  uint64_t valid = 0;
  int n = 0;
#pragma unroll
  for (int dj = -F; dj <= F; ++dj)
#pragma unroll
    for (int di = -F; di <= F; ++di) {
      const int k = (dj + F) * S + (di + F);
      const int jj = j + dj, i2 = ii + di;
      const bool ok = dj >= -fh && dj <= fh && di >= -fw && di <= fw &&
                      jj >= 0 && jj < ny && i2 >= 0 && i2 < nx;
      vb[k] = ok ? wk.f_bkg[b0 + jj * nx + i2] : 0.0;
      vr[k] = ok ? wk.f_rms[b0 + jj * nx + i2] : 0.0;
      if (ok) { valid |= 1ull << k; ++n; }
    }
  const double mb = median_window<MAXN>(vb, valid, n);
  const double mr = median_window<MAXN>(vr, valid, n);
  wk.tb[0][node] = mb;
  wk.tr[0][node] = mr;
  if (fr.o_bkg) fr.o_bkg[i] = mb;
  if (fr.o_rms) fr.o_rms[i] = mr;
}

// Natural-spline second derivatives, one thread per mesh line.  Pass 0:
// fxx along every row and fyy along every column, of both meshes; pass 1:
// fxxyy along every column of fxx, of both meshes.  Lines of frame f start
// at fr.line0[pass]; per frame pass 0 has 2(ny + nx) lines, pass 1 2 nx.
template <int PASS>
__global__ __launch_bounds__(64) void k_mesh_spline(Work wk, ipp_params p) {
  const int line = blockIdx.x * 64 + threadIdx.x;
  if (line >= wk.total_lines[PASS]) return;
  int lo = 0, hi = wk.nframes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (wk.frames[mid].line0[PASS] <= line) lo = mid; else hi = mid - 1;
  }
  const FrameDev& fr = wk.frames[lo];
  const int l = line - fr.line0[PASS];
  const int ny = fr.ny, nx = fr.nx, b0 = fr.node0;
  const size_t T = (size_t)wk.total_nodes;
  if (PASS == 0) {
    if (l < 2 * ny) {                 // rows: fxx
      const int j = l % ny, m = l / ny;
      natural_line(m ? wk.tr[0] : wk.tb[0], m ? wk.tr[1] : wk.tb[1],
                   wk.sc0 + m * T, wk.sc1 + m * T, b0 + j * nx, 1, nx,
                   p.mesh_w, fr.w);
    } else {                          // columns: fyy
      const int c = l - 2 * ny, i = c % nx, m = c / nx;
      natural_line(m ? wk.tr[0] : wk.tb[0], m ? wk.tr[2] : wk.tb[2],
                   wk.sc0 + (2 + m) * T, wk.sc1 + (2 + m) * T, b0 + i, nx,
                   ny, p.mesh_h, fr.h);
    }
  } else {                            // columns of fxx: fxxyy
    const int i = l % nx, m = l / nx;
    natural_line(m ? wk.tr[1] : wk.tb[1], m ? wk.tr[3] : wk.tb[3],
                 wk.sc0 + m * T, wk.sc1 + m * T, b0 + i, nx, ny, p.mesh_h,
                 fr.h);
  }
}

template __global__ void k_mesh_filter<1>(Work, ipp_params);
template __global__ void k_mesh_filter<2>(Work, ipp_params);
template __global__ void k_mesh_filter<3>(Work, ipp_params);
template __global__ void k_mesh_spline<0>(Work, ipp_params);
template __global__ void k_mesh_spline<1>(Work, ipp_params);
template __global__ void k_mesh_stats_w<16>(Work, ipp_params);
template __global__ void k_mesh_stats_w<64>(Work, ipp_params);
template __global__ void k_mesh_stats<64>(Work, ipp_params);

}  // namespace ipp
