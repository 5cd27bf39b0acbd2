// Background mesh: sigma-clipped statistics of every region (Sec. 2.2.2,
// Eq. 1-4 and the clipping loop), then invalid-node fill, median filter and
// natural-spline tables per frame.
//
// k_mesh_stats: one 256-thread workgroup per region.  The region's pixels
// stay in registers as order-preserving uint32 keys of their float32 values.
// Every set the clipping loop visits is a key interval of the region's
// finite, unmasked pixels, so each median is an order statistic of that one
// multiset: a 2048-bin histogram over its key range is built once, and each
// query narrows one bin with a second histogram and an exact rank count over
// the few remaining keys.  Means and deviations are binary64 block sums in a
// fixed order.
#include "ipp_internal.h"
#include "kernels.h"

namespace ipp {

namespace {

constexpr int kBins = 2048;
constexpr int kGather = 256;

struct MeshLds {
  uint32_t c1[kBins + 1];     // level-1 exclusive prefix counts
  uint32_t h2[kBins];         // per-query histogram
  uint32_t list[kGather];     // gathered keys of one bin
  uint32_t sel[4];            // query results
  uint32_t ured[kWaves];
  int ired[kWaves];
  double dred[kWaves];
};

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

// Key of rank `rank` among the included keys.  Level-1 prefix counts in
// L.c1 over [kmin, kmin + bins << sh1).
template <int PPT>
__device__ uint32_t select_rank(const uint32_t (&key)[PPT], int rank,
                                uint32_t kmin, uint32_t kmax, int sh1,
                                MeshLds& L) {
  // level 1: binary search of the prefix array (every thread, broadcast)
  int lo_b = 0, hi_b = kBins - 1;
  while (lo_b < hi_b) {
    int mid = (lo_b + hi_b + 1) >> 1;
    if ((int)L.c1[mid] <= rank) lo_b = mid; else hi_b = mid - 1;
  }
  uint64_t lo = (uint64_t)kmin + ((uint64_t)lo_b << sh1);
  uint64_t hi = lo + ((1ull << sh1) - 1);
  if (hi > kmax) hi = kmax;
  int base = (int)L.c1[lo_b];
  int cnt = (int)(L.c1[lo_b + 1] - L.c1[lo_b]);
  for (int level = 0; level < 4; ++level) {
    if (lo == hi) return (uint32_t)lo;
    if (cnt <= kGather) {
      // gather the keys of [lo, hi] and rank them exactly
      __syncthreads();
      if (threadIdx.x == 0) L.sel[3] = 0;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        uint32_t v = key[k];
        if (v != kSentinel && v >= lo && v <= hi) {
          uint32_t slot = atomicAdd(&L.sel[3], 1u);
          L.list[slot] = v;
        }
      }
      __syncthreads();
      const int want = rank - base;
      if ((int)threadIdx.x < cnt) {
        const uint32_t me = L.list[threadIdx.x];
        int less = 0;
        for (int i = 0; i < cnt; ++i) {
          uint32_t o = L.list[i];
          less += (o < me) || (o == me && i < (int)threadIdx.x);
        }
        if (less == want) L.sel[0] = me;
      }
      __syncthreads();
      uint32_t res = L.sel[0];
      __syncthreads();
      return res;
    }
    // narrow with a second histogram over [lo, hi]
    uint32_t range = (uint32_t)(hi - lo);
    int bits = 32 - __clz(range);
    int sh = bits > 11 ? bits - 11 : 0;
    for (int i = threadIdx.x; i < kBins; i += kBlock) L.h2[i] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      uint32_t v = key[k];
      if (v != kSentinel && v >= lo && v <= hi)
        atomicAdd(&L.h2[(uint32_t)(v - lo) >> sh], 1u);
    }
    __syncthreads();
    find_rank_bin(L.h2, rank - base, L.sel, L.ired);
    uint32_t b = L.sel[0];
    int pre = (int)L.sel[1];
    cnt = (int)L.sel[2];
    __syncthreads();
    lo = lo + ((uint64_t)b << sh);
    uint64_t nhi = lo + ((1ull << sh) - 1);
    hi = nhi < hi ? nhi : hi;
    base += pre;
  }
  return (uint32_t)lo;  // not reached: the key range is exhausted by then
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
  return k;
}

}  // namespace

template <int PPT>
__global__ __launch_bounds__(kBlock) void k_mesh_stats(Work wk,
                                                       ipp_params p) {
  __shared__ MeshLds L;
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
  int r = threadIdx.x / tw, c = threadIdx.x - (threadIdx.x / tw) * tw;
  const int qr = kBlock / tw, qc = kBlock - (kBlock / tw) * tw;
  int nloc = 0;
  uint32_t kmin_l = kSentinel, kmax_l = 0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    uint32_t kk = kSentinel;
    if (k * kBlock + (int)threadIdx.x < P) {
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
  const int n0 = block_sum(nloc, L.ired);
  const uint32_t kmin = block_min(kmin_l, L.ured);
  const uint32_t kmax = block_max(kmax_l, L.ured);

  double out_bkg = __builtin_nan(""), out_rms = __builtin_nan("");
  int out_n = 0;
  if (n0 > 0) {
    // ---- level-1 histogram over [kmin, kmax] ------------------------
    const uint32_t range = kmax - kmin;
    const int bits = 32 - __clz(range);
    const int sh1 = bits > 11 ? bits - 11 : 0;
    for (int i = threadIdx.x; i < kBins; i += kBlock) L.h2[i] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PPT; ++k)
      if (key[k] != kSentinel) atomicAdd(&L.h2[(key[k] - kmin) >> sh1], 1u);
    __syncthreads();
    {
      const int t = threadIdx.x;
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
      // statistics of the current set
      const int r0 = below + (nS - 1) / 2;
      uint32_t k0 = select_rank<PPT>(key, r0, kmin, kmax, sh1, L);
      double m0 = (double)key2f(k0);
      if ((nS & 1) == 0) {
        // next order statistic: k0 again if duplicated, else the next key
        int le = 0;
        uint32_t nx_l = kSentinel;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
          uint32_t v = key[k];
          if (v != kSentinel) {
            le += (v <= k0);
            if (v > k0) nx_l = min(nx_l, v);
          }
        }
        le = block_sum(le, L.ired);
        uint32_t nx = block_min(nx_l, L.ured);
        uint32_t k1 = (le > r0 + 1) ? k0 : nx;
        m0 = (m0 + (double)key2f(k1)) / 2.0;
      }
      med = m0;
      double s1 = 0.0;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        uint32_t v = key[k];
        if (v != kSentinel && v >= klo && v <= khi) s1 += (double)key2f(v);
      }
      s1 = block_sum(s1, L.dred);
      mean = s1 / (double)nS;
      double s2 = 0.0;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        uint32_t v = key[k];
        if (v != kSentinel && v >= klo && v <= khi) {
          double d = (double)key2f(v) - mean;
          s2 += d * d;
        }
      }
      s2 = block_sum(s2, L.dred);
      sd = sqrt(s2 / (double)nS);
      have = true;
      if (it == p.clip_iters) break;
      // reject outside median +- k sigma
      const double lo = med - p.clip_sigma * sd;
      const double hi = med + p.clip_sigma * sd;
      uint32_t nlo = key_ceil(lo), nhi = key_floor(hi);
      nlo = nlo > klo ? nlo : klo;
      nhi = nhi < khi ? nhi : khi;
      int cb = 0, cin = 0;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        uint32_t v = key[k];
        if (v != kSentinel) {
          cb += (v < nlo);
          cin += (v >= nlo && v <= nhi);
        }
      }
      cb = block_sum(cb, L.ired);
      cin = block_sum(cin, L.ired);
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
  if (threadIdx.x == 0) {
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
template __global__ void k_mesh_stats<4>(Work, ipp_params);
template __global__ void k_mesh_stats<16>(Work, ipp_params);
template __global__ void k_mesh_stats<64>(Work, ipp_params);

}  // namespace ipp
