// Detection (Sec. 2.2.5): background removal and threshold, connection of
// detected pixels into candidates, and candidate pre-analysis.
//
// Labelling is two-level.  k_tile_ccl labels each TH x TW tile in LDS with
// a lock-free union-find (union by minimum index, so a tile component's
// root is its first pixel in raster order) and emits one record per tile
// component that touches an inner tile border or is already large enough
// to keep.  k_border joins records across tile borders with the same
// union-find on records in global memory, k_resolve folds every record
// into its root, and the kept candidates are numbered 1..K in raster order
// of their first pixel through per-row counts, a scan and a within-row
// rank.  k_relabel writes the final label map; k_source_stats measures
// each candidate with exact integer sums (one wavefront per candidate).
#include "ipp_internal.h"
#include "kernels.h"
#include "spline_tile.h"

namespace ipp {

namespace {

template <int TH, int TW, bool CONN8>
struct CclLds {
  static constexpr int NP = TH * TW;
  static constexpr int NSEG = NP / 64;         // 64-pixel segments
  static constexpr int NRUN = NP / 2;          // runs: at most every other pixel
  static constexpr int NCMP = CONN8 ? NP / 4 : NP / 2;
  union {
    SplineLds<TH, TW> spl;                     // until the threshold is taken
    struct {
      int parent[NRUN];        // union-find over runs; after numbering a
                               // root holds -2 - (its component id)
      uint16_t rq[NRUN];       // head pixel of each run
      int npix[NCMP];
      int xmin[NCMP];
      int xmax[NCMP];
      int ymax[NCMP];
      int16_t rootp[NCMP];
      int16_t rloc[NCMP];
    } cc;
  } u;
  // one bit per pixel, 64 consecutive raster pixels per word: detected,
  // run heads; one bit per run: component roots
  uint64_t fgbits[NSEG];
  uint64_t headbits[NSEG];
  uint64_t rootbits[NRUN / 64];
  int scnt[NSEG];              // runs before each segment
  int rcnt[NRUN / 64];         // roots before each word of rootbits
  int ired[16];
  int nrun, ncomp;
  long long rbase;
};

__device__ __forceinline__ int lds_load(const int* a) {
  return __atomic_load_n(a, __ATOMIC_RELAXED);
}

__device__ __forceinline__ int lfind(int* parent, int x) {
  int px = lds_load(&parent[x]);
  while (px != x) {
    x = px;
    px = lds_load(&parent[x]);
  }
  return x;
}

__device__ __forceinline__ void lunion(int* parent, int a, int b) {
  while (true) {
    a = lfind(parent, a);
    b = lfind(parent, b);
    if (a == b) return;
    if (a < b) { int t = a; a = b; b = t; }
    int old = atomicMin(&parent[a], b);
    if (old == a) return;
    a = old;
  }
}

__device__ __forceinline__ int gload(const int32_t* a) {
  return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int gfind(int32_t* parent, int x) {
  int px = gload(&parent[x]);
  while (px != x) {
    x = px;
    px = gload(&parent[x]);
  }
  return x;
}

__device__ __forceinline__ void gunion(int32_t* parent, int a, int b) {
  while (true) {
    a = gfind(parent, a);
    b = gfind(parent, b);
    if (a == b) return;
    if (a < b) { int t = a; a = b; b = t; }
    int old = atomicMin(&parent[a], b);
    if (old == a) return;
    a = old;
  }
}

}  // namespace

// ---------------------------------------------------------------------
// Plain-path background maps: B32 = fl32(B64), R32 = fl32(R64).
// ---------------------------------------------------------------------
template <int TH, int TW>
__global__ __launch_bounds__(kBlock) void k_bkg_maps(Work wk, ipp_params p) {
  __shared__ SplineLds<TH, TW> S;
  const int tile = blockIdx.x;
  const int f = find_frame(wk.frames, wk.nframes, tile, &FrameDev::dtile0);
  const FrameDev fr = wk.frames[f];
  const int lt = tile - fr.dtile0, ty = lt / fr.dtx, tx = lt - ty * fr.dtx;
  const int y0 = ty * TH, x0 = tx * TW;
  spline_prologue<TH, TW>(wk, fr, p, y0, x0, S);
#pragma unroll 4
  for (int k = 0; k < TH * TW / kBlock; ++k) {
    const int q = threadIdx.x + kBlock * k;
    const int r = q / TW, c = q % TW;
    const int y = y0 + r, x = x0 + c;
    if (y < fr.h && x < fr.w) {
      double b, rr;
      spline_pixel<TH, TW>(S, r, c, &b, &rr);
      const int64_t o = (int64_t)y * fr.w + x;
      fr.bkg[o] = (float)b;
      fr.rms[o] = (float)rr;
    }
  }
}

// ---------------------------------------------------------------------
// Tile kernel: threshold + LDS labelling + records.
//
// NT threads per tile.  Pixel q = t + NT k of the tile (raster order)
// belongs to lane t % 64 of wave t / 64, so each wave instruction covers 64
// consecutive pixels of a row (two half rows for 32-wide tiles).  Detected
// pixels that are horizontally contiguous within such a segment form a
// run.  Runs are numbered in raster order of their first pixel (the head)
// and listed; the union-find works on run numbers, with one union per run
// of the row above that touches a run (and one across a segment split
// inside a row), and counts, bounding boxes and border contact are
// accumulated once per run.  Every pass over runs walks the dense list.
// ---------------------------------------------------------------------
template <int TH, int TW, bool FUSED, bool CONN8, int NT>
__global__ __launch_bounds__(NT) void k_tile_ccl(Work wk, ipp_params p,
                                                 int write_rms) {
  using Lds = CclLds<TH, TW, CONN8>;
  constexpr int NP = Lds::NP;
  constexpr int NSEG = Lds::NSEG;
  constexpr int NRUN = Lds::NRUN;
  constexpr int NCMP = Lds::NCMP;
  constexpr int NW = NT / kWave;              // waves per tile
  constexpr int PPT = NP / NT;                // pixels per thread
  static_assert((TW >= 32 && kWave % TW == 0) || TW % kWave == 0,
                "tile width must divide or be divided by the wave size");
  static_assert(NSEG == kWave && NT % TW == 0 && PPT <= 16 && NW <= 16,
                "4096-pixel tiles, 256 or 512 threads");
  __shared__ Lds L;
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1), wv = t / kWave;
  const int tile = blockIdx.x;
  const int f = find_frame(wk.frames, wk.nframes, tile, &FrameDev::dtile0);
  const FrameDev fr = wk.frames[f];
  const int lt = tile - fr.dtile0, ty = lt / fr.dtx, tx = lt - ty * fr.dtx;
  const int y0 = ty * TH, x0 = tx * TW;

  // Pixel q = t + NT k lies in tile column c = t % TW for every k (TW
  // divides NT) and in tile row t / TW + (NT / TW) k.  A wave instruction
  // covers one row (TW >= 64) or two (TW = 32): the row of the wave's first
  // lane is wave-uniform, so loads and stores take a scalar row pointer and
  // a per-lane 32-bit byte offset fixed for the whole loop.
  constexpr int RSTEP = NT / TW;
  const int c = t % TW;
  const int rw = __builtin_amdgcn_readfirstlane((wv * kWave) / TW);
  const int dr = (wv * kWave + lane) / TW - (wv * kWave) / TW;  // 0 or 1
  const int x = x0 + c;
  const bool xin = x < fr.w;
  const bool interior = y0 + TH <= fr.h && x0 + TW <= fr.w;
  const uint32_t offI = (uint32_t)dr * ((uint32_t)fr.pitch * 4u) +
                        (uint32_t)x * 4u;
  const uint32_t offB = (uint32_t)dr * ((uint32_t)fr.w * 4u) +
                        (uint32_t)x * 4u;
  const char* prow = uniform_ptr(
      (const char*)(fr.pix + (int64_t)(y0 + rw) * fr.pitch));
  const int64_t pstep = (int64_t)RSTEP * fr.pitch * 4;

  // the tile's pixels are requested first, so that their latency overlaps
  // the spline prologue
  float Ipx[PPT], Bv[FUSED ? 1 : PPT], Rv[FUSED ? 1 : PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int y = y0 + rw + dr + RSTEP * k;
    const bool in = interior || (xin && y < fr.h);
    const char* pk = uniform_ptr(prow + pstep * k);
    Ipx[k] = in ? gld((const float*)(pk + offI)) : 0.0f;
    if (!FUSED) {
      const int64_t o = (int64_t)y * fr.w + x;
      Bv[k] = in ? gld(fr.bkg + o) : 0.0f;
      Rv[k] = in ? gld(fr.rms + o) : 0.0f;
    }
  }
  if (FUSED) spline_prologue<TH, TW, NT>(wk, fr, p, y0, x0, L.u.spl);

  // lanes that start / end a row inside the wave's 64-pixel segment
  uint64_t row_first = 1ull, row_last = 1ull << 63;
  if (TW < kWave) {
    for (int l = 0; l < kWave; l += TW) {
      row_first |= 1ull << l;
      row_last |= 1ull << (l + TW - 1);
    }
  }

  // ---- threshold: v = I - B32 > nsigma * R32; runs ----------------------
  // Every prefetched pixel is consumed here, before the loop, so that the
  // loop's stores are never waited on together with a pending load.
  uint32_t finm = 0;
#pragma unroll
  for (int k = 0; k < PPT; ++k) finm |= (uint32_t)isfinite(Ipx[k]) << k;
  SplineX sx;
  if (FUSED) sx = spline_x<TH, TW>(L.u.spl, c);
  char* brow = FUSED ? uniform_ptr((char*)(fr.bkg + (int64_t)(y0 + rw) * fr.w))
                     : nullptr;
  char* rrow = FUSED ? uniform_ptr((char*)(fr.rms + (int64_t)(y0 + rw) * fr.w))
                     : nullptr;
  const int64_t bstep = (int64_t)RSTEP * fr.w * 4;
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    const int r = rw + dr + RSTEP * k;
    const bool in = interior || (xin && y0 + r < fr.h);
    bool det = false;
    if (in) {
      const float I = Ipx[k];
      float B32, R32;
      if (FUSED) {
        double b, rr;
        spline_at<TH, TW>(L.u.spl, sx, r, &b, &rr);
        B32 = (float)b;
        R32 = (float)rr;
        gst((float*)(uniform_ptr(brow + bstep * k) + offB), B32);
        if (write_rms)
          gst((float*)(uniform_ptr(rrow + bstep * k) + offB), R32);
      } else {
        B32 = Bv[k];
        R32 = Rv[k];
      }
      const double v = (double)I - (double)B32;
      const double thr = p.det_nsigma * (double)R32;
      det = ((finm >> k) & 1u) && (v > thr);
    }
    const uint64_t m = __builtin_amdgcn_ballot_w64(det);
    if (lane == 0) {
      L.fgbits[wv + NW * k] = m;
      L.headbits[wv + NW * k] = m & (~(m << 1) | row_first);
    }
  }
  __syncthreads();

  // ---- runs, numbered in raster order of their heads ---------------------
  if (wv == 0) {                   // exclusive scan of the 64 head counts
    const int v = __popcll(L.headbits[lane]);
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int u = __shfl_up(x, o, kWave);
      if (lane >= o) x += u;
    }
    L.scnt[lane] = x - v;
    if (lane == kWave - 1) L.nrun = x;
  }
  if (t < NRUN / 64) L.rootbits[t] = 0;
  __syncthreads();
  const int nrun = L.nrun;
  int* parent = L.u.cc.parent;
  uint16_t* rq = L.u.cc.rq;
  {
    // thread t lists the heads among PPT bits of segment t / (64 / PPT)
    constexpr int TPS = kWave / PPT;
    const int seg = t / TPS, b0 = (t % TPS) * PPT;
    const uint64_t hw = L.headbits[seg];
    uint32_t h = (uint32_t)(hw >> b0) & ((1u << PPT) - 1u);
    int j = L.scnt[seg] + (b0 ? __popcll(hw & (~0ull >> (64 - b0))) : 0);
    while (h) {
      const int b = b0 + __builtin_ctz(h);
      h &= h - 1;
      rq[j] = (uint16_t)(seg * kWave + b);
      parent[j] = j;
      ++j;
    }
  }
  __syncthreads();

  auto fg_at = [&](int q) -> bool {
    return (L.fgbits[q >> 6] >> (q & 63)) & 1ull;
  };
  // length of the run whose head is q
  auto run_len = [&](int q) -> int {
    const int b = q & 63;
    const uint64_t stop = ~L.fgbits[q >> 6] | (row_last << 1);
    return b == 63 ? 1
                   : 1 + __builtin_ctzll((stop >> (b + 1)) | (1ull << (63 - b)));
  };
  // number of the run holding detected pixel q (runs lie inside a segment)
  auto run_of = [&](int q) -> int {
    const int b = q & 63;
    const uint64_t hb =
        L.headbits[q >> 6] & (b == 63 ? ~0ull : ((2ull << b) - 1));
    return L.scnt[q >> 6] + __popcll(hb) - 1;
  };

  // ---- unions with the runs of the row above ----------------------------
  for (int j = t; j < nrun; j += NT) {
    const int q = rq[j];
    const int r = q / TW, c = q % TW;
    // a row run cut by a segment boundary (tiles wider than 64): the run
    // holding q - 1 is the previous run
    if ((q & 63) == 0 && c > 0 && fg_at(q - 1)) lunion(parent, j, j - 1);
    if (r == 0) continue;
    const int c1 = c + run_len(q) - 1;
    const int lo = CONN8 ? max(c - 1, 0) : c;
    const int hi = CONN8 ? min(c1 + 1, TW - 1) : c1;
    // one union per run of the row above that meets [lo, hi]
    int x = q - TW + (lo - c);
    const int xe = q - TW + (hi - c);
    while (x <= xe) {
      const uint64_t w = L.fgbits[x >> 6] >> (x & 63);
      if (!w) { x = ((x >> 6) + 1) << 6; continue; }
      x += __builtin_ctzll(w);
      if (x > xe) break;
      lunion(parent, j, run_of(x));
      const uint64_t z = ~(L.fgbits[x >> 6] >> (x & 63));
      x = z ? x + __builtin_ctzll(z) : ((x >> 6) + 1) << 6;
    }
  }
  __syncthreads();
  // every run points at its root
  for (int j = t; j < nrun; j += NT) {
    const int root = lfind(parent, j);
    parent[j] = root;
    if (root == j) atomicOr((unsigned long long*)&L.rootbits[j >> 6],
                            1ull << (j & 63));
  }
  __syncthreads();

  // ---- component ids in raster order of their roots --------------------
  if (wv == 0) {                   // exclusive scan of the root counts
    const int v = lane < NRUN / 64 ? __popcll(L.rootbits[lane]) : 0;
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const int u = __shfl_up(x, o, kWave);
      if (lane >= o) x += u;
    }
    if (lane < NRUN / 64) L.rcnt[lane] = x - v;
    if (lane == kWave - 1) L.ncomp = x;
  }
  __syncthreads();
  const int ncomp = L.ncomp;
  for (int j = t; j < nrun; j += NT) {
    if (parent[j] != j) continue;
    const uint64_t bits = L.rootbits[j >> 6];
    const uint64_t lt = (j & 63) ? (bits & (~0ull >> (64 - (j & 63)))) : 0;
    const int id = L.rcnt[j >> 6] + __popcll(lt);
    parent[j] = -2 - id;
    L.u.cc.rootp[id] = (int16_t)rq[j];
  }
  for (int c = t; c < ncomp; c += NT) {
    L.u.cc.npix[c] = 0;
    L.u.cc.xmin[c] = TW;
    L.u.cc.xmax[c] = -1;
    L.u.cc.ymax[c] = -1;
  }
  __syncthreads();

  // ---- per-run pixel count, bounding box, inner-border contact ----------
  const bool nb_up = y0 > 0, nb_down = y0 + TH < fr.h;
  const bool nb_left = x0 > 0, nb_right = x0 + TW < fr.w;
  for (int j = t; j < nrun; j += NT) {
    const int q = rq[j];
    const int r = q / TW, c = q % TW;
    const int len = run_len(q);
    const int ce = c + len - 1;
    const int pj = parent[j];
    const int id = pj < 0 ? -2 - pj : -2 - parent[pj];
    if (pj >= 0) parent[j] = -2 - id;   // every run now holds its id
    atomicAdd(&L.u.cc.npix[id], len);
    atomicMin(&L.u.cc.xmin[id], c);
    atomicMax(&L.u.cc.xmax[id], ce);
    atomicMax(&L.u.cc.ymax[id], r);
    const bool edge = (r == 0 && nb_up) || (r == TH - 1 && nb_down) ||
                      (c == 0 && nb_left) || (ce == TW - 1 && nb_right);
    if (edge) atomicOr(&L.u.cc.npix[id], 1 << 30);
  }
  __syncthreads();

  // ---- kept components -> records ---------------------------------------
  constexpr int CPT = NCMP / NT;
  int kc = 0;
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int c = t * CPT + i;
    if (c < ncomp) {
      const int np = L.u.cc.npix[c];
      kc += ((np >> 30) & 1) || ((np & 0x3FFFFFFF) >= p.min_area);
    }
  }
  int ktot;
  int ex = block_exclusive_scan<NW>(kc, L.ired, &ktot);
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int c = t * CPT + i;
    if (c < ncomp) {
      const int np = L.u.cc.npix[c];
      const bool kept = ((np >> 30) & 1) || ((np & 0x3FFFFFFF) >= p.min_area);
      L.u.cc.rloc[c] = kept ? (int16_t)ex : (int16_t)-1;
      ex += kept;
    }
  }
  if (t == 0) {
    long long base = 0;
    if (ktot > 0)
      base = (long long)atomicAdd((unsigned long long*)&wk.counters[0],
                                  (unsigned long long)ktot);
    if (base + ktot > wk.rec_cap)
      atomicOr((unsigned long long*)&wk.counters[2], 1ull);
    L.rbase = base;
    wk.tile_rbase[tile] = (int32_t)(base < wk.rec_cap ? base : wk.rec_cap);
  }
  __syncthreads();
  const long long rbase = L.rbase;
  for (int c = t; c < ncomp; c += NT) {
    const int rl = L.u.cc.rloc[c];
    if (rl < 0) continue;
    const long long rec = rbase + rl;
    if (rec >= wk.rec_cap) continue;
    const int rp = L.u.cc.rootp[c];
    const int rr = rp / TW, rc = rp % TW;
    Rec R;
    R.minidx = (y0 + rr) * fr.w + (x0 + rc);
    R.npix = L.u.cc.npix[c] & 0x3FFFFFFF;
    R.xmin = x0 + L.u.cc.xmin[c];
    R.xmax = x0 + L.u.cc.xmax[c];
    R.ymin = y0 + rr;
    R.ymax = y0 + L.u.cc.ymax[c];
    R.frame = f;
    R.pad = 0;
    wk.recs[rec] = R;
    wk.rparent[rec] = (int32_t)rec;
    wk.rlabel[rec] = 0;
  }
  // ---- run map of the tile: detected / head bits, runs before each
  // segment, per run its record index + 1 ----------------------------------
  uint8_t* tm = wk.tmap + (size_t)tile * kTmapBytes;
  if (t < 64) {
    gst((uint64_t*)(tm + kTmapFg) + t, L.fgbits[t]);
  } else if (t < 128) {
    gst((uint64_t*)(tm + kTmapHead) + (t - 64), L.headbits[t - 64]);
  } else if (t < 192) {
    gst((uint16_t*)(tm + kTmapSeg) + (t - 128), (uint16_t)L.scnt[t - 128]);
  }
  for (int j = t; j < nrun; j += NT) {
    const int rl = L.u.cc.rloc[-2 - parent[j]];
    const uint16_t v =
        (rl >= 0 && rbase + rl < wk.rec_cap) ? (uint16_t)(rl + 1) : 0;
    gst((uint16_t*)(tm + kTmapRun) + j, v);
  }
  // ---- edge records: the record of every pixel on the tile's border -----
  static_assert(2 * (TH + TW) <= kEdgeInts, "edge records of a tile");
  int32_t* te = wk.tedge + (size_t)tile * kEdgeInts;
  for (int e = t; e < 2 * (TH + TW); e += NT) {
    int q;
    if (e < TW) q = e;                                   // top row
    else if (e < 2 * TW) q = (TH - 1) * TW + (e - TW);   // bottom row
    else if (e < 2 * TW + TH) q = (e - 2 * TW) * TW;     // left column
    else q = (e - 2 * TW - TH) * TW + TW - 1;            // right column
    int32_t rec = -1;
    if (fg_at(q)) {
      const int rl = L.u.cc.rloc[-2 - parent[run_of(q)]];
      if (rl >= 0 && rbase + rl < wk.rec_cap) rec = (int32_t)(rbase + rl);
    }
    gst(te + e, rec);
  }
}

// ---------------------------------------------------------------------
// Join records across the right and bottom border of every tile.
// ---------------------------------------------------------------------
template <int TH, int TW>
__global__ __launch_bounds__((border_threads<TH, TW>())) void k_border(
    Work wk, ipp_params p) {
  const int tile = blockIdx.x;
  const int f = find_frame(wk.frames, wk.nframes, tile, &FrameDev::dtile0);
  const FrameDev fr = wk.frames[f];
  const int lt = tile - fr.dtile0, ty = lt / fr.dtx, tx = lt - ty * fr.dtx;
  const int y0 = ty * TH, x0 = tx * TW;
  const bool c8 = p.connectivity == 8;
  // record of frame pixel (y, x) on the border of its tile (-1: none),
  // from that tile's edge records
  auto edge_rec = [&](int y, int x) {
    const int tl = fr.dtile0 + (y / TH) * fr.dtx + (x / TW);
    const int ly = y % TH, lx = x % TW;
    const int idx = lx == 0 ? 2 * TW + ly
                  : lx == TW - 1 ? 2 * TW + TH + ly
                  : ly == 0 ? lx : TW + lx;
    return gld(wk.tedge + (size_t)tl * kEdgeInts + idx);
  };
  const int t = threadIdx.x;
  if (t < TH) {                       // right border
    const int y = y0 + t, x = x0 + TW - 1;
    if (y < fr.h && x + 1 < fr.w) {
      const int ra = edge_rec(y, x);
      if (ra >= 0) {
        for (int dy = c8 ? -1 : 0; dy <= (c8 ? 1 : 0); ++dy) {
          const int yy = y + dy;
          if (yy < 0 || yy >= fr.h) continue;
          const int rb = edge_rec(yy, x + 1);
          if (rb >= 0) gunion(wk.rparent, ra, rb);
        }
      }
    }
  } else if (t < TH + TW) {           // bottom border
    const int y = y0 + TH - 1, x = x0 + (t - TH);
    if (x < fr.w && y + 1 < fr.h) {
      const int ra = edge_rec(y, x);
      if (ra >= 0) {
        for (int dx = c8 ? -1 : 0; dx <= (c8 ? 1 : 0); ++dx) {
          const int xx = x + dx;
          if (xx < 0 || xx >= fr.w) continue;
          const int rb = edge_rec(y + 1, xx);
          if (rb >= 0) gunion(wk.rparent, ra, rb);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------
// Record-level passes (grid-stride over the records in use).
// ---------------------------------------------------------------------
__device__ __forceinline__ long long nrec_used(const Work& wk) {
  const long long u = wk.counters[0];
  return u < wk.rec_cap ? u : wk.rec_cap;
}

__global__ __launch_bounds__(kBlock) void k_resolve(Work wk, ipp_params p) {
  const long long n = nrec_used(wk);
  for (long long r = blockIdx.x * (long long)kBlock + threadIdx.x; r < n;
       r += (long long)gridDim.x * kBlock) {
    const int root = gfind(wk.rparent, (int)r);
    if (root != r) {
      wk.rparent[r] = root;
      const Rec R = wk.recs[r];
      Rec* T = &wk.recs[root];
      atomicAdd(&T->npix, R.npix);
      atomicMin(&T->minidx, R.minidx);
      atomicMin(&T->xmin, R.xmin);
      atomicMax(&T->xmax, R.xmax);
      atomicMin(&T->ymin, R.ymin);
      atomicMax(&T->ymax, R.ymax);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_heads(Work wk, ipp_params p) {
  const long long n = nrec_used(wk);
  for (long long r = blockIdx.x * (long long)kBlock + threadIdx.x; r < n;
       r += (long long)gridDim.x * kBlock) {
    if (wk.rparent[r] != r) continue;
    const Rec R = wk.recs[r];
    if (R.npix < p.min_area) continue;
    const FrameDev& fr = wk.frames[R.frame];
    atomicAdd(&wk.row_count[fr.row0 + R.minidx / fr.w], 1);
  }
}

// Exclusive scan of n <= 2^20 ints in blocks of 1024.
__global__ __launch_bounds__(kBlock) void k_scan_blocks(const int32_t* in,
                                                        int32_t* blocks,
                                                        int n) {
  __shared__ int red[kWaves];
  const int b0 = blockIdx.x * 1024;
  int s = 0;
  for (int i = 0; i < 4; ++i) {
    const int j = b0 + threadIdx.x * 4 + i;
    if (j < n) s += in[j];
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) blocks[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_scan_top(int32_t* blocks,
                                                     int nblocks,
                                                     int64_t* total) {
  __shared__ int red[kWaves];
  int v[4];
  int s = 0;
  for (int i = 0; i < 4; ++i) {
    const int j = threadIdx.x * 4 + i;
    v[i] = j < nblocks ? blocks[j] : 0;
    s += v[i];
  }
  int tot;
  int ex = block_exclusive_scan(s, red, &tot);
  for (int i = 0; i < 4; ++i) {
    const int j = threadIdx.x * 4 + i;
    if (j < nblocks) blocks[j] = ex;
    ex += v[i];
  }
  if (threadIdx.x == 0) *total = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const int32_t* in,
                                                       const int32_t* blocks,
                                                       int32_t* out, int n) {
  __shared__ int red[kWaves];
  const int b0 = blockIdx.x * 1024;
  int v[4];
  int s = 0;
  for (int i = 0; i < 4; ++i) {
    const int j = b0 + threadIdx.x * 4 + i;
    v[i] = j < n ? in[j] : 0;
    s += v[i];
  }
  int tot;
  int ex = block_exclusive_scan(s, red, &tot) + blocks[blockIdx.x];
  for (int i = 0; i < 4; ++i) {
    const int j = b0 + threadIdx.x * 4 + i;
    if (j < n) out[j] = ex;
    ex += v[i];
  }
}

__global__ void k_frame_offsets(Work wk, ipp_sources src) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < wk.nframes)
    src.frame_offsets[f] = wk.row_start[wk.frames[f].row0];
  if (f == 0) {
    src.frame_offsets[wk.nframes] = wk.counters[3];
    if (src.n_total) *src.n_total = wk.counters[3];
  }
}

__global__ __launch_bounds__(kBlock) void k_scatter(Work wk, ipp_params p) {
  const long long n = nrec_used(wk);
  for (long long r = blockIdx.x * (long long)kBlock + threadIdx.x; r < n;
       r += (long long)gridDim.x * kBlock) {
    if (wk.rparent[r] != r) continue;
    const Rec R = wk.recs[r];
    if (R.npix < p.min_area) continue;
    const FrameDev& fr = wk.frames[R.frame];
    const int g = fr.row0 + R.minidx / fr.w;
    const int slot = atomicAdd(&wk.row_cursor[g], 1);
    wk.bucket[wk.row_start[g] + slot] = (int32_t)r;
  }
}

__global__ __launch_bounds__(kBlock) void k_rank(Work wk, ipp_params p,
                                                 ipp_sources src) {
  const long long n = wk.counters[3];
  for (long long e = blockIdx.x * (long long)kBlock + threadIdx.x; e < n;
       e += (long long)gridDim.x * kBlock) {
    const int r = wk.bucket[e];
    const Rec R = wk.recs[r];
    const FrameDev& fr = wk.frames[R.frame];
    const int g = fr.row0 + R.minidx / fr.w;
    const int s0 = wk.row_start[g], cnt = wk.row_count[g];
    int rank = 0;
    for (int i = 0; i < cnt; ++i)
      rank += wk.recs[wk.bucket[s0 + i]].minidx < R.minidx;
    const long long out = (long long)s0 + rank;
    const int label = (int)(out - wk.row_start[fr.row0]) + 1;
    wk.rlabel[r] = label;
    if (out < src.capacity) {
      src.frame[out] = R.frame;
      src.label[out] = label;
      src.npix[out] = R.npix;
      src.xmin[out] = R.xmin;
      src.xmax[out] = R.xmax;
      src.ymin[out] = R.ymin;
      src.ymax[out] = R.ymax;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_reclabel(Work wk) {
  const long long n = nrec_used(wk);
  for (long long r = blockIdx.x * (long long)kBlock + threadIdx.x; r < n;
       r += (long long)gridDim.x * kBlock) {
    const int root = wk.rparent[r];
    if (root != r) wk.rlabel[r] = wk.rlabel[root];
  }
}

template <int TH, int TW>
__global__ __launch_bounds__(kBlock) void k_relabel(Work wk, ipp_params p) {
  __shared__ uint64_t fgs[64], hds[64];
  __shared__ int segs[64];
  __shared__ int runlab[2048];         // label of every run of the tile
  const int tile = blockIdx.x;
  const int f = find_frame(wk.frames, wk.nframes, tile, &FrameDev::dtile0);
  const FrameDev fr = wk.frames[f];
  const int lt = tile - fr.dtile0, ty = lt / fr.dtx, tx = lt - ty * fr.dtx;
  const int y0 = ty * TH, x0 = tx * TW;
  const int rb = wk.tile_rbase[tile];
  const uint8_t* tm = wk.tmap + (size_t)tile * kTmapBytes;
  const int t = threadIdx.x;
  // the run entries of runs 8t .. 8t+7 are requested with the header (the
  // 2048 possible runs fill 256 x 16 bytes), so only the label gathers wait
  // on the run count
  static_assert(kBlock * 8 >= 2048, "one 16-byte group of runs per thread");
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const v4u rr = gld((const v4u*)(tm + kTmapRun) + t);
  if (t < 64) {
    fgs[t] = gld((const uint64_t*)(tm + kTmapFg) + t);
    hds[t] = gld((const uint64_t*)(tm + kTmapHead) + t);
    segs[t] = gld((const uint16_t*)(tm + kTmapSeg) + t);
  }
  __syncthreads();
  // every run's label first (one gather per run), then pixels from LDS
  const int nruns = segs[63] + __popcll(hds[63]);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int r = 8 * t + i;
    if (r >= nruns) break;
    const int l = (int)((rr[i >> 1] >> (16 * (i & 1))) & 0xFFFFu);
    const long long rec = (long long)rb + l - 1;
    runlab[r] = (l && rec < wk.rec_cap) ? gld(wk.rlabel + rec) : 0;
  }
  __syncthreads();
  // label of detected tile pixel q: that of its run
  auto label_at = [&](int q) -> int {
    const int seg = q >> 6, b = q & 63;
    const uint64_t upto = b == 63 ? ~0ull : ((2ull << b) - 1);
    return runlab[segs[seg] + __popcll(hds[seg] & upto) - 1];
  };
  // whole tile inside the frame and 4-pixel groups aligned: int4 stores
  const bool vec = y0 + TH <= fr.h && x0 + TW <= fr.w && (fr.w & 3) == 0 &&
                   ((uintptr_t)fr.labels & 15) == 0;
  if (vec) {
#pragma unroll
    for (int k = 0; k < TH * TW / 4 / kBlock; ++k) {
      const int q = (t + kBlock * k) * 4;
      const int64_t o = (int64_t)(y0 + q / TW) * fr.w + x0 + q % TW;
      const uint32_t d = (uint32_t)(fgs[q >> 6] >> (q & 63)) & 0xFu;
      typedef int v4i __attribute__((ext_vector_type(4)));
      v4i out = {0, 0, 0, 0};
      if (d) {
        if (d & 1u) out.x = label_at(q);
        if (d & 2u) out.y = label_at(q + 1);
        if (d & 4u) out.z = label_at(q + 2);
        if (d & 8u) out.w = label_at(q + 3);
      }
      gst((v4i*)(fr.labels + o), out);
    }
    return;
  }
#pragma unroll 4
  for (int k = 0; k < TH * TW / kBlock; ++k) {
    const int q = t + kBlock * k;
    const int y = y0 + q / TW, x = x0 + q % TW;
    if (y < fr.h && x < fr.w) {
      const bool det = (fgs[q >> 6] >> (q & 63)) & 1ull;
      gst(fr.labels + (int64_t)y * fr.w + x, det ? label_at(q) : 0);
    }
  }
}

// ---------------------------------------------------------------------
// Source table: one wavefront per candidate, exact sums.
// ---------------------------------------------------------------------
namespace {

struct U128 {
  uint64_t lo, hi;
};

__device__ __forceinline__ U128 add128(U128 a, U128 b) {
  U128 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo);
  return r;
}
__device__ __forceinline__ U128 from_i64(int64_t v) {
  U128 r;
  r.lo = (uint64_t)v;
  r.hi = v < 0 ? ~0ull : 0ull;
  return r;
}
// v * m for m >= 0 small (< 2^31)
__device__ __forceinline__ U128 mul_i64(int64_t v, int64_t m) {
  const __int128 p = (__int128)v * (__int128)m;
  U128 r;
  r.lo = (uint64_t)p;
  r.hi = (uint64_t)(p >> 64);
  return r;
}
// Wave reductions: rows of 16 lanes by DPP moves (involutions, so both
// lanes of a pair combine the same two values), then the four row results
// in a fixed order.  Integer sums are exact, so any order gives the same
// result.
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t u) {
  const uint32_t lo = (uint32_t)dpp_mov<CTRL>((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)dpp_mov<CTRL>((int)(uint32_t)(u >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t read_lane_u64(uint64_t u, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u,
                                                          lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane(
      (int)(uint32_t)(u >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}
template <int CTRL>
__device__ __forceinline__ U128 dpp128(U128 v) {
  U128 r;
  r.lo = dpp_u64<CTRL>(v.lo);
  r.hi = dpp_u64<CTRL>(v.hi);
  return r;
}
// Correctly rounded (to nearest, ties to even) conversion to binary64.
__device__ double to_double(U128 v) {
  const bool neg = (int64_t)v.hi < 0;
  unsigned __int128 u = ((unsigned __int128)v.hi << 64) | v.lo;
  if (neg) u = (unsigned __int128)0 - u;
  if (u == 0) return 0.0;
  const uint64_t hi = (uint64_t)(u >> 64), lo = (uint64_t)u;
  const int top = hi ? 127 - __clzll(hi) : 63 - __clzll(lo);
  double r;
  if (top < 53) {
    r = (double)(uint64_t)u;
  } else {
    const int sh = top - 52;
    uint64_t mant = (uint64_t)(u >> sh);
    const unsigned __int128 rem = u & ((((unsigned __int128)1) << sh) - 1);
    const unsigned __int128 half = ((unsigned __int128)1) << (sh - 1);
    if (rem > half || (rem == half && (mant & 1))) mant += 1;
    r = ldexp((double)mant, sh);
  }
  return neg ? -r : r;
}

__device__ __forceinline__ bool exact_range(float a) {
  const float m = fabsf(a);
  return m == 0.0f || (m >= 0.03125f && m <= 16777216.0f);
}

}  // namespace

// Sums of one lane's pixels of a candidate: D = v * 2^28 rounded to an
// integer, and its first moments about the bounding-box corner.
struct StatAcc {
  U128 S, Sx, Sy;
  uint64_t ux, uy;
  double pk;
  int pidx;
  uint32_t flags;
};

// The fixed-point weight D = round(v 2^28) of a pixel value.  Beyond the
// int64 range of the sums it is clamped to +-(2^62 - 1), decided in
// binary64: every binary64 value >= 2^62 exceeds 2^62 - 1 and every smaller
// one is at most 2^62 - 512, so the comparison with 2^62 is exact.
__device__ __forceinline__ int64_t fixed_point_d(double v, bool* clamped) {
  const double s = rint(v * 268435456.0);            // v 2^28
  const int64_t dmax = (int64_t)(((uint64_t)1 << 62) - 1);
  if (s >= 0x1p62) { *clamped = true; return dmax; }
  if (s <= -0x1p62) { *clamped = true; return -dmax; }
  return (int64_t)s;
}

__device__ __forceinline__ void stat_init(StatAcc& a) {
  a.S = {0, 0};
  a.Sx = {0, 0};
  a.Sy = {0, 0};
  a.ux = 0;
  a.uy = 0;
  a.pk = -__builtin_inf();
  a.pidx = 0x7FFFFFFF;
  a.flags = 0;
}

// Pixel (x, y) of frame fr for the candidate with the given label and
// bounding-box corner (xmin, ymin).  The label and the two values are
// loaded together; a pixel of another label contributes zeros.
// The label, value and background of one bounding-box pixel.
struct PixIn {
  int lab;
  float I, B;
};
__device__ __forceinline__ PixIn stat_load(const FrameDev& fr, int x, int y) {
  const int64_t o = (int64_t)y * fr.w + x;
  PixIn q;
  q.lab = gld(fr.labels + o);
  q.I = gld(fr.pix + (int64_t)y * fr.pitch + x);
  q.B = gld(fr.bkg + o);
  return q;
}

__device__ __forceinline__ void stat_acc(StatAcc& a, const FrameDev& fr,
                                         const PixIn& q, int label, int x,
                                         int y, int xmin, int ymin) {
  const bool mem = q.lab == label;
  const float I = q.I, B = q.B;
  const double v = (double)I - (double)B;
  bool inexact = !(exact_range(I) && exact_range(B));
  const int64_t D = mem ? fixed_point_d(v, &inexact) : 0;
  if (mem && inexact) a.flags |= IPP_SRC_INEXACT_SUM_RANGE;
  a.S = add128(a.S, from_i64(D));
  a.Sx = add128(a.Sx, mul_i64(D, x - xmin));
  a.Sy = add128(a.Sy, mul_i64(D, y - ymin));
  a.ux += mem ? (uint64_t)(x - xmin) : 0;
  a.uy += mem ? (uint64_t)(y - ymin) : 0;
  const int idx = y * fr.w + x;
  if (mem && (v > a.pk || (v == a.pk && idx < a.pidx))) {
    a.pk = v;
    a.pidx = idx;
  }
}

__device__ __forceinline__ void stat_pixel(StatAcc& a, const FrameDev& fr,
                                           int label, int x, int y,
                                           int xmin, int ymin) {
  stat_acc(a, fr, stat_load(fr, x, y), label, x, y, xmin, ymin);
}

// Peak: largest value, ties to the smallest index (associative, so any
// reduction order gives the same pair).
__device__ __forceinline__ void stat_take(StatAcc& a, double pv, int pi) {
  if (pv > a.pk || (pv == a.pk && pi < a.pidx)) {
    a.pk = pv;
    a.pidx = pi;
  }
}

template <int CTRL>
__device__ __forceinline__ void stat_dpp_step(StatAcc& a) {
  a.S = add128(a.S, dpp128<CTRL>(a.S));
  a.Sx = add128(a.Sx, dpp128<CTRL>(a.Sx));
  a.Sy = add128(a.Sy, dpp128<CTRL>(a.Sy));
  a.ux += dpp_u64<CTRL>(a.ux);
  a.uy += dpp_u64<CTRL>(a.uy);
  const double pv = dpp_mov<CTRL>(a.pk);
  const int pi = dpp_mov<CTRL>(a.pidx);
  stat_take(a, pv, pi);
  a.flags |= (uint32_t)dpp_mov<CTRL>((int)a.flags);
}

// Every lane of each row of 16 lanes ends with that row's totals.
__device__ __forceinline__ void stat_row16(StatAcc& a) {
  stat_dpp_step<0xB1>(a);          // quad_perm [1,0,3,2]
  stat_dpp_step<0x4E>(a);          // quad_perm [2,3,0,1]
  stat_dpp_step<0x141>(a);         // row_half_mirror
  stat_dpp_step<0x140>(a);         // row_mirror
}

// Totals of the whole wave (after stat_row16), wave-uniform.
__device__ __forceinline__ void stat_rows_combine(StatAcc& a) {
  StatAcc r[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    r[i].S.lo = read_lane_u64(a.S.lo, 16 * i);
    r[i].S.hi = read_lane_u64(a.S.hi, 16 * i);
    r[i].Sx.lo = read_lane_u64(a.Sx.lo, 16 * i);
    r[i].Sx.hi = read_lane_u64(a.Sx.hi, 16 * i);
    r[i].Sy.lo = read_lane_u64(a.Sy.lo, 16 * i);
    r[i].Sy.hi = read_lane_u64(a.Sy.hi, 16 * i);
    r[i].ux = read_lane_u64(a.ux, 16 * i);
    r[i].uy = read_lane_u64(a.uy, 16 * i);
    r[i].pk = read_lane(a.pk, 16 * i);
    r[i].pidx = read_lane(a.pidx, 16 * i);
    r[i].flags = (uint32_t)read_lane((int)a.flags, 16 * i);
  }
  a = r[0];
#pragma unroll
  for (int i = 1; i < 4; ++i) {
    a.S = add128(a.S, r[i].S);
    a.Sx = add128(a.Sx, r[i].Sx);
    a.Sy = add128(a.Sy, r[i].Sy);
    a.ux += r[i].ux;
    a.uy += r[i].uy;
    stat_take(a, r[i].pk, r[i].pidx);
    a.flags |= r[i].flags;
  }
}

// Table row of a candidate from its totals.
__device__ __forceinline__ void stat_finish(const StatAcc& a,
                                            ipp_sources& src, long long row,
                                            int xmin, int ymin, int fw) {
  const double two_q = 268435456.0;
  uint32_t flags = a.flags;
  const double dS = to_double(a.S);
  double cx, cy;
  if ((int64_t)a.S.hi > 0 || ((int64_t)a.S.hi == 0 && a.S.lo > 0)) {
    cx = (double)xmin + to_double(a.Sx) / dS;
    cy = (double)ymin + to_double(a.Sy) / dS;
  } else {
    flags |= IPP_SRC_NONPOSITIVE_FLUX;
    const double np = (double)src.npix[row];
    cx = (double)xmin + (double)(long long)a.ux / np;
    cy = (double)ymin + (double)(long long)a.uy / np;
  }
  src.flux_iso[row] = dS / two_q;
  src.x[row] = cx;
  src.y[row] = cy;
  src.peak[row] = a.pk;
  src.peak_x[row] = a.pidx % fw;
  src.peak_y[row] = a.pidx / fw;
  src.flags[row] = flags;
}

// One wavefront measures four consecutive table rows: those whose bounding
// box holds at most 16 pixels together, one row of 16 lanes per candidate
// (one pixel per lane, DPP reductions inside the row), then each larger one
// over the whole wave.
__global__ __launch_bounds__(kBlock) void k_source_stats(Work wk,
                                                         ipp_sources src) {
  const int lane = threadIdx.x & (kWave - 1);
  long long nrows = wk.counters[3];
  if (nrows > src.capacity) nrows = src.capacity;
  // wave index made provably uniform, so per-row loads are scalar
  const long long wid =
      blockIdx.x * (long long)kWaves +
      __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const long long nw = (long long)gridDim.x * (kBlock / kWave);
  const long long nquads = (nrows + 3) >> 2;
  for (long long qd = wid; qd < nquads; qd += nw) {
    const long long r0 = qd * 4;
    const int seg = lane >> 4, sl = lane & 15;
    const long long rowp = r0 + seg;
    const bool have = rowp < nrows;
    int pxmin = 0, pymin = 0, pbw = 1, parea = 0;
    if (have) {
      pxmin = src.xmin[rowp];
      pymin = src.ymin[rowp];
      pbw = src.xmax[rowp] - pxmin + 1;
      parea = pbw * (src.ymax[rowp] - pymin + 1);
    }
    const bool small = have && parea <= 16;
    const uint64_t smask = __builtin_amdgcn_ballot_w64(small);
    if (smask) {
      // ---- the small candidates, 16 lanes each -------------------------
      StatAcc a;
      stat_init(a);
      int fw = 1;
      if (small) {
        const int f = src.frame[rowp];
        const FrameDev fr = wk.frames[f];
        fw = fr.w;
        if (sl < parea) {
          // small integers: the correctly rounded quotient floors exactly
          const int ey = (int)((float)sl / (float)pbw);
          const int ex = sl - ey * pbw;
          stat_pixel(a, fr, src.label[rowp], pxmin + ex, pymin + ey, pxmin,
                     pymin);
        }
      }
      stat_row16(a);
      if (small && sl == 0) stat_finish(a, src, rowp, pxmin, pymin, fw);
    }
    // ---- each larger candidate over the whole wave -----------------------
    for (int k = 0; k < 4; ++k) {
      const long long row = r0 + k;
      if (row >= nrows) break;
      if ((smask >> (16 * k)) & 1ull) continue;
      const int f = src.frame[row];
      const int label = src.label[row];
      const int xmin = src.xmin[row], xmax = src.xmax[row];
      const int ymin = src.ymin[row], ymax = src.ymax[row];
      const FrameDev fr = wk.frames[f];
      const int bw = xmax - xmin + 1;
      const long long area = (long long)bw * (ymax - ymin + 1);
      StatAcc a;
      stat_init(a);
      // bounding-box position of element e, stepped without divisions;
      // two elements per lane and step, both loaded before either is used
      int ey = lane / bw, ex = lane - (lane / bw) * bw;
      const int dy = kWave / bw, dx = kWave - (kWave / bw) * bw;
      for (long long e = lane; e < area; e += 2 * kWave) {
        const int y0 = ymin + ey, x0 = xmin + ex;
        ey += dy; ex += dx;
        if (ex >= bw) { ex -= bw; ++ey; }
        const int y1 = ymin + ey, x1 = xmin + ex;
        ey += dy; ex += dx;
        if (ex >= bw) { ex -= bw; ++ey; }
        const bool two = e + kWave < area;
        const PixIn q0 = stat_load(fr, x0, y0);
        PixIn q1 = {0, 0.0f, 0.0f};
        if (two) q1 = stat_load(fr, x1, y1);
        stat_acc(a, fr, q0, label, x0, y0, xmin, ymin);
        if (two) stat_acc(a, fr, q1, label, x1, y1, xmin, ymin);
      }
      stat_row16(a);
      stat_rows_combine(a);
      if (lane == 0) stat_finish(a, src, row, xmin, ymin, fr.w);
    }
  }
}

// ---------------------------------------------------------------------
// Second-order moments of each table row's footprint: one wavefront per
// row, exact int128 sums of D, D dx, D dy, D dx^2, D dy^2, D dx dy over the
// bounding box (D = v 2^28 as in the source table, dx and dy from the
// bounding-box corner), each rounded to binary64 once; then the moments and
// the ellipse they describe in a fixed order of binary64 operations.
// ---------------------------------------------------------------------
namespace {
struct MomAcc {
  U128 S, Sx, Sy, Sxx, Syy, Sxy;
};

__device__ __forceinline__ U128 shfl_xor128(U128 v, int m) {
  U128 r;
  const uint32_t l0 = (uint32_t)__shfl_xor((int)(uint32_t)v.lo, m, kWave);
  const uint32_t l1 = (uint32_t)__shfl_xor((int)(uint32_t)(v.lo >> 32), m,
                                           kWave);
  const uint32_t h0 = (uint32_t)__shfl_xor((int)(uint32_t)v.hi, m, kWave);
  const uint32_t h1 = (uint32_t)__shfl_xor((int)(uint32_t)(v.hi >> 32), m,
                                           kWave);
  r.lo = ((uint64_t)l1 << 32) | l0;
  r.hi = ((uint64_t)h1 << 32) | h0;
  return r;
}

__device__ __forceinline__ U128 wave_sum128(U128 v) {
#pragma unroll
  for (int m = kWave / 2; m > 0; m >>= 1) v = add128(v, shfl_xor128(v, m));
  return v;
}

__device__ __forceinline__ void mom_acc(MomAcc& a, const PixIn& q, int label,
                                        int dx, int dy) {
  const double v = (double)q.I - (double)q.B;
  bool clamped = false;
  const int64_t D = q.lab == label ? fixed_point_d(v, &clamped) : 0;
  a.S = add128(a.S, from_i64(D));
  a.Sx = add128(a.Sx, mul_i64(D, dx));
  a.Sy = add128(a.Sy, mul_i64(D, dy));
  a.Sxx = add128(a.Sxx, mul_i64(D, (int64_t)dx * dx));
  a.Syy = add128(a.Syy, mul_i64(D, (int64_t)dy * dy));
  a.Sxy = add128(a.Sxy, mul_i64(D, (int64_t)dx * dy));
}
}  // namespace

// Moments and ellipse from the six sums (binary64, fixed order).
__device__ __forceinline__ void mom_finish(const MomAcc& a, double* out) {
  const bool pos = (int64_t)a.S.hi > 0 || ((int64_t)a.S.hi == 0 && a.S.lo > 0);
  if (!pos) {
    for (int k = 0; k < 6; ++k) out[k] = __builtin_nan("");
    return;
  }
  const double fS = to_double(a.S);
  const double mx = to_double(a.Sx) / fS;
  const double my = to_double(a.Sy) / fS;
  const double x2 = to_double(a.Sxx) / fS - mx * mx;
  const double y2 = to_double(a.Syy) / fS - my * my;
  const double xy = to_double(a.Sxy) / fS - mx * my;
  const double t = (x2 + y2) / 2.0;
  const double hd = (x2 - y2) / 2.0;
  const double r = sqrt(hd * hd + xy * xy);
  out[0] = x2;
  out[1] = y2;
  out[2] = xy;
  out[3] = sqrt(t + r);
  out[4] = sqrt(fmax(t - r, 0.0));
  out[5] = atan2(2.0 * xy, x2 - y2) / 2.0;
}

// Sum over the 16 lanes of a row (lanes 16k .. 16k+15).
__device__ __forceinline__ U128 row_sum128(U128 v) {
#pragma unroll
  for (int m = 8; m > 0; m >>= 1) v = add128(v, shfl_xor128(v, m));
  return v;
}

// One wavefront takes four consecutive rows: those whose bounding box holds
// at most 16 pixels together, 16 lanes each, then each larger one over the
// whole wave.
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(4))) void k_source_moments(Work wk,
                                                           ipp_sources src,
                                                           double* mom) {
  const int lane = threadIdx.x & (kWave - 1);
  long long nrows = src.capacity;
  if (src.n_total && *src.n_total < nrows) nrows = *src.n_total;
  const long long wid =
      blockIdx.x * (long long)kWaves +
      __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const long long nw = (long long)gridDim.x * (kBlock / kWave);
  const long long nquads = (nrows + 3) >> 2;
  const int seg = lane >> 4, sl = lane & 15;
  for (long long qd = wid; qd < nquads; qd += nw) {
    const long long r0 = qd * 4;
    // ---- the small rows, 16 lanes each -----------------------------------
    {
      const long long rowp = r0 + seg;
      bool small = false;
      int f = 0, label = 0, xmin = 0, ymin = 0, bw = 1, area = 0;
      if (rowp < nrows) {
        f = src.frame[rowp];
        if (f >= 0 && f < wk.nframes) {
          const FrameDev& fd = wk.frames[f];
          label = src.label[rowp];
          xmin = max(src.xmin[rowp], 0);
          ymin = max(src.ymin[rowp], 0);
          const int xmax = min(src.xmax[rowp], fd.w - 1);
          const int ymax = min(src.ymax[rowp], fd.h - 1);
          if (xmin <= xmax && ymin <= ymax) {
            bw = xmax - xmin + 1;
            area = bw * (ymax - ymin + 1);
            small = area <= 16;
          }
        }
      }
      const uint64_t smask = __builtin_amdgcn_ballot_w64(small);
      if (smask) {
        MomAcc a;
        a.S = a.Sx = a.Sy = a.Sxx = a.Syy = a.Sxy = from_i64(0);
        if (small && sl < area) {
          // small integers: the correctly rounded quotient floors exactly
          const int ey = (int)((float)sl / (float)bw);
          const int ex = sl - ey * bw;
          const FrameDev fr = wk.frames[f];
          mom_acc(a, stat_load(fr, xmin + ex, ymin + ey), label, ex, ey);
        }
        a.S = row_sum128(a.S);
        a.Sx = row_sum128(a.Sx);
        a.Sy = row_sum128(a.Sy);
        a.Sxx = row_sum128(a.Sxx);
        a.Syy = row_sum128(a.Syy);
        a.Sxy = row_sum128(a.Sxy);
        if (small && sl == 0) mom_finish(a, mom + 6 * rowp);
      }
      // ---- each larger (or unusable) row over the whole wave -------------
      for (int k = 0; k < 4; ++k) {
        const long long row = r0 + k;
        if (row >= nrows) break;
        if ((smask >> (16 * k)) & 1ull) continue;
        const int fk = src.frame[row];
        double* out = mom + 6 * row;
        if (fk < 0 || fk >= wk.nframes) {
          if (lane < 6) out[lane] = __builtin_nan("");
          continue;
        }
        const FrameDev fr = wk.frames[fk];
        const int lab = src.label[row];
        const int x0 = max(src.xmin[row], 0), x1 = min(src.xmax[row], fr.w - 1);
        const int y0 = max(src.ymin[row], 0), y1 = min(src.ymax[row], fr.h - 1);
        MomAcc a;
        a.S = a.Sx = a.Sy = a.Sxx = a.Syy = a.Sxy = from_i64(0);
        if (x0 <= x1 && y0 <= y1) {
          const int w = x1 - x0 + 1;
          const long long ar = (long long)w * (y1 - y0 + 1);
          int ey = lane / w, ex = lane - (lane / w) * w;
          const int dy = kWave / w, dx = kWave - (kWave / w) * w;
          // two bounding-box steps per lane, both loaded before either is
          // summed
          for (long long e = lane; e < ar; e += 2 * kWave) {
            const int ya = ey, xa = ex;
            ey += dy; ex += dx;
            if (ex >= w) { ex -= w; ++ey; }
            const int yb = ey, xb = ex;
            ey += dy; ex += dx;
            if (ex >= w) { ex -= w; ++ey; }
            const bool two = e + kWave < ar;
            const PixIn q0 = stat_load(fr, x0 + xa, y0 + ya);
            PixIn q1 = {0, 0.0f, 0.0f};
            if (two) q1 = stat_load(fr, x0 + xb, y0 + yb);
            mom_acc(a, q0, lab, xa, ya);
            if (two) mom_acc(a, q1, lab, xb, yb);
          }
        }
        a.S = wave_sum128(a.S);
        a.Sx = wave_sum128(a.Sx);
        a.Sy = wave_sum128(a.Sy);
        a.Sxx = wave_sum128(a.Sxx);
        a.Syy = wave_sum128(a.Syy);
        a.Sxy = wave_sum128(a.Sxy);
        if (lane == 0) mom_finish(a, out);
      }
    }
  }
}

#define IPP_TILE_INST(TH, TW)                                              \
  template __global__ void k_bkg_maps<TH, TW>(Work, ipp_params);           \
  template __global__ void k_tile_ccl<TH, TW, true, true, kTileThreads>(Work, ipp_params, \
                                                          int);             \
  template __global__ void k_tile_ccl<TH, TW, true, false, kTileThreads>(Work,           \
                                                           ipp_params, int); \
  template __global__ void k_tile_ccl<TH, TW, false, true, kTileThreads>(Work,           \
                                                           ipp_params, int); \
  template __global__ void k_tile_ccl<TH, TW, false, false, kTileThreads>(Work,          \
                                                            ipp_params, int); \
  template __global__ void k_border<TH, TW>(Work, ipp_params);             \
  template __global__ void k_relabel<TH, TW>(Work, ipp_params);

IPP_TILE_INST(64, 64)
IPP_TILE_INST(32, 128)
IPP_TILE_INST(128, 32)

}  // namespace ipp
