// Internal definitions shared by the HIP kernels and the host side of
// libipp: device frame descriptors, the workspace layout, and small
// block-level helpers for 256-thread (4 x wave64) workgroups on gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ipp.h"

namespace ipp {

constexpr int kBlock = 256;          // threads per workgroup everywhere
constexpr int kWave = 64;            // CDNA wavefront
constexpr int kWaves = kBlock / kWave;
constexpr uint32_t kSentinel = 0xFFFFFFFFu;  // excluded pixel key
constexpr int kFixedBits = 28;       // fraction bits of the exact sums
constexpr int kMaxNcol = 8;          // mesh columns a detection tile spans

// Device-side descriptor of one frame of a batch.
struct FrameDev {
  const float* pix;
  const uint8_t* mask;
  int64_t pitch;
  int32_t h, w;
  int32_t ny, nx;        // mesh nodes
  int32_t node0;         // first node (= first mesh region) in batch arrays
  int32_t dty, dtx;      // detection tile grid
  int32_t dtile0;        // first detection tile in batch arrays
  int32_t row0;          // first row in batch row arrays
  int64_t pix0;          // first pixel in batch pixel arrays
  float* bkg;            // maps (inputs in map mode, outputs otherwise)
  float* rms;
  int32_t* labels;
  double* o_bkg_raw;     // optional mesh outputs
  double* o_rms_raw;
  int32_t* o_n;
  double* o_bkg;
  double* o_rms;
  float* dpix;           // pixel gradient (photometry backward), or null
  int32_t line0[2];      // first mesh line of each spline pass
  int32_t* objects;      // object map written by deblending, or null
};

// Stamp convolution and subtraction (k_subtract.hip).
constexpr int kSubMaxHw = 15;       // kernel half-width
constexpr int kSubMaxStamp = 32;    // stamp size
constexpr int kSubMaxGauss = 4;     // Gaussians of the basis
constexpr int kSubMaxOrder = 7;     // order i + j of each
constexpr int kSubMaxBasis = kSubMaxGauss * (kSubMaxOrder + 1) *
                             (kSubMaxOrder + 2) / 2;
struct SubFrame {
  const float* I;        // science frame
  const float* R;        // template, same shape
  int64_t pitchI, pitchR;
  int32_t h, w;
  int32_t nsy, nsx;      // stamps per column and per row
  int64_t stamp0;        // first stamp of the frame in the batch
  float* D;              // difference, dense h x w
  const double* coef;    // a_n polynomials, then B's
};
struct SubBasis {
  int32_t hw, stamp, ngauss, spatial_order, bkg_order, nbasis;
  int32_t order[kSubMaxGauss];
  double sigma[kSubMaxGauss];
};

// Frame of the gray-scale calls: input, output and the zscale sample grid.
struct GrayFrame {
  const float* pix;
  int64_t pitch;
  int32_t h, w;
  int32_t s;             // zscale sample step
  int32_t sy, sx;        // sample grid rows, columns (sy * sx <= kZMax)
  int32_t row0;          // first row of the frame among the batch's rows
  float* out;            // h x w, row pitch w (nullable where unused)
};
constexpr int kZMax = 1024;       // zscale sample capacity
constexpr int kMaxBins = 4096;    // histogram equalization bins
// workgroups of the asinh backward (grid-stride): its binary64 block
// partials fill at most 2 * kAsinhMaxBlocks doubles
constexpr int kAsinhMaxBlocks = 2048;

// Partial candidate: the piece of a connected component inside one
// detection tile that touches the tile border or is large enough to keep.
struct Rec {
  int32_t minidx;        // first pixel in frame raster order (y*w + x)
  int32_t npix;
  int32_t xmin, xmax, ymin, ymax;
  int32_t frame;
  int32_t pad;
};

// Device pointers of one call's workspace (carved out by the host).
struct Work {
  FrameDev* frames;
  int32_t nframes;
  int32_t total_nodes;
  int32_t total_dtiles;
  int32_t total_rows;
  int32_t total_lines[2];
  int64_t total_pix;
  // mesh, one entry per node of every frame
  double* m_bkg;         // raw estimator value
  double* m_rms;
  int32_t* m_n;
  double* f_bkg;         // after fill
  double* f_rms;
  int32_t* f_pass;       // pass at which a node became known (-1 unknown)
  double* tb[4];         // spline tables of the background: f, fxx, fyy, fxxyy
  double* tr[4];         // same for the rms
  double* sc0;           // Thomas scratch
  double* sc1;
  uint32_t* frame_flags; // per frame
  // detection
  uint8_t* tmap;         // per detection tile: its run map (kTmap*)
  int32_t* tedge;        // per detection tile: record of each edge pixel
  int32_t* tile_rbase;   // per detection tile: first record
  Rec* recs;
  int32_t* rparent;      // union-find parent of each record
  int32_t* rlabel;       // final frame-local label of each record (0 = none)
  int64_t rec_cap;
  int32_t* row_count;    // per batch row: kept candidates starting there
  int32_t* row_start;    // exclusive scan of row_count
  int32_t* row_cursor;
  int32_t* bucket;       // record of each kept candidate, grouped by row
  int32_t* scan_blocks;  // per scan block partial sums
  int64_t* counters;     // [0] records used [1] record capacity
                         // [2] overflow bits [3] candidates found
};

// Run map of one detection tile (4096 pixels, 64 segments of 64 raster
// pixels), kTmapBytes bytes per tile: detected bits, run-head bits, the
// exclusive prefix of head counts per segment, and per run (raster order
// of heads) its record index within the tile + 1 (0: not kept).
constexpr int kTmapFg = 0;              // uint64_t[64]
constexpr int kTmapHead = 512;          // uint64_t[64]
constexpr int kTmapSeg = 1024;          // uint16_t[64]
constexpr int kTmapRun = 1152;          // uint16_t[2048]
constexpr int kTmapBytes = 1152 + 4096;

// Edge records of one detection tile, kEdgeInts int32 per tile: the record
// index of every pixel on the tile's border (-1: none), top row [0, TW),
// bottom row [TW, 2TW), left column [2TW, 2TW+TH), right column
// [2TW+TH, 2TW+2TH).
constexpr int kEdgeInts = 320;          // 2 (TH + TW) for 32x128 tiles

// ---------------------------------------------------------------- helpers
// Stores and loads through the global address space (the pointers come
// from descriptors in memory, where the compiler would use flat accesses).
template <typename T>
__device__ __forceinline__ void gst(T* a, T v) {
  *(__attribute__((address_space(1))) T*)a = v;
}
template <typename T>
__device__ __forceinline__ T gld(const T* a) {
  return *(const __attribute__((address_space(1))) T*)a;
}
// A wave-uniform pointer moved to scalar registers, so that loads can take
// it as their scalar base.
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t u = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return (T*)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint32_t f2key(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key2f(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __uint_as_float(u);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = v + __shfl_xor(v, o, kWave);
  return v;
}

// Wave ballot of a predicate, and the number of set bits of a mask below
// the calling lane (two mbcnt instructions).
__device__ __forceinline__ uint64_t ballot(bool b) {
  return __builtin_amdgcn_ballot_w64(b);
}
__device__ __forceinline__ int lanes_before(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi(
      (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Lane moves inside rows of 16 lanes (DPP: no LDS round trip).  The
// patterns used are involutions, so both lanes of a pair add the same two
// values and every lane ends with a bit-identical sum.  Every lane of
// every row is written (permutations inside a row), so no lane keeps an
// old value and none is needed.
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)dpp_mov<CTRL>((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)dpp_mov<CTRL>((int)(uint32_t)(u >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ double read_lane(double v, int lane) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u,
                                                          lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane(
      (int)(uint32_t)(u >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ int read_lane(int v, int lane) {
  return __builtin_amdgcn_readlane(v, lane);
}
template <typename T>
__device__ __forceinline__ T row16_sum(T v) {
  v = v + dpp_mov<0xB1>(v);        // quad_perm [1,0,3,2]
  v = v + dpp_mov<0x4E>(v);        // quad_perm [2,3,0,1]
  v = v + dpp_mov<0x141>(v);       // row_half_mirror
  v = v + dpp_mov<0x140>(v);       // row_mirror
  return v;
}
// Row broadcasts (DPP row_bcast:15 / row_bcast:31): the last lane of the
// previous row (of row 1) to the rows in ROWS; lanes of other rows read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_bcast(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_bcast(double v) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)dpp_bcast<CTRL, ROWS>((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)dpp_bcast<CTRL, ROWS>((int)(uint32_t)(u >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
// Wave sums of binary64 and int: rows by DPP, then the four row sums r0..r3
// combined as (r0 + r1) + (r2 + r3): rows 1 and 3 add the last lanes of
// rows 0 and 2, row 3 then adds the last lane of row 1, and lane 63's value
// is read (addition commutes bit for bit, so the order is that one).  The
// result is wave-uniform; every lane must be active.
template <typename T>
__device__ __forceinline__ T wave_sum_rows(T v) {
  v = row16_sum(v);
  v = v + dpp_bcast<0x142, 0xA>(v);
  v = v + dpp_bcast<0x143, 0x8>(v);
  return read_lane(v, 63);
}
__device__ __forceinline__ double wave_sum(double v) {
  return wave_sum_rows(v);
}
__device__ __forceinline__ int wave_sum(int v) { return wave_sum_rows(v); }
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, kWave);
    v = u < v ? u : v;
  }
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, kWave);
    v = u > v ? u : v;
  }
  return v;
}

// Block-wide reductions for 256 threads.  `red` is LDS scratch of at least
// kWaves elements of T; the result is returned to every thread.  The
// combination order is fixed, so floating-point sums are deterministic.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  T r = (red[0] + red[1]) + (red[2] + red[3]);
  return r;
}
template <typename T>
__device__ __forceinline__ T block_min(T v, T* red) {
  v = wave_min(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  T a = red[0] < red[1] ? red[0] : red[1];
  T b = red[2] < red[3] ? red[2] : red[3];
  return a < b ? a : b;
}
template <typename T>
__device__ __forceinline__ T block_max(T v, T* red) {
  v = wave_max(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  T a = red[0] > red[1] ? red[0] : red[1];
  T b = red[2] > red[3] ? red[2] : red[3];
  return a > b ? a : b;
}

// Exclusive scan over the threads of a block of NW waves (int).  `red` is
// LDS scratch of NW ints.  Returns the exclusive prefix; *total gets the
// sum.
template <int NW = kWaves>
__device__ __forceinline__ int block_exclusive_scan(int v, int* red,
                                                    int* total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  int x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int u = __shfl_up(x, o, kWave);
    if (lane >= o) x += u;
  }
  __syncthreads();
  if (lane == kWave - 1) red[w] = x;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    off += i < w ? red[i] : 0;
    tot += red[i];
  }
  *total = tot;
  return off + x - v;
}

// Frame owning a flat index, given each frame's first index (ascending).
__device__ __forceinline__ int find_frame(const FrameDev* fr, int nframes,
                                          int idx, int FrameDev::*first) {
  int lo = 0, hi = nframes - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (fr[mid].*first <= idx) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Natural-spline node coordinate along one axis: centre of region i.
__device__ __forceinline__ double node_coord(int i, int m, int n) {
  int a = i * m;
  int b = min(a + m, n);
  return 0.5 * (double)(a + b - 1);
}

// Weights (A, B, C, D) of S(t) = A f_j + B f_{j+1} + C M_j + D M_{j+1} for
// the natural cubic spline on nodes node_coord(0..n-1), extended linearly
// beyond the end nodes; j is returned in *j (j+1 clamped for n == 1).
__device__ __forceinline__ void spline_weights(double t, int m, int len,
                                               int n, int* jout,
                                               double* w4) {
  if (n == 1) {
    *jout = 0;
    w4[0] = 1.0; w4[1] = 0.0; w4[2] = 0.0; w4[3] = 0.0;
    return;
  }
  // interval: largest j <= n-2 with t_j <= t (t_0 if below)
  int j = (int)floor((t - (0.5 * (m - 1))) / (double)m);
  j = max(0, min(j, n - 2));
  double tj = node_coord(j, m, len);
  double tj1 = node_coord(j + 1, m, len);
  if (t < tj && j > 0) { --j; tj1 = tj; tj = node_coord(j, m, len); }
  if (t > tj1 && j < n - 2) { ++j; tj = tj1; tj1 = node_coord(j + 1, m, len); }
  double h = tj1 - tj;
  *jout = j;
  if (t < tj) {                 // left extension (j == 0)
    double u = (t - tj) / h;
    w4[0] = 1.0 - u; w4[1] = u;
    w4[2] = -u * h * h / 3.0; w4[3] = -u * h * h / 6.0;
  } else if (t > tj1) {         // right extension (j == n-2)
    double u = (t - tj1) / h;
    w4[0] = -u; w4[1] = 1.0 + u;
    w4[2] = u * h * h / 6.0; w4[3] = u * h * h / 3.0;
  } else {
    double A = (tj1 - t) / h;
    double B = (t - tj) / h;
    w4[0] = A; w4[1] = B;
    w4[2] = (A * A * A - A) * (h * h) / 6.0;
    w4[3] = (B * B * B - B) * (h * h) / 6.0;
  }
}

}  // namespace ipp
