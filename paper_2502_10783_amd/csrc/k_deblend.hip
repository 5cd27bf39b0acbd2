// Deblending and cleaning of detection candidates (Sec. 2.2.5), one thread
// per candidate (the paper's mapping of these phases), and the object maps
// and table that follow from them.
//
//   k_db_need    scratch bytes of each candidate (256-byte units)
//   k_scan64_*   exclusive scans (scratch offsets, then object offsets)
//   k_db_run     per candidate: its values into scratch, deblend_one()
//   k_db_write   per candidate: object ids into the object maps, the
//                objects' rows (frame, label, parent, pixel count, box)
//   k_db_offsets per-frame object offsets and count
//   k_db_flags   BLENDED on the objects of split candidates (after the
//                pre-analysis kernel has filled the rows)
#include "deblend_core.h"
#include "ipp_internal.h"
#include "kernels.h"

namespace ipp {

namespace {
__device__ __forceinline__ long long table_rows(const ipp_sources& t) {
  long long n = t.capacity;
  if (t.n_total && *t.n_total < n) n = *t.n_total;
  return n;
}

__device__ __forceinline__ int64_t block_scan64(int64_t v, int64_t* red,
                                                int64_t* total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t u = __shfl_up(x, o, kWave);
    if (lane >= o) x += u;
  }
  __syncthreads();
  if (lane == kWave - 1) red[w] = x;
  __syncthreads();
  int64_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    off += i < w ? red[i] : 0;
    tot += red[i];
  }
  *total = tot;
  return off + x - v;
}
}  // namespace

__global__ __launch_bounds__(kBlock) void k_db_need(ipp_sources cand,
                                                    int64_t* need) {
  const long long n = table_rows(cand);
  for (long long r = blockIdx.x * (long long)kBlock + threadIdx.x;
       r <= cand.capacity; r += (long long)gridDim.x * kBlock) {
    int64_t u = 0;
    if (r < n && cand.npix[r] >= 2) {
      const int64_t A = (int64_t)(cand.xmax[r] - cand.xmin[r] + 1) *
                        (cand.ymax[r] - cand.ymin[r] + 1);
      u = (int64_t)((db::scratch_bytes(A, cand.npix[r]) + 255) / 256);
    }
    need[r] = u;
  }
}

// Exclusive scan of n int64 values: block sums of 1024 values, a scan of
// the block sums by one workgroup (chunks of 1024 with a carry), and the
// scan inside each block.
__global__ __launch_bounds__(kBlock) void k_scan64_blocks(const int64_t* in,
                                                          int64_t* blocks,
                                                          int64_t n) {
  __shared__ int64_t red[kWaves];
  const int64_t b0 = blockIdx.x * (int64_t)1024;
  int64_t s = 0;
  for (int i = 0; i < 4; ++i) {
    const int64_t j = b0 + threadIdx.x * 4 + i;
    if (j < n) s += in[j];
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) blocks[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_scan64_top(int64_t* blocks,
                                                       int64_t nblocks,
                                                       int64_t* total) {
  __shared__ int64_t red[kWaves];
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < nblocks; c0 += 1024) {
    int64_t v[4];
    int64_t s = 0;
    for (int i = 0; i < 4; ++i) {
      const int64_t j = c0 + threadIdx.x * 4 + i;
      v[i] = j < nblocks ? blocks[j] : 0;
      s += v[i];
    }
    int64_t tot;
    int64_t ex = block_scan64(s, red, &tot) + carry;
    for (int i = 0; i < 4; ++i) {
      const int64_t j = c0 + threadIdx.x * 4 + i;
      if (j < nblocks) blocks[j] = ex;
      ex += v[i];
    }
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan64_apply(const int64_t* in,
                                                         const int64_t* blocks,
                                                         int64_t* out,
                                                         int64_t n) {
  __shared__ int64_t red[kWaves];
  const int64_t b0 = blockIdx.x * (int64_t)1024;
  int64_t v[4];
  int64_t s = 0;
  for (int i = 0; i < 4; ++i) {
    const int64_t j = b0 + threadIdx.x * 4 + i;
    v[i] = j < n ? in[j] : 0;
    s += v[i];
  }
  int64_t tot;
  int64_t ex = block_scan64(s, red, &tot) + blocks[blockIdx.x];
  for (int i = 0; i < 4; ++i) {
    const int64_t j = b0 + threadIdx.x * 4 + i;
    if (j < n) out[j] = ex;
    ex += v[i];
  }
}

// One thread per candidate.  off: scratch offsets (256-byte units), *tot:
// their total; a candidate whose block would pass the pool is left whole
// and the overflow bit is set (the call's diagnostics report it).
__global__ __launch_bounds__(64) void k_db_run(
    Work wk, ipp_sources cand, const int64_t* off, const int64_t* tot,
    char* pool, int64_t pool_units, double nsigma, int conn, int nthresh,
    int clean, double mincont, double kc, int64_t* cnt) {
  const long long n = table_rows(cand);
  const bool fits = *tot <= pool_units;
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
       r <= cand.capacity; r += (long long)gridDim.x * blockDim.x) {
    if (r >= n) {
      cnt[r] = 0;
      continue;
    }
    const int m = cand.npix[r];
    if (m < 2 || !fits) {            // whole (the diagnostics report a
      cnt[r] = 1;                    // pool too small)
      continue;
    }
    const int f = cand.frame[r];
    const FrameDev fr = wk.frames[f];
    const int lab = cand.label[r];
    db::Cand c;
    c.x0 = cand.xmin[r];
    c.y0 = cand.ymin[r];
    c.bw = cand.xmax[r] - c.x0 + 1;
    c.bh = cand.ymax[r] - c.y0 + 1;
    c.npix = m;
    c.t0 = nsigma * (double)fr.rms[(int64_t)cand.peak_y[r] * fr.w +
                                   cand.peak_x[r]];
    c.peak = cand.peak[r];
    c.conn = conn;
    c.nthresh = nthresh;
    c.clean = clean;
    c.mincont = mincont;
    c.kc = kc;
    const int64_t A = (int64_t)c.bw * c.bh;
    db::Scratch s = db::carve(pool + off[r] * 256, A, m);
    const double ninf = -__builtin_inf();
    for (int y = 0; y < c.bh; ++y) {
      const int64_t row = (int64_t)(c.y0 + y);
      for (int x = 0; x < c.bw; ++x) {
        const int64_t q = row * fr.w + c.x0 + x;
        const bool mem = fr.labels[q] == lab;
        const double v =
            (double)fr.pix[row * fr.pitch + c.x0 + x] - (double)fr.bkg[q];
        s.val[y * c.bw + x] = mem ? v : ninf;
      }
    }
    int k = db::deblend_one(c, s);
    if (k < 0) {
      atomicOr((unsigned long long*)&wk.counters[2], 2ull);
      k = 1;
      for (int64_t p = 0; p < A; ++p)
        if (s.asg[p] != -1) s.asg[p] = 0;
    }
    cnt[r] = k;
  }
}

__global__ __launch_bounds__(kBlock) void k_db_zero(Work wk) {
  for (int f = blockIdx.y; f < wk.nframes; f += gridDim.y) {
    const FrameDev fr = wk.frames[f];
    const int64_t np = (int64_t)fr.h * fr.w;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < np;
         i += (int64_t)gridDim.x * kBlock)
      fr.objects[i] = 0;
  }
}

// One thread per candidate: its objects' rows and their ids in the map.
__global__ __launch_bounds__(64) void k_db_write(
    Work wk, ipp_sources cand, const int64_t* off, const int64_t* tot,
    const char* pool, int64_t pool_units, const int64_t* cnt,
    const int64_t* ooff, ipp_sources obj, int32_t* parent) {
  const long long n = table_rows(cand);
  const bool fits = *tot <= pool_units;
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
       r < n; r += (long long)gridDim.x * blockDim.x) {
    const int f = cand.frame[r];
    const FrameDev fr = wk.frames[f];
    const int lab = cand.label[r];
    const int64_t base = ooff[r];
    const int64_t first = ooff[cand.frame_offsets[f]];
    const int k = (int)cnt[r];
    const int x0 = cand.xmin[r], y0 = cand.ymin[r];
    const int bw = cand.xmax[r] - x0 + 1, bh = cand.ymax[r] - y0 + 1;
    for (int j = 0; j < k; ++j) {
      const int64_t o = base + j;
      if (o >= obj.capacity) break;
      obj.frame[o] = f;
      obj.label[o] = (int32_t)(o - first + 1);
      parent[o] = lab;
      if (k == 1) {
        obj.npix[o] = cand.npix[r];
        obj.xmin[o] = x0;
        obj.xmax[o] = cand.xmax[r];
        obj.ymin[o] = y0;
        obj.ymax[o] = cand.ymax[r];
      } else {
        obj.npix[o] = 0;
        obj.xmin[o] = 0x7FFFFFFF;
        obj.xmax[o] = -1;
        obj.ymin[o] = 0x7FFFFFFF;
        obj.ymax[o] = -1;
      }
    }
    const int32_t id0 = (int32_t)(base - first + 1);
    if (k == 1 || !fits || cand.npix[r] < 2) {
      for (int y = 0; y < bh; ++y)
        for (int x = 0; x < bw; ++x) {
          const int64_t q = (int64_t)(y0 + y) * fr.w + x0 + x;
          if (fr.labels[q] == lab) fr.objects[q] = id0;
        }
      continue;
    }
    const int64_t A = (int64_t)bw * bh;
    const db::Scratch s =
        db::carve((char*)pool + off[r] * 256, A, cand.npix[r]);
    for (int y = 0; y < bh; ++y)
      for (int x = 0; x < bw; ++x) {
        const int a = s.asg[y * bw + x];
        if (a < 0) continue;
        const int64_t q = (int64_t)(y0 + y) * fr.w + x0 + x;
        fr.objects[q] = id0 + a;
        const int64_t o = base + a;
        if (o >= obj.capacity) continue;
        obj.npix[o] += 1;
        const int px = x0 + x, py = y0 + y;
        if (px < obj.xmin[o]) obj.xmin[o] = px;
        if (px > obj.xmax[o]) obj.xmax[o] = px;
        if (py < obj.ymin[o]) obj.ymin[o] = py;
        if (py > obj.ymax[o]) obj.ymax[o] = py;
      }
  }
}

__global__ void k_db_offsets(Work wk, ipp_sources cand, const int64_t* ooff,
                             const int64_t* total, ipp_sources obj) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f <= wk.nframes)
    obj.frame_offsets[f] =
        f < wk.nframes ? ooff[cand.frame_offsets[f]] : *total;
  if (f == 0) {
    if (obj.n_total) *obj.n_total = *total;
    wk.counters[3] = *total;
  }
}

__global__ __launch_bounds__(kBlock) void k_db_flags(
    ipp_sources cand, const int64_t* cnt, const int64_t* total,
    ipp_sources obj, const int32_t* parent) {
  long long n = *total;
  if (n > obj.capacity) n = obj.capacity;
  for (long long o = blockIdx.x * (long long)kBlock + threadIdx.x; o < n;
       o += (long long)gridDim.x * kBlock) {
    const int64_t cr = cand.frame_offsets[obj.frame[o]] + parent[o] - 1;
    if (cnt[cr] > 1) obj.flags[o] |= IPP_SRC_BLENDED;
  }
}

}  // namespace ipp

namespace ipp {
__global__ void k_db_diag(const int64_t* tot, int64_t pool_units,
                          const int64_t* counters, int64_t* diag) {
  if (threadIdx.x == 0) {
    diag[0] = tot[0] * 256;
    diag[1] = pool_units * 256;
    diag[2] = (tot[0] > pool_units ? 1 : 0) | counters[2];
    diag[3] = tot[1];
  }
}
}  // namespace ipp
