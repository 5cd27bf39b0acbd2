// Deblending and cleaning of detection candidates (Sec. 2.2.5), a
// wavefront or a workgroup per candidate, and the object maps and table
// that follow from them.
//
//   k_db_need    scratch bytes of each candidate (256-byte units)
//   k_scan64_*   exclusive scans (scratch offsets, then object offsets)
//   k_db_small   boxes of up to kDbSmallBox pixels, a wavefront each
//   k_db_large   larger boxes, a workgroup each
//   k_db_write   a wavefront per candidate: object ids into the object
//                maps, the objects' rows (frame, label, parent, pixel
//                count, box)
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
                                                    int64_t* need,
                                                    int32_t* big,
                                                    int64_t* nbig) {
  const long long n = table_rows(cand);
  const long long rows = cand.capacity + 1;
  for (long long r = blockIdx.x * (long long)kBlock + threadIdx.x;
       r <= cand.capacity; r += (long long)gridDim.x * kBlock) {
    int64_t u = 0;
    if (r < n && cand.npix[r] >= 2) {
      const int64_t A = (int64_t)(cand.xmax[r] - cand.xmin[r] + 1) *
                        (cand.ymax[r] - cand.ymin[r] + 1);
      u = (int64_t)((db::pool_bytes(A, cand.npix[r]) + 255) / 256);
      // the workgroup kernel's rows, largest boxes first (the two ends of
      // one list of `rows` entries cannot meet)
      if (A > kDbBigBox) {
        const long long k =
            (long long)atomicAdd((unsigned long long*)&nbig[0], 1ull);
        big[k] = (int32_t)r;
      } else if (A > kDbSmallBox) {
        const long long k =
            (long long)atomicAdd((unsigned long long*)&nbig[1], 1ull);
        big[rows - 1 - k] = (int32_t)r;
      }
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

// ---------------------------------------------------------------------------
// Deblending of one candidate by a group of threads: one wavefront (NW = 1,
// four candidates per workgroup) or the whole workgroup (NW = 4).  Every
// step of the serial description is a pass of the group over the bounding
// box (or over the roots, chains or objects), in raster order where order
// matters: connected components by a lock-free union-find whose roots are
// the components' smallest pixel indices, ranks by ballot prefix counts,
// exact sums by per-key wavefront reductions and atomic limb additions.
// The union-find and chain arrays sit in LDS when the box fits (APX
// pixels) and in the candidate's pool scratch otherwise; the per-root
// arrays likewise (RCAP roots).
// ---------------------------------------------------------------------------

namespace {

template <int NW>
struct Grp {
  static constexpr int T = kWave * NW;
  int tid, lane, wave;
  int* red;          // LDS, NW ints
  int64_t* red64;    // LDS, 2 NW int64

  __device__ __forceinline__ void sync() const {
    if constexpr (NW == 1) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    } else {
      __syncthreads();
    }
  }
  // Orders LDS accesses only (a level of a wavefront's candidate whose
  // shared words are all in LDS: its global stores need not complete).
  __device__ __forceinline__ void sync_lds() const {
    if constexpr (NW == 1) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    } else {
      __syncthreads();
    }
  }
  __device__ __forceinline__ bool any(bool f) const {
    if constexpr (NW == 1) return ballot(f) != 0;
    else return __syncthreads_or(f ? 1 : 0) != 0;
  }
  // Rank of a set flag among the group's threads (thread order) and the
  // number of set flags; called by every thread of the group.
  __device__ __forceinline__ int rank(bool f, int* total) const {
    const uint64_t b = ballot(f);
    const int below = lanes_before(b);
    if constexpr (NW == 1) {
      *total = __popcll(b);
      return below;
    } else {
      __syncthreads();
      if (lane == 0) red[wave] = __popcll(b);
      __syncthreads();
      int off = 0, tot = 0;
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        const int c = red[i];
        off += i < wave ? c : 0;
        tot += c;
      }
      *total = tot;
      return off + below;
    }
  }
  // Group sums of two int64 values, returned to every thread.
  __device__ __forceinline__ void sum2(int64_t& a, int64_t& b) const {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
      a += __shfl_xor(a, o, kWave);
      b += __shfl_xor(b, o, kWave);
    }
    if constexpr (NW > 1) {
      __syncthreads();
      if (lane == 0) {
        red64[2 * wave] = a;
        red64[2 * wave + 1] = b;
      }
      __syncthreads();
      a = 0;
      b = 0;
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        a += red64[2 * i];
        b += red64[2 * i + 1];
      }
    }
  }
};

// LDS of one group: APX pixels of union-find and chain words, RCAP roots
// per level, and (a wavefront's candidates, NW = 1) one byte per chain
// record that a level found a node below the chain's top insignificant.
template <int NW, int APX, int RCAP>
struct DbLds {
  static constexpr int kClr = NW == 1 ? 2 * APX + 16 : 1;
  int par[APX], ch[APX];
  int64_t accL[RCAP], accH[RCAP];
  int accN[RCAP], pch[RCAP], nch[RCAP];
  int red[NW];
  int64_t red64[2 * NW];
  uint8_t clr[kClr];
};

// Accesses of words that other threads of the group update atomically.
__device__ __forceinline__ int ld_at(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t ld_at(const int64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_at(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void add_at(int64_t* p, int64_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void add_at(int* p, int v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void min_at(int* p, int v) {
  __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Union-find over par (-1: not in the level's mask).  Every word points to
// a smaller index of the same component (linking puts the larger root
// under the smaller), so a component's root is its first pixel.  The find
// halves the path it walks: a word is overwritten with its grandparent,
// which keeps both properties; a link that such a write replaces belongs
// to a union whose atomic found its target already linked, and that union
// joins the target's new root itself before it returns.
__device__ __forceinline__ int uf_find(int* par, int x) {
  while (true) {
    const int px = ld_at(par + x);
    if (px == x) return x;
    const int gp = ld_at(par + px);
    if (gp == px) return px;
    st_at(par + x, gp);
    x = gp;
  }
}
__device__ __forceinline__ void uf_unite(int* par, int a, int b) {
  while (true) {
    a = uf_find(par, a);
    b = uf_find(par, b);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old =
        __hip_atomic_fetch_min(par + b, a, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    if (old == b) return;
    b = old;       // b was linked meanwhile: join a with b's new parent
  }
}

// Adds NV int64 values of each active lane to the accumulators of its key
// (op(key, j, sum)): the wavefront first sums the values of equal keys,
// one lane per distinct key then adds them.
template <int NV, class Op>
__device__ __forceinline__ void keyed_add(bool act, int key,
                                          const int64_t* v, int lane,
                                          Op&& op) {
  uint64_t left = ballot(act);
  while (left) {
    const int lead = __ffsll((unsigned long long)left) - 1;
    const int k0 = __builtin_amdgcn_readlane(key, lead);
    const bool in = act && key == k0;
    left &= ~ballot(in);
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      int64_t s = in ? v[j] : 0;
#pragma unroll
      for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
      if (lane == lead) op(k0, j, s);
    }
    act = act && !in;
  }
}
// The same with the minimum of one int per key (op(key, min)).
template <class Op>
__device__ __forceinline__ void keyed_min(bool act, int key, int v, int lane,
                                          Op&& op) {
  uint64_t left = ballot(act);
  while (left) {
    const int lead = __ffsll((unsigned long long)left) - 1;
    const int k0 = __builtin_amdgcn_readlane(key, lead);
    const bool in = act && key == k0;
    left &= ~ballot(in);
    int s = in ? v : 0x7FFFFFFF;
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) s = min(s, __shfl_xor(s, o, kWave));
    if (lane == lead) op(k0, s);
    act = act && !in;
  }
}

__device__ __forceinline__ void limbs4(__int128 t, int64_t* l) {
  const unsigned __int128 u = (unsigned __int128)t;
  l[0] = (int64_t)(uint32_t)u;
  l[1] = (int64_t)(uint32_t)(u >> 32);
  l[2] = (int64_t)(uint32_t)(u >> 64);
  l[3] = (int64_t)(t >> 96);
}

__device__ __forceinline__ void chain_init(db::Chain& c, double F,
                                           int parent) {
  c.F_top = F;
  c.nobj_sum = 0;
  c.parent = parent;
  c.cnt = 0;
  c.nsig = 0;
  c.one = -1;
  c.nobj = 1;
  c.mode = 0;
  c.bmode = 0;
  c.allsig = 1;
  c.reached = 0;
  c.objof = -1;
  c.slot = -1;
  c.first = 0x7FFFFFFF;
}

struct DbCand {
  int lab, x0, y0, bw, bh, m;
  double t0, peak;
};

// Deblends one candidate; returns the object count (every thread of the
// group gets it) with s.asg set for every member, or -1 when the chain
// records would exceed the scratch (not reachable with the bounds of
// pool_bytes).  Every thread of the group calls it.
template <int NW, int APX, int RCAP>
__device__ int deblend_group(const Grp<NW>& g, DbLds<NW, APX, RCAP>& L,
                             const FrameDev& fr, const DbCand& c, int conn,
                             int nthresh, int clean, double mincont,
                             double kc, db::Pool& s) {
  constexpr int T = Grp<NW>::T;
  const int A = c.bw * c.bh;
  const int bw = c.bw;
  const double inv_bw = 1.0 / (double)bw;
  auto row_of = [&](int p) {
    int y = (int)((double)p * inv_bw);
    if (y * bw > p) --y;
    else if ((y + 1) * bw <= p) ++y;
    return y;
  };
  // a wavefront's candidate (NW = 1, at most APX pixels and, with either
  // connectivity, at most APX / 2 roots per level) keeps every word a level
  // shares in LDS, so its levels synchronise on LDS alone and its chain
  // records are only written (children counted, significance flags kept in
  // LDS); a workgroup's candidate may use the pool
  constexpr bool kLds = NW == 1;
  static_assert(!kLds || 2 * RCAP >= APX, "a level's roots fit the LDS");
  int* par = (kLds || A <= APX) ? L.par : s.par;
  int* ch = (kLds || A <= APX) ? L.ch : s.ch;
  const double ninf = -__builtin_inf();

  // members' values, the candidate's flux
  int64_t fl = 0, fh = 0;
  for (int c0 = 0; c0 < A; c0 += T) {
    const int p = c0 + g.tid;
    if (p < A) {
      const int y = row_of(p), x = p - y * bw;
      const int64_t row = c.y0 + y;
      const int64_t q = row * fr.w + c.x0 + x;
      const bool mem = fr.labels[q] == c.lab;
      const double v =
          (double)fr.pix[row * fr.pitch + c.x0 + x] - (double)fr.bkg[q];
      s.val[p] = mem ? v : ninf;
      s.asg[p] = mem ? 0 : -1;
      ch[p] = 0;
      if (mem) {
        const int64_t d = db::fixed_d(v);
        fl += (int64_t)(uint32_t)d;
        fh += d >> 32;
      }
    }
  }
  g.sync();
  if (!(c.t0 > 0.0) || c.m < 2 || !(c.peak > c.t0)) return 1;
  g.sum2(fl, fh);
  const double froot = db::to_f64(db::from_limbs2(fl, fh)) * 0x1p-28;
  const double fmin = mincont * froot;
  double q = c.peak / c.t0;
  for (int k = nthresh; k > 1; k >>= 1) q = sqrt(q);
  if (g.tid == 0) chain_init(s.chains[0], froot, -1);
  if constexpr (kLds) {
    if (g.tid == 0) L.clr[0] = 0;
  }
  g.sync();

  // levels upward: components, their intensities, chain records
  auto lsync = [&] {
    if constexpr (kLds) g.sync_lds();
    else g.sync();
  };
  int nch = 1;
  bool fail = false;
  double t = c.t0;
  // the last full level: its mask size, roots and per-root arrays
  int nup_prev = -1, nroots = 0;
  int64_t *aL = nullptr, *aH = nullptr;
  int *aN = nullptr, *pc = nullptr, *nc = nullptr;
  for (int i = 1; i < nthresh; ++i) {
    t = t * q;
    // the level's mask; each horizontal run of a wavefront's 64 pixels
    // points to its first pixel, which points to the pixel before it when
    // the run goes on from the previous 64
    int nup = 0;                       // this wave's mask pixels
    for (int c0 = 0; c0 < A; c0 += T) {
      const int p = c0 + g.tid;
      bool up = false;
      int x = 0;
      if (p < A) {
        up = s.val[p] > t;
        x = p - row_of(p) * bw;
      }
      const uint64_t um = ballot(up);
      nup += __popcll(um);
      const uint64_t starts = (um & ~(um << 1)) | (um & ballot(x == 0)) | (um & 1ull);
      if (p < A) {
        int v = -1;
        if (up) {
          const int j =
              63 - __builtin_clzll(starts & ((2ull << g.lane) - 1ull));
          if (j < g.lane) v = p - (g.lane - j);
          else v = (g.lane == 0 && x > 0 && s.val[p - 1] > t) ? p - 1 : p;
        }
        par[p] = v;
      }
    }
    if (!g.any(nup > 0)) break;
    // the masks are nested, so a mask of the previous full level's size is
    // that mask: the same components, each its parent node's only child;
    // every chain goes on and only the intensities above this level change
    {
      int all = nup;
      if constexpr (NW > 1) {
        __syncthreads();
        if (g.lane == 0) g.red[g.wave] = nup;
        __syncthreads();
        all = 0;
        for (int w = 0; w < NW; ++w) all += g.red[w];
      }
      nup = all;
    }
    if (nup == nup_prev) {
      for (int k = g.tid; k < nroots; k += T) {
        const double F =
            db::to_f64(db::from_limbs2(ld_at(aL + k), ld_at(aH + k))) *
                0x1p-28 -
            (double)ld_at(aN + k) * t;
        if (!(F > fmin)) {
          if constexpr (kLds) L.clr[nc[k]] = 1;
          else s.chains[nc[k]].allsig = 0;
        }
      }
      lsync();
      continue;
    }
    nup_prev = nup;
    lsync();
    // links to the row above: a run's first pixel takes its upper-left and
    // upper neighbours, every pixel its upper-right one (8-connectivity),
    // which covers every pair of the run and the row above; with
    // 4-connectivity every pixel its upper neighbour
    for (int c0 = 0; c0 < A; c0 += T) {
      const int p = c0 + g.tid;
      if (p < A && ld_at(par + p) >= 0) {
        const int y = row_of(p), x = p - y * bw;
        if (y > 0) {
          const int u = p - bw;
          if (conn == 8) {
            if (!(x > 0 && ld_at(par + p - 1) >= 0)) {
              if (x > 0 && ld_at(par + u - 1) >= 0) uf_unite(par, p, u - 1);
              if (ld_at(par + u) >= 0) uf_unite(par, p, u);
            }
            if (x + 1 < bw && ld_at(par + u + 1) >= 0)
              uf_unite(par, p, u + 1);
          } else if (ld_at(par + u) >= 0) {
            uf_unite(par, p, u);
          }
        }
      }
    }
    lsync();
    for (int c0 = 0; c0 < A; c0 += T) {
      const int p = c0 + g.tid;
      if (p < A && ld_at(par + p) >= 0) {
        const int r = uf_find(par, p);
        if (r != p) st_at(par + p, r);
      }
    }
    lsync();
    // roots in raster order: a root's word becomes -2 - rank
    nroots = 0;
    for (int c0 = 0; c0 < A; c0 += T) {
      const int p = c0 + g.tid;
      const bool isroot = p < A && ld_at(par + p) == p;
      int tot;
      const int k = nroots + g.rank(isroot, &tot);
      if (isroot) par[p] = -2 - k;
      nroots += tot;
    }
    const bool rl = kLds || nroots <= RCAP;
    aL = rl ? L.accL : s.accL;
    aH = rl ? L.accH : s.accH;
    aN = rl ? L.accN : s.accN;
    pc = rl ? L.pch : s.pch;
    nc = rl ? L.nch : s.nch;
    for (int k = g.tid; k < nroots; k += T) {
      aL[k] = 0;
      aH[k] = 0;
      aN[k] = 0;
    }
    lsync();
    // exact sums of the weights and counts per component
    for (int c0 = 0; c0 < A; c0 += T) {
      const int p = c0 + g.tid;
      bool up = false;
      int key = 0;
      int64_t v[3] = {0, 0, 0};
      if (p < A) {
        const int pv = ld_at(par + p);
        if (pv != -1) {
          up = true;
          key = pv <= -2 ? -2 - pv : -2 - ld_at(par + pv);
          if (pv <= -2) pc[key] = ch[p];
          const int64_t d = db::fixed_d(s.val[p]);
          v[0] = (int64_t)(uint32_t)d;
          v[1] = d >> 32;
          v[2] = 1;
        }
      }
      keyed_add<3>(up, key, v, g.lane, [&](int k, int j, int64_t sum) {
        if (j == 0) add_at(aL + k, sum);
        else if (j == 1) add_at(aH + k, sum);
        else add_at(aN + k, (int)sum);
      });
    }
    lsync();
    // children per parent chain (a wavefront's candidate: counted from the
    // roots' parent words in LDS)
    if constexpr (!kLds) {
      for (int k = g.tid; k < nroots; k += T) st_at(&s.chains[pc[k]].cnt, 0);
      g.sync();
      for (int k = g.tid; k < nroots; k += T) add_at(&s.chains[pc[k]].cnt, 1);
      g.sync();
    }
    // a parent with one child: its chain goes on; else a chain per child,
    // numbered in root order
    for (int k0 = 0; k0 < nroots; k0 += T) {
      const int k = k0 + g.tid;
      bool fresh = false;
      int pcv = 0;
      double F = 0.0;
      if (k < nroots) {
        pcv = pc[k];
        F = db::to_f64(db::from_limbs2(ld_at(aL + k), ld_at(aH + k))) *
                0x1p-28 -
            (double)ld_at(aN + k) * t;
        if constexpr (kLds) {
          int nk = 0;
          for (int j2 = 0; j2 < nroots; ++j2) nk += pc[j2] == pcv ? 1 : 0;
          fresh = nk != 1;
        } else {
          fresh = ld_at(&s.chains[pcv].cnt) != 1;
        }
      }
      int tot;
      const int j = nch + g.rank(fresh, &tot);
      if (k < nroots) {
        if (!fresh) {
          if constexpr (kLds) {
            if (!(F > fmin)) L.clr[pcv] = 1;
          } else {
            s.chains[pcv].allsig &= F > fmin ? 1 : 0;
          }
          nc[k] = pcv;
        } else {
          if (j < s.chain_cap) {
            chain_init(s.chains[j], F, pcv);
            if constexpr (kLds) L.clr[j] = 0;
          }
          nc[k] = j;
        }
      }
      nch += tot;
    }
    if (nch > s.chain_cap) {
      fail = true;
      break;
    }
    lsync();
    for (int c0 = 0; c0 < A; c0 += T) {
      const int p = c0 + g.tid;
      if (p < A) {
        const int pv = ld_at(par + p);
        if (pv != -1) ch[p] = nc[pv <= -2 ? -2 - pv : -2 - ld_at(par + pv)];
      }
    }
    lsync();
  }
  g.sync();
  if (fail) return -1;
  if constexpr (kLds) {
    for (int j = g.tid; j < nch; j += T)
      if (L.clr[j]) s.chains[j].allsig = 0;
    g.sync();
  }

  // pruning, children before parents (they were created later), then the
  // object path, parents before children: one thread
  if (g.tid == 0) {
    for (int k = nch - 1; k >= 0; --k) {
      db::Chain& C = s.chains[k];
      int bmode = 0;
      int64_t nb = 1;
      if (C.nsig >= 2) {
        bmode = 1;
        nb = C.nobj_sum;
      } else if (C.nsig == 1 && s.chains[C.one].nobj >= 2) {
        bmode = 2;
        nb = s.chains[C.one].nobj;
      }
      C.bmode = bmode;
      if (bmode != 0 && C.allsig) {
        C.mode = 1;
        C.nobj = (int32_t)nb;
      } else {
        C.mode = 0;
        C.nobj = 1;
      }
      if (C.parent >= 0 && C.F_top > fmin) {
        db::Chain& P = s.chains[C.parent];
        P.nsig += 1;
        P.nobj_sum += C.nobj;
        P.one = k;
      }
    }
    if (s.chains[0].nobj >= 2) {
      for (int k = 0; k < nch; ++k) {
        db::Chain& C = s.chains[k];
        if (k == 0) {
          C.reached = 1;
        } else {
          const db::Chain& P = s.chains[C.parent];
          C.reached = P.reached && P.mode == 1 &&
                      ((P.bmode == 1 && C.F_top > fmin) ||
                       (P.bmode == 2 && P.one == k));
        }
        const bool obj = C.reached && C.mode == 0;
        C.objof = obj ? k : (k > 0 ? s.chains[C.parent].objof : -1);
      }
    }
  }
  g.sync();
  if (ld_at(&s.chains[0].nobj) < 2) return 1;

  // seeds: the first pixel of each object chain (par reused for marks)
  for (int c0 = 0; c0 < A; c0 += T) {
    const int p = c0 + g.tid;
    int o = -1;
    if (p < A) {
      par[p] = -1;
      if (s.asg[p] >= 0) {
        o = s.chains[ch[p]].objof;
        if (o < 0) s.asg[p] = -2;          // not in a seed
      }
    }
    keyed_min(o >= 0, o, p, g.lane,
              [&](int k, int v) { min_at(&s.chains[k].first, v); });
  }
  g.sync();
  for (int j = g.tid; j < nch; j += T) {
    if (s.chains[j].objof == j) {
      const int f = ld_at(&s.chains[j].first);
      if (f != 0x7FFFFFFF) par[f] = j;
    }
  }
  g.sync();
  // object slots in raster order of the first pixels
  int K = 0;
  for (int c0 = 0; c0 < A; c0 += T) {
    const int p = c0 + g.tid;
    const int j = p < A ? ld_at(par + p) : -1;
    int tot;
    const int k = K + g.rank(j >= 0, &tot);
    if (j >= 0 && k < s.obj_cap) {
      s.chains[j].slot = k;
      db::Obj& b = s.objs[k];
      for (int a = 0; a < 5; ++a)
        for (int l = 0; l < 4; ++l) b.m[a][l] = 0;
      b.fin[0] = 0;
      b.fin[1] = 0;
      b.nfin = 0;
      b.first = p;
      b.xmin = 0x7FFFFFFF;
      b.ymin = row_of(p);
      b.target = -1;
    }
    K += tot;
  }
  if (K > s.obj_cap) return -1;
  g.sync();
  for (int c0 = 0; c0 < A; c0 += T) {
    const int p = c0 + g.tid;
    int k = -1, x = 0;
    if (p < A && s.asg[p] >= 0) {
      k = s.chains[s.chains[ch[p]].objof].slot;
      s.asg[p] = k;
      x = p - row_of(p) * bw;
    }
    keyed_min(k >= 0, k, x, g.lane,
              [&](int kk, int v) { min_at(&s.objs[kk].xmin, v); });
  }
  g.sync();
  // seed moments about each seed's corner, one sum at a time
  for (int c0 = 0; c0 < A; c0 += T) {
    const int p = c0 + g.tid;
    int k = -1;
    int64_t d = 0, dx = 0, dy = 0;
    if (p < A) {
      k = s.asg[p];
      if (k >= 0) {
        const db::Obj& b = s.objs[k];
        const int y = row_of(p), x = p - y * bw;
        d = db::fixed_d(s.val[p]);
        dx = x - ld_at(&b.xmin);
        dy = y - b.ymin;
      }
    }
    for (int a = 0; a < 5; ++a) {
      const int64_t f = a == 0   ? 1
                        : a == 1 ? dx
                        : a == 2 ? dy
                        : a == 3 ? dx * dx
                                 : dy * dy;
      int64_t v[4];
      limbs4((__int128)d * f, v);
      keyed_add<4>(k >= 0, k, v, g.lane, [&](int kk, int j, int64_t sum) {
        add_at(&s.objs[kk].m[a][j], sum);
      });
    }
  }
  g.sync();
  for (int k = g.tid; k < K; k += T) {
    db::Obj& b = s.objs[k];
    int64_t l[5][4];
    for (int a = 0; a < 5; ++a)
      for (int j = 0; j < 4; ++j) l[a][j] = ld_at(&b.m[a][j]);
    const double fS = db::to_f64(db::from_limbs4(l[0]));
    const double mx = db::to_f64(db::from_limbs4(l[1])) / fS;
    const double my = db::to_f64(db::from_limbs4(l[2])) / fS;
    const double x2 = db::to_f64(db::from_limbs4(l[3])) / fS - mx * mx;
    const double y2 = db::to_f64(db::from_limbs4(l[4])) / fS - my * my;
    const int xmin = ld_at(&b.xmin);
    b.F = fS * 0x1p-28;
    b.xc = (double)(c.x0 + xmin) + mx;
    b.yc = (double)(c.y0 + b.ymin) + my;
    b.s2 = (x2 + y2) + 1.0 / 6.0;
  }
  g.sync();
  // the other pixels: the brightest model
  for (int c0 = 0; c0 < A; c0 += T) {
    const int p = c0 + g.tid;
    if (p < A && s.asg[p] == -2) {
      const int py = row_of(p);
      const double x = (double)(c.x0 + p - py * bw);
      const double y = (double)(c.y0 + py);
      double best = -1.0;
      int bk = 0;
      for (int k = 0; k < K; ++k) {
        const db::Obj& b = s.objs[k];
        const double dx = x - b.xc;
        const double dy = y - b.yc;
        const double d2 = dx * dx + dy * dy;
        const double den = b.s2 + d2;
        const double sc = (b.F * b.s2) / (den * den);
        if (sc > best) {
          best = sc;
          bk = k;
        }
      }
      s.asg[p] = bk;
    }
  }
  g.sync();
  if (!clean) return K;

  // cleaning
  for (int c0 = 0; c0 < A; c0 += T) {
    const int p = c0 + g.tid;
    int k = -1;
    int64_t v[3] = {0, 0, 0};
    if (p < A) {
      k = s.asg[p];
      if (k >= 0) {
        const int64_t d = db::fixed_d(s.val[p]);
        v[0] = (int64_t)(uint32_t)d;
        v[1] = d >> 32;
        v[2] = 1;
      }
    }
    keyed_add<3>(k >= 0, k, v, g.lane, [&](int kk, int j, int64_t sum) {
      if (j < 2) add_at(&s.objs[kk].fin[j], sum);
      else add_at(&s.objs[kk].nfin, sum);
    });
  }
  g.sync();
  const double pi = 3.14159265358979311600;   // binary64 nearest to pi
  for (int o = g.tid; o < K; o += T) {
    db::Obj& b = s.objs[o];
    const double mu =
        db::to_f64(db::from_limbs2(ld_at(&b.fin[0]), ld_at(&b.fin[1]))) *
        0x1p-28 / (double)ld_at(&b.nfin);
    double tot = 0.0, best = -1.0;
    int bm = -1;
    for (int m = 0; m < K; ++m) {
      if (m == o) continue;
      const db::Obj& n = s.objs[m];
      const bool brighter = n.F > b.F || (n.F == b.F && m < o);
      if (!brighter) continue;
      const double dx = b.xc - n.xc;
      const double dy = b.yc - n.yc;
      const double d2 = dx * dx + dy * dy;
      double den = n.s2 + d2;
      den = den * den;
      den = pi * den;
      const double cm = kc * ((n.F * n.s2) / den);
      tot += cm;
      if (cm > best) {
        best = cm;
        bm = m;
      }
    }
    b.target = (bm >= 0 && mu - tot < c.t0) ? bm : o;
  }
  g.sync();
  // follow merges to an object that stays; number the survivors in order
  for (int o = g.tid; o < K; o += T) {
    int k = o;
    while (s.objs[k].target != k) k = s.objs[k].target;
    s.objs[o].final_obj = k;
  }
  g.sync();
  int nk = 0;
  for (int o0 = 0; o0 < K; o0 += T) {
    const int o = o0 + g.tid;
    const bool surv = o < K && s.objs[o].final_obj == o;
    int tot;
    const int r = nk + g.rank(surv, &tot);
    if (o < K) s.objs[o].idx = surv ? r : -1;
    nk += tot;
  }
  g.sync();
  for (int c0 = 0; c0 < A; c0 += T) {
    const int p = c0 + g.tid;
    if (p < A) {
      const int k = s.asg[p];
      if (k >= 0) s.asg[p] = s.objs[s.objs[k].final_obj].idx;
    }
  }
  g.sync();
  return nk;
}

// Candidates with bounding boxes of more than amin and at most amax
// pixels, one per group, taken from the queue counter in row order; with
// `trivial`, also the counts of the rows
// that need no deblending (beyond the table: 0; single pixels, or every
// row when the pool is too small: 1).
template <int NW, int APX, int RCAP>
__device__ __forceinline__ void db_groups(
    Work wk, ipp_sources cand, const int64_t* off, const int64_t* tot,
    char* pool, int64_t pool_units, double nsigma, int conn, int nthresh,
    int clean, double mincont, double kc, int64_t* cnt, int64_t* queue,
    int64_t amin, int64_t amax, bool trivial, const int32_t* big = nullptr,
    const int64_t* nbig = nullptr) {
  constexpr int G = kBlock / (kWave * NW);
  __shared__ DbLds<NW, APX, RCAP> lds[G];
  const int gi = threadIdx.x / (kWave * NW);
  Grp<NW> g;
  g.tid = threadIdx.x % (kWave * NW);
  g.lane = threadIdx.x & (kWave - 1);
  g.wave = g.tid / kWave;
  g.red = lds[gi].red;
  g.red64 = lds[gi].red64;
  const long long n = table_rows(cand);
  const bool fits = *tot <= pool_units;
  if (trivial) {
    for (long long r = blockIdx.x * (long long)kBlock + threadIdx.x;
         r <= cand.capacity; r += (long long)gridDim.x * kBlock) {
      if (r >= n) cnt[r] = 0;
      else if (cand.npix[r] < 2 || !fits) cnt[r] = 1;
    }
  }
  if (!fits) return;
  __shared__ long long next_row;
  while (true) {
    // the next row from the queue (a wavefront's lane 0, or the
    // workgroup's thread 0 through LDS)
    long long r = 0;
    if constexpr (NW == 1) {
      long long v = 0;
      if (g.lane == 0)
        v = (long long)atomicAdd((unsigned long long*)queue, 1ull);
      r = __shfl(v, 0, kWave);
    } else {
      if (g.tid == 0)
        next_row = (long long)atomicAdd((unsigned long long*)queue, 1ull);
      __syncthreads();
      r = next_row;
      __syncthreads();
    }
    if (big) {                         // the workgroup kernel's list
      const long long nb0 = nbig[0], nb1 = nbig[1];
      if (r >= nb0 + nb1) break;
      r = r < nb0 ? big[r] : big[cand.capacity - (r - nb0)];
    }
    if (r >= n) break;
    const int m = cand.npix[r];
    DbCand c;
    c.x0 = cand.xmin[r];
    c.y0 = cand.ymin[r];
    c.bw = cand.xmax[r] - c.x0 + 1;
    c.bh = cand.ymax[r] - c.y0 + 1;
    const int64_t A = (int64_t)c.bw * c.bh;
    if (m < 2 || A <= amin || A > amax) continue;
    const int f = cand.frame[r];
    const FrameDev fr = wk.frames[f];
    c.lab = cand.label[r];
    c.m = m;
    c.t0 = nsigma * (double)fr.rms[(int64_t)cand.peak_y[r] * fr.w +
                                   cand.peak_x[r]];
    c.peak = cand.peak[r];
    db::Pool s = db::carve(pool + off[r] * 256, A, m);
    int k = deblend_group<NW, APX, RCAP>(g, lds[gi], fr, c, conn, nthresh,
                                         clean, mincont, kc, s);
    if (k < 0) {
      if (g.tid == 0)
        atomicOr((unsigned long long*)&wk.counters[2], 2ull);
      k = 1;
      for (int64_t p = g.tid; p < A; p += Grp<NW>::T)
        if (s.asg[p] != -1) s.asg[p] = 0;
    }
    if (g.tid == 0) cnt[r] = k;
    g.sync();
  }
}

}  // namespace

// Boxes of up to 512 pixels: a wavefront per candidate.
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(3))) void k_db_small(
    Work wk, ipp_sources cand, const int64_t* off, const int64_t* tot,
    char* pool, int64_t pool_units, double nsigma, int conn, int nthresh,
    int clean, double mincont, double kc, int64_t* cnt, int64_t* queue) {
  db_groups<1, kDbSmallBox, kDbSmallBox / 2>(wk, cand, off, tot, pool, pool_units,
                                 nsigma, conn, nthresh, clean, mincont, kc,
                                 cnt, queue, -1, kDbSmallBox, true);
}

// Larger boxes: a workgroup per candidate (LDS arrays up to 4096 pixels
// and 1024 roots, the pool beyond), taken from the list k_db_need made:
// boxes over kDbBigBox pixels first, so that the longest candidates start
// first.
__global__ __launch_bounds__(kBlock) void k_db_large(
    Work wk, ipp_sources cand, const int64_t* off, const int64_t* tot,
    char* pool, int64_t pool_units, double nsigma, int conn, int nthresh,
    int clean, double mincont, double kc, int64_t* cnt, int64_t* queue,
    const int32_t* big, const int64_t* nbig) {
  db_groups<kWaves, 4096, 1024>(wk, cand, off, tot, pool, pool_units,
                                nsigma, conn, nthresh, clean, mincont, kc,
                                cnt, queue, kDbSmallBox, INT64_MAX, false,
                                big, nbig);
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

// One wavefront per candidate: its objects' rows (lane-parallel), then its
// bounding box in rounds of 64 pixels (positions stepped without division):
// the ids in the object map and, for a split candidate, each object's pixel
// count and box, reduced over the round per object and added to its row
// with one atomic per object and round (integer sums, minima and maxima:
// the same whatever the order).
__global__ __launch_bounds__(kBlock) void k_db_write(
    Work wk, ipp_sources cand, const int64_t* off, const int64_t* tot,
    const char* pool, int64_t pool_units, const int64_t* cnt,
    const int64_t* ooff, ipp_sources obj, int32_t* parent) {
  const long long n = table_rows(cand);
  const bool fits = *tot <= pool_units;
  const int lane = threadIdx.x & (kWave - 1);
  const long long wid =
      blockIdx.x * (long long)kWaves +
      __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const long long nw = (long long)gridDim.x * kWaves;
  for (long long r = wid; r < n; r += nw) {
    const int f = cand.frame[r];
    const FrameDev fr = wk.frames[f];
    const int lab = cand.label[r];
    const int64_t base = ooff[r];
    const int64_t first = ooff[cand.frame_offsets[f]];
    const int k = (int)cnt[r];
    const int x0 = cand.xmin[r], y0 = cand.ymin[r];
    const int bw = cand.xmax[r] - x0 + 1, bh = cand.ymax[r] - y0 + 1;
    for (int j = lane; j < k; j += kWave) {
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
    const int64_t A = (int64_t)bw * bh;
    const int dy = kWave / bw, dx = kWave - (kWave / bw) * bw;
    int y = lane / bw, x = lane - (lane / bw) * bw;
    if (k == 1 || !fits || cand.npix[r] < 2) {
      for (int64_t e0 = 0; e0 < A; e0 += kWave) {
        if (e0 + lane < A) {
          const int64_t q = (int64_t)(y0 + y) * fr.w + x0 + x;
          if (fr.labels[q] == lab) fr.objects[q] = id0;
        }
        y += dy;
        x += dx;
        if (x >= bw) {
          x -= bw;
          ++y;
        }
      }
      continue;
    }
    // the rows' initial values are in memory before the atomics below
    // (this wave's stores completed; the atomics are performed in the
    // same L2): a workgroup-scope release, which waits for them without
    // the device-scope cache write-back
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    const db::Pool s =
        db::carve((char*)pool + off[r] * 256, A, cand.npix[r]);
    for (int64_t e0 = 0; e0 < A; e0 += kWave) {
      const int64_t e = e0 + lane;
      int a = -1;
      const int px = x0 + x, py = y0 + y;
      if (e < A) {
        a = s.asg[e];
        if (a >= 0) fr.objects[(int64_t)py * fr.w + px] = id0 + a;
      }
      y += dy;
      x += dx;
      if (x >= bw) {
        x -= bw;
        ++y;
      }
      bool act = a >= 0 && base + a < obj.capacity;
      uint64_t left = ballot(act);
      while (left) {
        const int lead = __ffsll((unsigned long long)left) - 1;
        const int k0 = __builtin_amdgcn_readlane(a, lead);
        const bool in = act && a == k0;
        const uint64_t m = ballot(in);
        left &= ~m;
        int xn = in ? px : 0x7FFFFFFF, xm = in ? px : -1;
        int yn = in ? py : 0x7FFFFFFF, ym = in ? py : -1;
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) {
          xn = min(xn, __shfl_xor(xn, o, kWave));
          xm = max(xm, __shfl_xor(xm, o, kWave));
          yn = min(yn, __shfl_xor(yn, o, kWave));
          ym = max(ym, __shfl_xor(ym, o, kWave));
        }
        if (lane == lead) {
          const int64_t o = base + k0;
          atomicAdd(&obj.npix[o], (int32_t)__popcll(m));
          atomicMin(&obj.xmin[o], xn);
          atomicMax(&obj.xmax[o], xm);
          atomicMin(&obj.ymin[o], yn);
          atomicMax(&obj.ymax[o], ym);
        }
        act = act && !in;
      }
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
