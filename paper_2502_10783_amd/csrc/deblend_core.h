// Records and helpers of multi-threshold deblending and cleaning
// (Sec. 2.2.5: deblending and cleaning phases), shared by the kernels in
// k_deblend.hip.
//
// Readings (the paper states the phases, not their formulas):
//  levels   t0 = nsigma R32(peak pixel); q = (peak / t0)^(1/N) by log2(N)
//           square roots; t_i = t_{i-1} q for i = 1 .. N-1 (binary64).
//  tree     at level i the candidate's pixels with v > t_i form components
//           (the detection's connectivity), each inside one component of
//           level i-1; the candidate is the root (level 0).
//  contrast a node is significant iff its intensity above its level,
//           fl(S 2^-28) - n t_i with S the exact sum of the fixed-point
//           weights, exceeds mincont times the candidate's flux.
//  pruning  bottom up: a leaf is one object; a node with >= 2 significant
//           children stands for their objects; with one, for that child's
//           objects if it has >= 2, else for itself; with none, itself.
//  seeds    the pixels of the object nodes, numbered in raster order of
//           their first pixels; the other pixels go to the seed whose
//           Moffat (index 2) model F s2 / (s2 + d^2)^2 is largest there
//           (F, barycentre and s2 = x2 + y2 + 1/6 from the seed's exact
//           moments), ties to the lower index.
//  cleaning an object whose mean value minus the modelled light of the
//           brighter objects at its seed barycentre, k_c F s2 /
//           (pi (s2 + d^2)^2) summed in index order, falls below t0 is
//           merged into the brightest such contributor.
//
// Tree representation: chains.  A node with exactly one child at the next
// level and that child carry the same objects unless the child's own
// subtree splits, and the intensity can only grow towards the root, so a
// run of single-child nodes is kept as one chain record (its top node's
// intensity, and whether every node below the top is significant).  Chains
// are created where a node has two or more children, numbered in the
// raster order of the children's first pixels; there are at most twice as
// many chains as leaves, and at most as many leaves as pixels.
//
// Exact sums: every sum of fixed-point weights is an integer sum, kept as
// 64-bit sums of 32-bit limbs (a term T = sum_j L_j 2^(32 j), L_0..L_2 in
// [0, 2^32), L_3 = T >> 96) so that they can be added in any order, by any
// thread, and rebuilt exactly as a 128-bit integer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ipp {
namespace db {

constexpr int kMaxLevels = 64;      // nthresh: a power of two in [2, 64]

struct Chain {
  double F_top;              // intensity above its level of the top node
  int64_t nobj_sum;          // objects of the significant child chains
  int32_t parent;            // chain of the parent node (-1: the root)
  int32_t cnt;               // children at the level being built
  int32_t nsig;              // significant child chains
  int32_t one;               // a significant child chain (nsig == 1)
  int32_t nobj;              // objects this chain stands for
  int32_t mode;              // 0 the top node is the object, 1 children's
  int32_t bmode;             // 1 all significant children, 2 the one
  int32_t allsig;            // every node below the top is significant
  int32_t reached, objof;    // on the object path; object chain (or -1)
  int32_t slot;              // seed index of an object chain
  int32_t first;             // first pixel of an object chain's seed
};

// One seed / object.  m[s][j]: limb j of the seed sums S = sum d,
// Sx = sum d dx, Sy = sum d dy, Sxx = sum d dx^2, Syy = sum d dy^2 (dx, dy
// about the seed's corner); fin: limbs 0 and 1 of the final pixels' sum
// (d = hi 2^32 + lo, hi the signed part), nfin their count.
struct Obj {
  int64_t m[5][4];
  int64_t fin[2];
  int64_t nfin;
  double F, xc, yc, s2;
  int32_t xmin, ymin, first, target;
  int32_t final_obj, idx;    // object after merges; survivor number
};

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

// Per-candidate scratch in the pool; A = bounding-box pixels, m =
// candidate pixels.  par / ch serve boxes too large for the kernel's LDS;
// the per-root arrays (indexed by the root's raster rank at a level) serve
// levels with more roots than the LDS holds.
struct Pool {
  double* val;      // [A] v of members, -inf elsewhere
  int32_t* par;     // [A] union-find parent (also the seed marks)
  int32_t* ch;      // [A] chain of each pixel's node
  int32_t* asg;     // [A] out: object index of members, -1 elsewhere
  int64_t* accL;    // [A] per root: low limb sums
  int64_t* accH;    // [A] per root: high (signed) limb sums
  int32_t* accN;    // [A] per root: pixel counts
  int32_t* pch;     // [A] per root: the parent node's chain
  int32_t* nch;     // [A] per root: the root's chain at this level
  Chain* chains;    // [2 m + 2]
  Obj* objs;        // [m + 1]
  int32_t chain_cap, obj_cap;
};

__host__ __device__ inline size_t pool_bytes(int64_t A, int64_t m) {
  return 3 * align16(8 * (size_t)A) + 6 * align16(4 * (size_t)A) +
         align16(sizeof(Chain) * (size_t)(2 * m + 2)) +
         align16(sizeof(Obj) * (size_t)(m + 1));
}

__host__ __device__ inline Pool carve(char* b, int64_t A, int64_t m) {
  Pool s;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* r = b + o;
    o += align16(bytes);
    return r;
  };
  s.val = (double*)take(8 * (size_t)A);
  s.accL = (int64_t*)take(8 * (size_t)A);
  s.accH = (int64_t*)take(8 * (size_t)A);
  s.par = (int32_t*)take(4 * (size_t)A);
  s.ch = (int32_t*)take(4 * (size_t)A);
  s.asg = (int32_t*)take(4 * (size_t)A);
  s.accN = (int32_t*)take(4 * (size_t)A);
  s.pch = (int32_t*)take(4 * (size_t)A);
  s.nch = (int32_t*)take(4 * (size_t)A);
  s.chains = (Chain*)take(sizeof(Chain) * (size_t)(2 * m + 2));
  s.objs = (Obj*)take(sizeof(Obj) * (size_t)(m + 1));
  s.chain_cap = (int32_t)(2 * m + 2);
  s.obj_cap = (int32_t)(m + 1);
  return s;
}

// Correctly rounded (nearest, ties to even) binary64 value of an int128.
__host__ __device__ inline double to_f64(__int128 v) {
  const bool neg = v < 0;
  unsigned __int128 u = neg ? (unsigned __int128)0 - (unsigned __int128)v
                            : (unsigned __int128)v;
  if (u == 0) return 0.0;
  const uint64_t hi = (uint64_t)(u >> 64), lo = (uint64_t)u;
  const int top = hi ? 127 - __builtin_clzll(hi) : 63 - __builtin_clzll(lo);
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

// Fixed-point weight of a value: round(v 2^28), clamped to +-(2^62 - 1)
// (binary64 comparison with 2^62 is exact: see the source table).
__host__ __device__ inline int64_t fixed_d(double v) {
  const double s = rint(v * 268435456.0);
  const int64_t dmax = (int64_t)(((uint64_t)1 << 62) - 1);
  if (s >= 0x1p62) return dmax;
  if (s <= -0x1p62) return -dmax;
  return (int64_t)s;
}

// The 128-bit value of four limb sums (see the header).
__host__ __device__ inline __int128 from_limbs4(const int64_t* l) {
  return (__int128)l[0] + ((__int128)l[1] << 32) + ((__int128)l[2] << 64) +
         ((__int128)l[3] << 96);
}

// The 128-bit value of a low (unsigned 32-bit terms) and a high (signed)
// limb sum.
__host__ __device__ inline __int128 from_limbs2(int64_t lo, int64_t hi) {
  return (__int128)lo + ((__int128)hi << 32);
}

}  // namespace db
}  // namespace ipp
