// Multi-threshold deblending and cleaning of one detection candidate
// (Sec. 2.2.5: deblending and cleaning phases), one thread per candidate as
// in the paper's own GPU mapping of these phases.  Host and device code:
// the kernel runs it per candidate on the GPU; the same routine compiled
// for the host checks the algorithm against the oracle without a GPU.
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
// run of single-child nodes is kept as one chain record (its top node, its
// bottom node, their intensities).  Chains are created where a node has
// two or more children; there are at most twice as many chains as leaves,
// and at most as many leaves as pixels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ipp {
namespace db {

constexpr int kMaxLevels = 64;      // nthresh: a power of two in [2, 64]

struct Chain {
  double F_top, F_bot;       // intensity above level at the top / bottom
  int64_t nobj_sum;          // objects of the significant child chains
  int32_t parent;            // chain of the parent node (-1: the root)
  int32_t lev_top, lev_bot;  // levels of the top and bottom nodes
  int32_t cnt;               // children at the level being built
  int32_t nsig;              // significant child chains
  int32_t one;               // a significant child chain (nsig == 1)
  int32_t nobj;              // objects this chain stands for
  int32_t mode;              // 0 the top node is the object, 1 children's
  int32_t bmode;             // 1 all significant children, 2 the one
  int32_t allsig;            // every node below the top is significant
  int32_t reached, objof, slot;
};

struct Obj {
  __int128 S, Sx, Sy, Sxx, Syy;      // exact seed sums (about seed corner)
  __int128 Sfin;                     // exact sum over the final pixels
  double F, xc, yc, s2;
  int64_t nfin;
  int32_t xmin, ymin, first, target;
};

// Per-candidate scratch; A = bounding-box pixels, m = candidate pixels.
struct Scratch {
  __int128* accS;   // [A]
  Obj* objs;        // [m + 1]
  Chain* chains;    // [2 m + 2]
  double* val;      // [A] v of members, -inf elsewhere (filled by caller)
  int32_t* par;     // [A]
  int32_t* ch;      // [A]
  int32_t* accN;    // [A]
  int32_t* roots;   // [A]
  int32_t* asg;     // [A] out: object index of members, -1 elsewhere
  int32_t chain_cap, obj_cap;
};

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

// Bytes of scratch for a bounding box of A pixels holding m candidate
// pixels, and the carving of a block of that size.
__host__ __device__ inline size_t scratch_bytes(int64_t A, int64_t m) {
  return align16(16 * (size_t)A) + align16(sizeof(Obj) * (size_t)(m + 1)) +
         align16(sizeof(Chain) * (size_t)(2 * m + 2)) +
         align16(8 * (size_t)A) + 5 * align16(4 * (size_t)A);
}

__host__ __device__ inline Scratch carve(char* b, int64_t A, int64_t m) {
  Scratch s;
  size_t o = 0;
  s.accS = (__int128*)(b + o);
  o += align16(16 * (size_t)A);
  s.objs = (Obj*)(b + o);
  o += align16(sizeof(Obj) * (size_t)(m + 1));
  s.chains = (Chain*)(b + o);
  o += align16(sizeof(Chain) * (size_t)(2 * m + 2));
  s.val = (double*)(b + o);
  o += align16(8 * (size_t)A);
  int32_t** ints[] = {&s.par, &s.ch, &s.accN, &s.roots, &s.asg};
  for (auto p : ints) {
    *p = (int32_t*)(b + o);
    o += align16(4 * (size_t)A);
  }
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

__host__ __device__ inline int uf_find(int32_t* par, int p) {
  while (par[p] != p) {
    par[p] = par[par[p]];
    p = par[p];
  }
  return p;
}

// Union linking the larger root to the smaller: a set's root is its
// smallest index, i.e. its first pixel in raster order.
__host__ __device__ inline void uf_union(int32_t* par, int a, int b) {
  a = uf_find(par, a);
  b = uf_find(par, b);
  if (a < b) par[b] = a;
  else if (b < a) par[a] = b;
}

struct Cand {
  int32_t bw, bh, x0, y0;   // bounding box
  int32_t npix;
  double t0, peak;
  int32_t conn, nthresh, clean;
  double mincont, kc;
};

// Deblends one candidate whose member values are in s.val.  Returns the
// number of objects (>= 1) with s.asg set for every member, or -1 when the
// chain or object records would exceed the scratch (not reachable with the
// bounds of scratch_bytes).
__host__ __device__ inline int deblend_one(const Cand& c, Scratch& s) {
  const int A = c.bw * c.bh;
  const double two_m28 = 0x1p-28;
  const double ninf = -__builtin_inf();          // value of non-members
  for (int p = 0; p < A; ++p) s.asg[p] = s.val[p] != ninf ? 0 : -1;
  if (!(c.t0 > 0.0) || c.npix < 2 || !(c.peak > c.t0)) return 1;

  // levels
  double lev[kMaxLevels];
  double q = c.peak / c.t0;
  for (int k = c.nthresh; k > 1; k >>= 1) q = sqrt(q);
  {
    double t = c.t0;
    for (int i = 1; i < c.nthresh; ++i) {
      t = t * q;
      lev[i] = t;
    }
  }
  // the candidate's flux and the contrast bound
  __int128 Sroot = 0;
  for (int p = 0; p < A; ++p)
    if (s.asg[p] == 0) Sroot += fixed_d(s.val[p]);
  const double froot = to_f64(Sroot) * two_m28;
  const double fmin = c.mincont * froot;

  // root chain
  int nch = 1;
  {
    Chain& r = s.chains[0];
    r.F_top = r.F_bot = froot;
    r.nobj_sum = 0;
    r.parent = -1;
    r.lev_top = r.lev_bot = 0;
    r.cnt = r.nsig = 0;
    r.one = -1;
    r.nobj = 1;
    r.mode = r.bmode = 0;
    r.allsig = 1;
    r.reached = 0;
    r.objof = -1;
    r.slot = -1;
  }
  for (int p = 0; p < A; ++p) s.ch[p] = 0;

  // levels upward: components, their intensities, chain records
  for (int i = 1; i < c.nthresh; ++i) {
    const double t = lev[i];
    int any = 0;
    for (int p = 0; p < A; ++p) {
      const bool up = s.val[p] > t;
      s.par[p] = up ? p : -1;
      any |= up;
    }
    if (!any) break;
    for (int y = 0; y < c.bh; ++y) {
      for (int x = 0; x < c.bw; ++x) {
        const int p = y * c.bw + x;
        if (s.par[p] < 0) continue;
        if (x > 0 && s.par[p - 1] >= 0) uf_union(s.par, p, p - 1);
        if (y > 0) {
          const int u = p - c.bw;
          if (s.par[u] >= 0) uf_union(s.par, p, u);
          if (c.conn == 8) {
            if (x > 0 && s.par[u - 1] >= 0) uf_union(s.par, p, u - 1);
            if (x + 1 < c.bw && s.par[u + 1] >= 0) uf_union(s.par, p, u + 1);
          }
        }
      }
    }
    int nroots = 0;
    for (int p = 0; p < A; ++p) {
      if (s.par[p] < 0) continue;
      const int r = uf_find(s.par, p);
      if (r == p) {                  // the root is the first pixel
        s.roots[nroots++] = p;
        s.accS[p] = 0;
        s.accN[p] = 0;
      }
      s.accS[r] += fixed_d(s.val[p]);
      s.accN[r] += 1;
    }
    for (int k = 0; k < nroots; ++k) s.chains[s.ch[s.roots[k]]].cnt = 0;
    for (int k = 0; k < nroots; ++k) s.chains[s.ch[s.roots[k]]].cnt += 1;
    for (int k = 0; k < nroots; ++k) {
      const int r = s.roots[k];
      const int pc = s.ch[r];
      const double F = to_f64(s.accS[r]) * two_m28 - (double)s.accN[r] * t;
      int nc = pc;
      if (s.chains[pc].cnt == 1) {   // the chain goes on
        s.chains[pc].lev_bot = i;
        s.chains[pc].F_bot = F;
        s.chains[pc].allsig &= F > fmin ? 1 : 0;
      } else {                       // a branch: a chain per child
        if (nch >= s.chain_cap) return -1;
        nc = nch++;
        Chain& ch = s.chains[nc];
        ch.F_top = ch.F_bot = F;
        ch.nobj_sum = 0;
        ch.parent = pc;
        ch.lev_top = ch.lev_bot = i;
        ch.cnt = ch.nsig = 0;
        ch.one = -1;
        ch.nobj = 1;
        ch.mode = ch.bmode = 0;
        ch.allsig = 1;
        ch.reached = 0;
        ch.objof = -1;
        ch.slot = -1;
      }
      s.accN[r] = nc;               // the root's chain at this level
    }
    for (int p = 0; p < A; ++p)
      if (s.par[p] >= 0) s.ch[p] = s.accN[uf_find(s.par, p)];
  }

  // pruning, children before parents (they were created later)
  for (int k = nch - 1; k >= 0; --k) {
    Chain& C = s.chains[k];
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
    // the chain's top stands for its bottom's objects only if every node
    // between passes them up (each significant)
    if (bmode != 0 && C.allsig) {
      C.mode = 1;
      C.nobj = (int32_t)nb;
    } else {
      C.mode = 0;
      C.nobj = 1;
    }
    if (C.parent >= 0 && C.F_top > fmin) {
      Chain& P = s.chains[C.parent];
      P.nsig += 1;
      P.nobj_sum += C.nobj;
      P.one = k;
    }
  }
  if (s.chains[0].nobj < 2) return 1;

  // objects, parents before children
  int K = 0;
  for (int k = 0; k < nch; ++k) {
    Chain& C = s.chains[k];
    if (k == 0) {
      C.reached = 1;
    } else {
      const Chain& P = s.chains[C.parent];
      C.reached = P.reached && P.mode == 1 &&
                  ((P.bmode == 1 && C.F_top > fmin) ||
                   (P.bmode == 2 && P.one == k));
    }
    const bool obj = C.reached && C.mode == 0;
    C.objof = obj ? k : (k > 0 ? s.chains[C.parent].objof : -1);
    C.slot = -1;
  }
  // seeds: object slots in raster order of their first pixels
  for (int p = 0; p < A; ++p) {
    if (s.asg[p] < 0) continue;
    const int o = s.chains[s.ch[p]].objof;
    if (o < 0) {
      s.asg[p] = -2;                 // not in a seed
      continue;
    }
    Chain& C = s.chains[o];
    if (C.slot < 0) {
      if (K >= s.obj_cap) return -1;
      C.slot = K;
      Obj& b = s.objs[K++];
      b.S = b.Sx = b.Sy = b.Sxx = b.Syy = b.Sfin = 0;
      b.nfin = 0;
      b.first = p;
      b.xmin = p % c.bw;
      b.ymin = p / c.bw;
      b.target = -1;
    }
    Obj& b = s.objs[C.slot];
    const int x = p % c.bw;
    if (x < b.xmin) b.xmin = x;
    s.asg[p] = C.slot;
  }
  // seed moments about each seed's corner, and the models
  for (int p = 0; p < A; ++p) {
    const int k = s.asg[p];
    if (k < 0) continue;
    Obj& b = s.objs[k];
    const int64_t d = fixed_d(s.val[p]);
    const int64_t dx = p % c.bw - b.xmin, dy = p / c.bw - b.ymin;
    b.S += d;
    b.Sx += (__int128)d * dx;
    b.Sy += (__int128)d * dy;
    b.Sxx += (__int128)d * (dx * dx);
    b.Syy += (__int128)d * (dy * dy);
  }
  for (int k = 0; k < K; ++k) {
    Obj& b = s.objs[k];
    const double fS = to_f64(b.S);
    const double mx = to_f64(b.Sx) / fS;
    const double my = to_f64(b.Sy) / fS;
    const double x2 = to_f64(b.Sxx) / fS - mx * mx;
    const double y2 = to_f64(b.Syy) / fS - my * my;
    b.F = fS * two_m28;
    b.xc = (double)(c.x0 + b.xmin) + mx;
    b.yc = (double)(c.y0 + b.ymin) + my;
    b.s2 = (x2 + y2) + 1.0 / 6.0;
  }
  // the other pixels: the brightest model
  for (int p = 0; p < A; ++p) {
    if (s.asg[p] != -2) continue;
    const double x = (double)(c.x0 + p % c.bw);
    const double y = (double)(c.y0 + p / c.bw);
    double best = -1.0;
    int bk = 0;
    for (int k = 0; k < K; ++k) {
      const Obj& b = s.objs[k];
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
  if (!c.clean) return K;

  // cleaning
  for (int p = 0; p < A; ++p) {
    const int k = s.asg[p];
    if (k < 0) continue;
    s.objs[k].Sfin += fixed_d(s.val[p]);
    s.objs[k].nfin += 1;
  }
  const double pi = 3.14159265358979311600;   // binary64 nearest to pi
  for (int o = 0; o < K; ++o) {
    Obj& b = s.objs[o];
    const double mu = to_f64(b.Sfin) * two_m28 / (double)b.nfin;
    double tot = 0.0, best = -1.0;
    int bm = -1;
    for (int m = 0; m < K; ++m) {
      if (m == o) continue;
      const Obj& n = s.objs[m];
      const bool brighter = n.F > b.F || (n.F == b.F && m < o);
      if (!brighter) continue;
      const double dx = b.xc - n.xc;
      const double dy = b.yc - n.yc;
      const double d2 = dx * dx + dy * dy;
      double den = n.s2 + d2;
      den = den * den;
      den = pi * den;
      const double cm = c.kc * ((n.F * n.s2) / den);
      tot += cm;
      if (cm > best) {
        best = cm;
        bm = m;
      }
    }
    b.target = (bm >= 0 && mu - tot < c.t0) ? bm : o;
  }
  // follow merges to an object that stays; number the survivors in order
  int nk = 0;
  for (int o = 0; o < K; ++o) {
    int k = o;
    while (s.objs[k].target != k) k = s.objs[k].target;
    s.objs[o].first = k;             // final object (reuses the field)
  }
  for (int o = 0; o < K; ++o)
    s.objs[o].xmin = s.objs[o].first == o ? nk++ : -1;  // survivor index
  for (int p = 0; p < A; ++p) {
    const int k = s.asg[p];
    if (k >= 0) s.asg[p] = s.objs[s.objs[k].first].xmin;
  }
  return nk;
}

}  // namespace db
}  // namespace ipp
