// Aperture photometry with a local sky annulus (Sec. 2.2.5: per-object
// aperture photometry).
//
// One wavefront per source, four sources per workgroup, no workgroup
// barriers.  The wave classifies every pixel of the source's window with
// the exact membership predicates (cheap), accumulates the aperture pixels
// that lie wholly inside the aperture, and compacts the rest of the work
// into its LDS slice: the aperture pixels cut by the circle, the annulus
// values with their weights, and the annulus pixels cut by either circle.
// The exact overlap areas (binary64; one atan2 per circle and pixel) are then
// computed over those dense task lists with every lane busy.  The annulus
// (value, weight) pairs are sorted in registers with a bitonic network;
// the k-sigma clipping of the sky works on contiguous ranges of the sorted
// values and the weighted sky sum is a sum over the final range.
#include <type_traits>

#include "ipp_internal.h"
#include "kernels.h"
#include "phot_geom.h"

namespace ipp {

namespace {

constexpr int kApTasks = 320;   // aperture pixels cut by a circle, r <= 16
constexpr int kEdges = 36;      // pixel edges per axis of a window, r <= 16

template <int NS>
struct ApLds {
  double pv[NS];                // annulus values
  double pw[NS];                // annulus weights
  // exact-overlap tasks: kind << 28 | annulus slot << 12 | wy << 6 | wx
  // (kind 0: cut by the aperture; 1: cut by the outer circle only; 2: by
  // the inner circle only; 3: by both)
  // the task list is consumed before the annulus values are sorted; the
  // sort's transposes and the sorted values then use the same space
  union {
    struct {
      int tk[NS + kApTasks];
      // square roots at the window's column and row edges for the
      // aperture, outer and inner circle: [circle][axis][edge]
      double sq[3 * 2 * kEdges];
    };
    double xs[NS + kWave];
  };
};

__device__ __forceinline__ void wave_lds_sync() {
  // wavefront scope: the wave's own LDS operations are performed in
  // order, so these order the code without waiting on memory
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


// ---- bitonic sort of the annulus values -------------------------------
// NS = 2^(P+6) binary64 values, 2^P per lane.  In layout S a lane's
// registers hold the elements whose index bits [S, S+P) give the register
// number, and the lane number supplies the other six bits (layout 0:
// e = lane * 2^P + k).  Every compare-exchange of the network is then
// between two registers of one lane; the network changes layout through
// LDS, one write and one read per register.  Blocks that the network sorts
// in descending order are negated for the length of their merge, so that
// every compare-exchange is ascending.

// v_min_f64 / v_max_f64 as single instructions: the values are never NaN,
// so the canonicalising moves the compiler adds around fmin/fmax are not
// needed.
__device__ __forceinline__ double min64(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}
__device__ __forceinline__ double max64(double a, double b) {
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// Element index of register 0 of this lane in layout S.
template <int P, int S>
__device__ __forceinline__ int lay_base(int lane) {
  return (lane & ((1 << S) - 1)) | ((lane >> S) << (S + P));
}

// LDS address of element e in a transpose from layout A to layout B:
// e + MUL * (e >> Q).  The element index is a disjoint sum of a lane part
// and a register part, so the address is a per-lane base plus a constant
// per register (an instruction offset).  Q and MUL are chosen so that the
// 32 lanes of a half-wave meet 32 different 8-byte bank slots on both
// sides of every transpose the network uses (at worst two lanes share
// one); every address is below NS + 64.
template <int P, int A, int B>
struct SortPad {
  static constexpr int S = A + B;          // the other layout, if one is 0
  static constexpr bool Z = A == 0 || B == 0;
  static constexpr int Q =
      Z ? (S <= P ? P : (S >= 5 ? 5 : (P == 2 && S == 3 ? 3 : 6)))
        : (B == 1 ? P + 1 : (P == 2 && B == 3 ? 4 : 5));
  static constexpr int MUL = Z ? 1 : 2;
  static __device__ __forceinline__ int at(int e) { return e + MUL * (e >> Q); }
};

template <int P, int A, int B>
__device__ __forceinline__ void relayout(double (&v)[1 << P], double* xs,
                                         int lane) {
  using Pad = SortPad<P, A, B>;
  const int wb = Pad::at(lay_base<P, A>(lane));
  const int rb = Pad::at(lay_base<P, B>(lane));
#pragma unroll
  for (int k = 0; k < (1 << P); ++k) xs[wb + Pad::at(k << A)] = v[k];
  wave_lds_sync();
#pragma unroll
  for (int k = 0; k < (1 << P); ++k) v[k] = xs[rb + Pad::at(k << B)];
  wave_lds_sync();
}

// Negate the elements whose index bit M is set (layout S).
template <int P, int M, int S>
__device__ __forceinline__ void negate_bit(double (&v)[1 << P], int lane) {
  if constexpr (M >= S && M < S + P) {
#pragma unroll
    for (int k = 0; k < (1 << P); ++k)
      if (k & (1 << (M - S))) v[k] = -v[k];
  } else {
    constexpr int LB = M < S ? M : M - P;   // the lane bit holding bit M
    const int sg = ((lane >> LB) & 1) << 31;
#pragma unroll
    for (int k = 0; k < (1 << P); ++k)
      v[k] = __hiloint2double(__double2hiint(v[k]) ^ sg, __double2loint(v[k]));
  }
}

// Ascending compare-exchange of registers k and k + 2^B (bit B of k clear).
template <int P, int B>
__device__ __forceinline__ void cx_regs(double (&v)[1 << P]) {
#pragma unroll
  for (int k = 0; k < (1 << P); ++k) {
    if (!(k & (1 << B))) {
      const int l = k | (1 << B);
      const double a = v[k], b = v[l];
      v[k] = min64(a, b);
      v[l] = max64(a, b);
    }
  }
}

template <int P, int M, int S>
__device__ __forceinline__ void bitonic_merge_from(double (&v)[1 << P],
                                                   double* xs, int lane);

// Stages J, J-1, .., 0 of the merge of blocks of 2^M elements, entered in
// layout S; a stage on bit J outside the layout's register bits first
// moves to the layout whose register bits end at J.
template <int P, int M, int J, int S>
__device__ __forceinline__ void bitonic_stages(double (&v)[1 << P],
                                               double* xs, int lane) {
  constexpr int N = P + 6;
  if constexpr (J < 0) {
    if constexpr (M < N) negate_bit<P, M, S>(v, lane);
    bitonic_merge_from<P, M + 1, S>(v, xs, lane);
  } else if constexpr (J >= S && J < S + P) {
    cx_regs<P, J - S>(v);
    bitonic_stages<P, M, J - 1, S>(v, xs, lane);
  } else {
    constexpr int S2 = J - P + 1 > 0 ? J - P + 1 : 0;
    relayout<P, S, S2>(v, xs, lane);
    cx_regs<P, J - S2>(v);
    bitonic_stages<P, M, J - 1, S2>(v, xs, lane);
  }
}

template <int P, int M, int S>
__device__ __forceinline__ void bitonic_merge_from(double (&v)[1 << P],
                                                   double* xs, int lane) {
  constexpr int N = P + 6;
  if constexpr (M <= N) {
    // blocks with bit M set are sorted descending (the last merge, M = N,
    // sorts the whole array ascending)
    if constexpr (M < N) negate_bit<P, M, S>(v, lane);
    bitonic_stages<P, M, M - 1, S>(v, xs, lane);
  } else {
    static_assert(S == 0, "the network ends in layout 0");
  }
}

// Ascending sort of v (layout 0); the sorted array is also left in xs at
// sorted_addr(e), for wave-uniform reads.
template <int P>
__device__ __forceinline__ void wave_sort(double (&v)[1 << P], double* xs,
                                          int lane) {
  bitonic_merge_from<P, 1, 0>(v, xs, lane);
#pragma unroll
  for (int k = 0; k < (1 << P); ++k) {
    const int e = (lane << P) | k;
    xs[e + (e >> P)] = v[k];
  }
  wave_lds_sync();
}

template <int P>
__device__ __forceinline__ double sorted_at(const double* xs, int e) {
  return xs[e + (e >> P)];
}

template <int NS>
__device__ void aperture_one(const Work& wk, const ipp_params& p,
                             ipp_sources& src, double* sky_lohi,
                             long long row, ApLds<NS>& L,
                             const double* atan_lds) {
  constexpr int PL = NS / kWave;
  constexpr int P = PL == 4 ? 2 : (PL == 8 ? 3 : 4);
  static_assert((1 << P) == PL, "NS is 256, 512 or 1024");
  const int lane = threadIdx.x & (kWave - 1);
  const int f = src.frame[row];
  const double cx = src.x[row], cy = src.y[row];
  const bool fok = f >= 0 && f < wk.nframes;
  const double R = p.r_ap > p.r_out ? p.r_ap : p.r_out;
  if (!fok || !(isfinite(cx) && isfinite(cy)) || fabs(cx) > 1e9 ||
      fabs(cy) > 1e9) {
    if (lane == 0) {
      src.flux_ap[row] = __builtin_nan("");
      src.sky[row] = __builtin_nan("");
      src.area_ap[row] = 0.0;
      src.area_ann[row] = 0.0;
      src.flags[row] |= IPP_SRC_APERTURE_OFF_EDGE | IPP_SRC_NO_SKY;
      if (sky_lohi) { sky_lohi[2 * row] = 0.0; sky_lohi[2 * row + 1] = -1.0; }
    }
    return;
  }
  const FrameDev fr = wk.frames[f];     // f is wave-uniform: SGPRs
  // window bounds: wave-uniform values, kept in scalar registers
  const int xa = __builtin_amdgcn_readfirstlane((int)ceil(cx - R - 0.5));
  const int xb = __builtin_amdgcn_readfirstlane((int)floor(cx + R + 0.5));
  const int ya = __builtin_amdgcn_readfirstlane((int)ceil(cy - R - 0.5));
  const int yb = __builtin_amdgcn_readfirstlane((int)floor(cy + R + 0.5));
  const int nwx = xb - xa + 1, npx = nwx * (yb - ya + 1);

  // ---- classify the window; compact the work -------------------------
  // Per pixel: the exact membership predicates, the value I - B and a place
  // in one of the compacted lists.  The count of pixels wholly inside the
  // aperture and the off-edge flags are wave-uniform (ballots).
  uint32_t flags = 0;                  // wave-uniform
  int nfull = 0;                       // pixels wholly inside the aperture
  double a_ap = 0.0, raw = 0.0;
  int nann = 0, ntk = 0;
  // squared radii as the membership predicates form them
  const double ra2 = p.r_ap * p.r_ap, ri2 = p.r_in * p.r_in;
  const double ro2 = p.r_out * p.r_out;
  const int dwr = kWave / nwx, dwc = kWave - (kWave / nwx) * nwx;
  // Row base of the window's first in-frame row (wave-uniform); loads take
  // 32-bit byte offsets from it (pitch <= 2^24, at most 35 rows).
  const int ry0 = min(max(ya, 0), fr.h - 1);
  const char* wpix =
      uniform_ptr((const char*)(fr.pix + (int64_t)ry0 * fr.pitch));
  const char* wbkg = uniform_ptr((const char*)(fr.bkg + (int64_t)ry0 * fr.w));
  const uint32_t pitchB = (uint32_t)fr.pitch * 4u, wB = (uint32_t)fr.w * 4u;
  // A window wholly inside the frame needs neither clamping nor an inside
  // test: its offsets advance by constant steps.
  const bool interior = xa >= 0 && ya >= 0 && xb < fr.w && yb < fr.h;

  // Squared nearest and farthest offsets of every window column and row
  // from the centre (the pixel's distances are sums of one of each: the
  // same two rounded squares and the same addition as computing them per
  // pixel).  They occupy the edge-root table, which is filled only after
  // the classification.
  double2* colT = (double2*)L.sq;              // [kEdges]
  double2* rowT = colT + kEdges;               // [kEdges]
  for (int e = lane; e < 2 * kEdges; e += kWave) {
    const bool col = e < kEdges;
    const int j = col ? e : e - kEdges;
    const double a = col ? fabs((double)(xa + j) - cx)
                         : fabs((double)(ya + j) - cy);
    const double n = fmax(a - 0.5, 0.0), fo = a + 0.5;
    double2 t;
    t.x = n * n;
    t.y = fo * fo;
    (col ? colT : rowT)[j] = t;
  }
  wave_lds_sync();

  auto classify = [&](auto edge_tag) {
    constexpr bool EDGE = decltype(edge_tag)::value;
    int wr = lane / nwx, wc = lane - (lane / nwx) * nwx;  // window row, col
    uint32_t offp = (uint32_t)wr * pitchB + (uint32_t)(xa + wc) * 4u;
    uint32_t offb = (uint32_t)wr * wB + (uint32_t)(xa + wc) * 4u;
    const uint32_t stepP = (uint32_t)dwr * pitchB + (uint32_t)dwc * 4u;
    const uint32_t stepB = (uint32_t)dwr * wB + (uint32_t)dwc * 4u;
    const uint32_t wrapP = pitchB - (uint32_t)nwx * 4u;
    const uint32_t wrapB = wB - (uint32_t)nwx * 4u;
    // Chunks of kChunk rounds of 64 pixels: all loads of a chunk are issued
    // before any is used, so their latencies overlap.
    constexpr int kChunk = 8;
    for (int e0 = 0; e0 < npx; e0 += kChunk * kWave) {
      float Iv[kChunk], Bv[kChunk];
      uint32_t st[kChunk];
      int pos[kChunk];
#pragma unroll
      for (int c = 0; c < kChunk; ++c) {
        if (e0 + c * kWave >= npx) break;            // wave-uniform
        const int e = e0 + c * kWave + lane;
        const int px = xa + wc, py = ya + wr;
        const bool live = e < npx;
        pos[c] = (wr << 6) | wc;
        // nearest and farthest point of the pixel square (touches / within)
        // (a lane past the window end reads a valid row of the table)
        const double2 tc = colT[wc], tr = rowT[min(wr, kEdges - 1)];
        const double near2 = tc.x + tr.x, far2 = tc.y + tr.y;
        // (bitwise logic: no branches)
        const bool in_ap = live & (near2 < ra2);
        const bool in_ann = live & (near2 < ro2) & !(far2 <= ri2);
        bool inside = true;
        if constexpr (EDGE) {
          // loads clamped into the frame: every lane loads, no branches
          inside = (px >= 0) & (px < fr.w) & (py >= 0) & (py < fr.h);
          const uint32_t qx = (uint32_t)min(max(px, 0), fr.w - 1);
          const uint32_t qr = (uint32_t)(min(max(py, 0), fr.h - 1) - ry0);
          Iv[c] = gld((const float*)(wpix + (qr * pitchB + qx * 4u)));
          Bv[c] = gld((const float*)(wbkg + (qr * wB + qx * 4u)));
        } else {
          // a lane past the window end loads the window's first pixel
          Iv[c] = gld((const float*)(wpix + (live ? offp : 0u)));
          Bv[c] = gld((const float*)(wbkg + (live ? offb : 0u)));
        }
        st[c] = (uint32_t)in_ap | ((uint32_t)in_ann << 1) |
                ((uint32_t)inside << 2) | ((uint32_t)(far2 <= ra2) << 3) |
                ((uint32_t)!(far2 <= ro2) << 4) |
                ((uint32_t)(near2 < ri2) << 5);
        wr += dwr;
        wc += dwc;
        offp += stepP;
        offb += stepB;
        if (wc >= nwx) {
          wc -= nwx;
          ++wr;
          offp += wrapP;
          offb += wrapB;
        }
      }
#pragma unroll
      for (int c = 0; c < kChunk; ++c) {
        if (e0 + c * kWave >= npx) break;            // wave-uniform
        const bool in_ap = st[c] & 1u, in_ann = st[c] & 2u;
        const bool ok = ((st[c] & 4u) != 0) & isfinite(Iv[c]);
        const double v = (double)Iv[c] - (double)Bv[c];
        if (ballot(in_ap & !ok)) flags |= IPP_SRC_APERTURE_OFF_EDGE;
        if (ballot(in_ann & !ok)) flags |= IPP_SRC_ANNULUS_OFF_EDGE;
        const bool whole = (st[c] & 8u) != 0;
        const bool full = in_ap & ok & whole;
        const bool ap_cut = in_ap & ok & !whole;
        const bool ann = in_ann & ok;
        const bool ann_cut = ann & ((st[c] & 48u) != 0);
        nfull += __popcll(ballot(full));
        if (full) raw += v;
        const uint64_t b1 = ballot(ap_cut);
        if (ap_cut) {
          const int s = ntk + lanes_before(b1);
          if (s < NS + kApTasks) L.tk[s] = pos[c];
        }
        ntk += __popcll(b1);
        const uint64_t b2 = ballot(ann);
        int slot = 0;
        if (ann) {
          slot = nann + lanes_before(b2);
          if (slot < NS) {
            L.pv[slot] = v;
            L.pw[slot] = 1.0;
          }
        }
        nann += __popcll(b2);
        const uint64_t b3 = ballot(ann_cut);
        if (ann_cut) {
          const int s = ntk + lanes_before(b3);
          const int kind = (int)((st[c] >> 4) & 3u);
          if (s < NS + kApTasks && slot < NS)
            L.tk[s] = (kind << 28) | (slot << 12) | pos[c];
        }
        ntk += __popcll(b3);
      }
    }
  };
  if (interior) classify(std::false_type{});
  else classify(std::true_type{});
  if (nann > NS) nann = NS;            // not reachable: NS bounds the ring
  if (ntk > NS + kApTasks) ntk = NS + kApTasks;  // not reachable either
  wave_lds_sync();

  // ---- exact overlaps over one dense task list ---------------------------
  // Every lane computes one overlap per task (two only for a pixel cut by
  // both annulus circles), whatever circle the task belongs to.
  // The square roots depend on one pixel edge and one circle each: they
  // are taken once per window edge (the window spans at most 34 pixels).
  {
    const double r2a = p.r_ap * p.r_ap, r2o = p.r_out * p.r_out;
    const double r2i = p.r_in * p.r_in;
    for (int e = lane; e < 6 * kEdges; e += kWave) {
      const int c = e / (2 * kEdges), j = e % kEdges;
      const bool col = (e / kEdges) % 2 == 0;
      const double r = c == 0 ? p.r_ap : (c == 1 ? p.r_out : p.r_in);
      const double r2 = c == 0 ? r2a : (c == 1 ? r2o : r2i);
      const double q = col ? ((double)(xa + j) - 0.5) - cx
                           : ((double)(ya + j) - 0.5) - cy;
      L.sq[e] = edge_root(q, r, r2);
    }
  }
  wave_lds_sync();
  {
    const double r2a = p.r_ap * p.r_ap, r2o = p.r_out * p.r_out;
    const double r2i = p.r_in * p.r_in;
    // overlap of a task pixel with circle c (0 aperture, 1 outer, 2 inner)
    auto overlap_c = [&](int c, double r, double r2, int wx, int wy,
                         const double* coef) {
      const int px = xa + wx, py = ya + wy;
      if (!touches(cx, cy, r, px, py)) return 0.0;
      if (within(cx, cy, r, px, py)) return 1.0;
      const double* sq = L.sq + c * 2 * kEdges;
      return overlap_cut(cx, cy, r, r2, px, py, sq[wx], sq[wx + 1],
                         sq[kEdges + wy], sq[kEdges + wy + 1], coef);
    };
    for (int j = lane; j < ntk; j += kWave) {
      // the series coefficients are read where they are used (an offset the
      // compiler cannot hoist keeps them out of registers across the loop)
      int co = 0;
      asm volatile("" : "+s"(co));
      const double* coef = atan_lds + co;
      const int t = L.tk[j];
      const int kind = t >> 28, slot = (t >> 12) & 0x3FF;
      const int wx = t & 63, wy = (t >> 6) & 63;
      const int px = xa + wx, py = ya + wy;
      const int c = kind == 0 ? 0 : (kind == 2 ? 2 : 1);
      const double r = kind == 0 ? p.r_ap : (kind == 2 ? p.r_in : p.r_out);
      const double r2 = kind == 0 ? r2a : (kind == 2 ? r2i : r2o);
      double w = overlap_c(c, r, r2, wx, wy, coef);
      if (kind == 0) {
        // only the aperture needs the value here (annulus values are in
        // the value list already)
        const uint32_t qr = (uint32_t)(py - ry0);
        const float I =
            gld((const float*)(wpix + (qr * pitchB + (uint32_t)px * 4u)));
        const double v =
            (double)I -
            (double)gld((const float*)(wbkg + (qr * wB + (uint32_t)px * 4u)));
        a_ap += w;
        raw += w * v;
      } else {
        if (kind == 3) w -= overlap_c(2, p.r_in, r2i, wx, wy, coef);
        else if (kind == 2) w = 1.0 - w;
        L.pw[slot] = w;
      }
    }
  }
  wave_lds_sync();

  // ---- sort the annulus values ------------------------------------------
  double sv[PL];
#pragma unroll
  for (int k = 0; k < PL; ++k) {
    const int e = lane * PL + k;
    sv[k] = e < nann ? L.pv[e] : __builtin_inf();
  }
  wave_sort<P>(sv, L.xs, lane);

  // ---- k-sigma clipping on the sorted range [a, bnd) ---------------------
  // Running sums of (v - c) and (v - c)^2 over the range, c a fixed shift
  // (the first median); each pass removes a prefix and a suffix of the
  // range, whose sizes are ballot counts over the sorted values (the +inf
  // padding counts as above every bound).
  const double c0 = nann > 0 ? sorted_at<P>(L.xs, (nann - 1) / 2) : 0.0;
  double S1 = 0.0, S2 = 0.0;
#pragma unroll
  for (int k = 0; k < PL; ++k) {
    const int e = lane * PL + k;
    const double d = e < nann ? sv[k] - c0 : 0.0;
    S1 += d;
    S2 += d * d;
  }
  S1 = wave_sum(S1);
  S2 = wave_sum(S2);
  int a = 0, bnd = nann;
  for (int it = 0; it < p.sky_clip_iters; ++it) {
    const int n = bnd - a;
    if (n == 0) break;
    const double med =
        (n & 1) ? sorted_at<P>(L.xs, a + (n - 1) / 2)
                : (sorted_at<P>(L.xs, a + n / 2 - 1) +
                   sorted_at<P>(L.xs, a + n / 2)) / 2.0;
    const double dm = S1 / (double)n;
    const double var = S2 / (double)n - dm * dm;
    const double sd = sqrt(var > 0.0 ? var : 0.0);
    const double lo = med - p.sky_clip_sigma * sd;
    const double hi = med + p.sky_clip_sigma * sd;
    int nlo = 0, nhi = 0;
#pragma unroll
    for (int k = 0; k < PL; ++k) {
      nlo += __popcll(ballot(sv[k] < lo));
      nhi += __popcll(ballot(sv[k] > hi));
    }
    const int cl = max(nlo - a, 0), ch = max(nhi - (NS - bnd), 0);
    if (cl == 0 && ch == 0) break;
    double r1 = 0.0, r2 = 0.0;
#pragma unroll
    for (int k = 0; k < PL; ++k) {
      const int e = lane * PL + k;
      const bool gone = (e >= a && e < a + cl) || (e >= bnd - ch && e < bnd);
      const double d = gone ? sv[k] - c0 : 0.0;
      r1 += d;
      r2 += d * d;
    }
    S1 -= wave_sum(r1);
    S2 -= wave_sum(r2);
    a += cl;
    bnd -= ch;
  }
  // the survivors are the values in [vlo, vhi] (clipping is by value)
  double vlo = 0.0, vhi = -1.0;
  if (bnd > a) { vlo = sorted_at<P>(L.xs, a); vhi = sorted_at<P>(L.xs, bnd - 1); }
  double num = 0.0, den = 0.0;
  for (int j = lane; j < nann; j += kWave) {
    const double v = L.pv[j], w = L.pw[j];
    if (v >= vlo && v <= vhi) {
      num += w * v;
      den += w;
    }
  }
  num = wave_sum(num);
  den = wave_sum(den);
  a_ap = (double)nfull + wave_sum(a_ap);
  raw = wave_sum(raw);
  if (lane == 0) {
    double sky = 0.0;
    if (den > 0.0) sky = num / den; else flags |= IPP_SRC_NO_SKY;
    src.flux_ap[row] = raw - sky * a_ap;
    src.sky[row] = sky;
    src.area_ap[row] = a_ap;
    src.area_ann[row] = den;
    src.flags[row] |= flags;
    if (sky_lohi) { sky_lohi[2 * row] = vlo; sky_lohi[2 * row + 1] = vhi; }
  }
  wave_lds_sync();                     // the slice is reused by the next row
}

}  // namespace

// NS: sort size (>= the annulus pixel count bound).
template <int NS>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(NS <= 512 ? 3 : 1))) void k_aperture_t(
    Work wk, ipp_params p,
                                                       ipp_sources src,
                                                       double* sky_lohi) {
  __shared__ ApLds<NS> L[kWaves];
  __shared__ double atan_lds[kAtanTerms];
  if (threadIdx.x < kAtanTerms) atan_lds[threadIdx.x] = atan_coef(threadIdx.x);
  __syncthreads();
  long long nrows = src.capacity;
  if (src.n_total && *src.n_total < nrows) nrows = *src.n_total;
  // wave index made provably uniform, so per-row loads are scalar
  const long long wid =
      blockIdx.x * (long long)kWaves +
      __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const long long nw = (long long)gridDim.x * kWaves;
  ApLds<NS>& mine = L[threadIdx.x / kWave];
  for (long long row = wid; row < nrows; row += nw)
    aperture_one<NS>(wk, p, src, sky_lohi, row, mine, atan_lds);
}

template __global__ void k_aperture_t<256>(Work, ipp_params, ipp_sources,
                                           double*);
template __global__ void k_aperture_t<512>(Work, ipp_params, ipp_sources,
                                           double*);
template __global__ void k_aperture_t<1024>(Work, ipp_params, ipp_sources,
                                            double*);

// ---------------------------------------------------------------------
// Backward of the aperture flux (the annulus clip mask held fixed: the
// survivors are the annulus pixels whose value lies in the forward's
// [vlo, vhi]).  With A = sum w_ap, W = sum m w_ann, sky = sum m w_ann v / W:
//   dF/dv_i = w_ap_i - A m_i w_ann_i / W
//   dF/dc   = sum v dw_ap/dc - sky dA/dc - A (sum m v dw_ann/dc
//             - sky sum m dw_ann/dc) / W
// One wavefront per source; pixel gradients are scattered with float
// atomics (dL/dI; dL/dB32 is its negative), centre gradients written per
// row.
// ---------------------------------------------------------------------
namespace {

template <int NS>
struct BwLds {
  // cut pixels: kind << 28 | wy << 6 | wx (kind 0: aperture, 1: annulus
  // survivor), and their weights
  int tk[NS + kApTasks];
  double tw[NS + kApTasks];
  double sq[3 * 2 * kEdges];     // edge square roots, as in the forward
};

// Per pixel of a source window, round by round (64 pixels): its window
// position, the exact membership distances and its two values.  Windows
// inside the frame load through 32-bit offsets advanced by constant steps;
// others through offsets clamped into the frame.
struct WinWalk {
  int xa, ya, nwx, npx, ry0;
  bool interior;
  const char* wpix;
  const char* wbkg;
  uint32_t pitchB, wB, stepP, stepB, wrapP, wrapB;
  int w, h, dwr, dwc;
  int wr, wc;
  uint32_t offp, offb;

  __device__ void init(const FrameDev& fr, int xa_, int xb, int ya_, int yb,
                       int lane) {
    xa = xa_;
    ya = ya_;
    nwx = xb - xa + 1;
    npx = nwx * (yb - ya + 1);
    w = fr.w;
    h = fr.h;
    ry0 = min(max(ya, 0), fr.h - 1);
    wpix = uniform_ptr((const char*)(fr.pix + (int64_t)ry0 * fr.pitch));
    wbkg = uniform_ptr((const char*)(fr.bkg + (int64_t)ry0 * fr.w));
    pitchB = (uint32_t)fr.pitch * 4u;
    wB = (uint32_t)fr.w * 4u;
    interior = xa >= 0 && ya >= 0 && xb < fr.w && yb < fr.h;
    dwr = kWave / nwx;
    dwc = kWave - dwr * nwx;
    stepP = (uint32_t)dwr * pitchB + (uint32_t)dwc * 4u;
    stepB = (uint32_t)dwr * wB + (uint32_t)dwc * 4u;
    wrapP = pitchB - (uint32_t)nwx * 4u;
    wrapB = wB - (uint32_t)nwx * 4u;
    wr = lane / nwx;
    wc = lane - wr * nwx;
    offp = (uint32_t)wr * pitchB + (uint32_t)(xa + wc) * 4u;
    offb = (uint32_t)wr * wB + (uint32_t)(xa + wc) * 4u;
  }
  // values of the current pixel; inside: the pixel lies in the frame
  __device__ void load(bool live, float* I, float* B, bool* inside) const {
    const int px = xa + wc, py = ya + wr;
    if (interior) {
      *inside = true;
      *I = gld((const float*)(wpix + (live ? offp : 0u)));
      *B = gld((const float*)(wbkg + (live ? offb : 0u)));
    } else {
      *inside = (px >= 0) & (px < w) & (py >= 0) & (py < h);
      const uint32_t qx = (uint32_t)min(max(px, 0), w - 1);
      const uint32_t qr = (uint32_t)(min(max(py, 0), h - 1) - ry0);
      *I = gld((const float*)(wpix + (qr * pitchB + qx * 4u)));
      *B = gld((const float*)(wbkg + (qr * wB + qx * 4u)));
    }
  }
  __device__ void advance() {
    wr += dwr;
    wc += dwc;
    offp += stepP;
    offb += stepB;
    if (wc >= nwx) {
      wc -= nwx;
      ++wr;
      offp += wrapP;
      offb += wrapB;
    }
  }
  // value of window pixel (wx, wy) (in the frame)
  __device__ double value_at(int wx, int wy) const {
    const uint32_t qr = (uint32_t)(ya + wy - ry0);
    const uint32_t qx = (uint32_t)(xa + wx);
    return (double)gld((const float*)(wpix + (qr * pitchB + qx * 4u))) -
           (double)gld((const float*)(wbkg + (qr * wB + qx * 4u)));
  }
};

// Nearest and farthest squared distance of window pixel (px, py) from the
// centre (the membership predicates compare them with r^2).
__device__ __forceinline__ void pixel_dist2(double cx, double cy, int px,
                                            int py, double* near2,
                                            double* far2) {
  const double ax = fabs((double)px - cx), ay = fabs((double)py - cy);
  const double nx = fmax(ax - 0.5, 0.0), ny = fmax(ay - 0.5, 0.0);
  const double fx = ax + 0.5, fy = ay + 0.5;
  *near2 = nx * nx + ny * ny;
  *far2 = fx * fx + fy * fy;
}

template <int NS>
__device__ void aperture_bwd_one(const Work& wk, const ipp_params& p,
                                 const ipp_sources& src,
                                 const double* sky_lohi, const double* gF,
                                 double* dxy, long long row, BwLds<NS>& L,
                                 const double* atan_lds) {
  const int lane = threadIdx.x & (kWave - 1);
  const int f = src.frame[row];
  const double cx = src.x[row], cy = src.y[row];
  const double g = gF[row];
  const bool fok = f >= 0 && f < wk.nframes;
  if (!fok || !(isfinite(cx) && isfinite(cy)) || fabs(cx) > 1e9 ||
      fabs(cy) > 1e9 || g == 0.0) {
    if (lane == 0 && dxy) { dxy[2 * row] = 0.0; dxy[2 * row + 1] = 0.0; }
    return;
  }
  const FrameDev fr = wk.frames[f];     // f is wave-uniform: SGPRs
  const double vlo = sky_lohi[2 * row], vhi = sky_lohi[2 * row + 1];
  const double R = p.r_ap > p.r_out ? p.r_ap : p.r_out;
  // window bounds: wave-uniform values, kept in scalar registers
  const int xa = __builtin_amdgcn_readfirstlane((int)ceil(cx - R - 0.5));
  const int xb = __builtin_amdgcn_readfirstlane((int)floor(cx + R + 0.5));
  const int ya = __builtin_amdgcn_readfirstlane((int)ceil(cy - R - 0.5));
  const int yb = __builtin_amdgcn_readfirstlane((int)floor(cy + R + 0.5));
  const double ra2 = p.r_ap * p.r_ap, ri2 = p.r_in * p.r_in;
  const double ro2 = p.r_out * p.r_out;

  // ---- pass 1: whole pixels summed, cut pixels listed ------------------
  // (aperture members: the square meets the disk; annulus survivors: it
  // meets the outer disk, is not inside the inner one, and its value lies
  // in the forward's [vlo, vhi])
  WinWalk W0;
  W0.init(fr, xa, xb, ya, yb, lane);
  double A = 0.0, Wt = 0.0, Sv = 0.0;
  int ntk = 0;
  // chunks of kBChunk rounds of 64 pixels: the loads of a chunk are all
  // issued before any is used
  constexpr int kBChunk = 4;
  for (int e00 = 0; e00 < W0.npx; e00 += kBChunk * kWave) {
  float Iv[kBChunk], Bv[kBChunk];
  bool insv[kBChunk];
  int posv[kBChunk];
#pragma unroll
  for (int c = 0; c < kBChunk; ++c) {
    if (e00 + c * kWave >= W0.npx) break;          // wave-uniform
    posv[c] = (W0.wr << 6) | W0.wc;
    W0.load(e00 + c * kWave + lane < W0.npx, &Iv[c], &Bv[c], &insv[c]);
    W0.advance();
  }
#pragma unroll
  for (int c = 0; c < kBChunk; ++c) {
    const int e0 = e00 + c * kWave;
    if (e0 >= W0.npx) break;                       // wave-uniform
    const bool live = e0 + lane < W0.npx;
    const int pos = posv[c];
    const int px = xa + (pos & 63), py = ya + (pos >> 6);
    const float I = Iv[c], B = Bv[c];
    const bool inside = insv[c];
    double near2, far2;
    pixel_dist2(cx, cy, px, py, &near2, &far2);
    const bool ok = live & inside & isfinite(I);
    const double v = (double)I - (double)B;
    const bool in_ap = ok & (near2 < ra2);
    const bool in_ann = ok & (near2 < ro2) & !(far2 <= ri2) & (v >= vlo) &
                        (v <= vhi);
    const bool ap_whole = in_ap & (far2 <= ra2);
    const bool ann_whole = in_ann & (far2 <= ro2) & !(near2 < ri2);
    A += ap_whole ? 1.0 : 0.0;
    if (ann_whole) {
      Wt += 1.0;
      Sv += v;
    }
    const bool ap_cut = in_ap & !ap_whole, ann_cut = in_ann & !ann_whole;
    const uint64_t b1 = ballot(ap_cut);
    if (ap_cut) {
      const int s = ntk + lanes_before(b1);
      if (s < NS + kApTasks) L.tk[s] = pos;
    }
    ntk += __popcll(b1);
    const uint64_t b2 = ballot(ann_cut);
    if (ann_cut) {
      const int s = ntk + lanes_before(b2);
      if (s < NS + kApTasks) L.tk[s] = (1 << 28) | pos;
    }
    ntk += __popcll(b2);
  }
  }
  if (ntk > NS + kApTasks) ntk = NS + kApTasks;   // not reachable
  // edge square roots of the window for the three circles
  for (int e = lane; e < 6 * kEdges; e += kWave) {
    const int c = e / (2 * kEdges), j = e % kEdges;
    const bool col = (e / kEdges) % 2 == 0;
    const double r = c == 0 ? p.r_ap : (c == 1 ? p.r_out : p.r_in);
    const double r2 = c == 0 ? ra2 : (c == 1 ? ro2 : ri2);
    const double q = col ? ((double)(xa + j) - 0.5) - cx
                         : ((double)(ya + j) - 0.5) - cy;
    L.sq[e] = edge_root(q, r, r2);
  }
  wave_lds_sync();

  // ---- pass 2: the cut pixels' weights and centre derivatives ----------
  double tvx = 0.0, tvy = 0.0, tax = 0.0, tay = 0.0;   // aperture terms
  double svx = 0.0, svy = 0.0, swx = 0.0, swy = 0.0;   // sky terms
  for (int j = lane; j < ntk; j += kWave) {
    int co = 0;
    asm volatile("" : "+s"(co));
    const double* coef = atan_lds + co;
    const int t = L.tk[j];
    const int wx = t & 63, wy = (t >> 6) & 63;
    const int px = xa + wx, py = ya + wy;
    const double v = W0.value_at(wx, wy);
    // overlap and its centre derivative for circle c
    auto circle = [&](int c, double r, double r2, double* gx, double* gy) {
      const double* sq = L.sq + c * 2 * kEdges;
      const double hx0 = sq[wx], hx1 = sq[wx + 1];
      const double xs0 = sq[kEdges + wy], xs1 = sq[kEdges + wy + 1];
      overlap_grad_roots(cx, cy, px, py, hx0, hx1, xs0, xs1, gx, gy);
      if (!touches(cx, cy, r, px, py)) return 0.0;
      if (within(cx, cy, r, px, py)) return 1.0;
      return overlap_cut(cx, cy, r, r2, px, py, hx0, hx1, xs0, xs1, coef);
    };
    double w, gx, gy;
    if ((t >> 28) == 0) {
      w = circle(0, p.r_ap, ra2, &gx, &gy);
      A += w;
      tvx += v * gx; tvy += v * gy;
      tax += gx; tay += gy;
    } else {
      double ix, iy;
      w = circle(1, p.r_out, ro2, &gx, &gy) -
          circle(2, p.r_in, ri2, &ix, &iy);
      gx -= ix;
      gy -= iy;
      Wt += w;
      Sv += w * v;
      svx += v * gx; svy += v * gy;
      swx += gx; swy += gy;
    }
    L.tw[j] = w;
  }
  A = wave_sum(A);
  Wt = wave_sum(Wt);
  Sv = wave_sum(Sv);
  tvx = wave_sum(tvx); tvy = wave_sum(tvy);
  tax = wave_sum(tax); tay = wave_sum(tay);
  svx = wave_sum(svx); svy = wave_sum(svy);
  swx = wave_sum(swx); swy = wave_sum(swy);
  const double sky = Wt > 0.0 ? Sv / Wt : 0.0;
  if (lane == 0 && dxy) {
    double dsx = 0.0, dsy = 0.0;
    if (Wt > 0.0) {
      dsx = (svx - sky * swx) / Wt;
      dsy = (svy - sky * swy) / Wt;
    }
    dxy[2 * row] = g * ((tvx - sky * tax) - A * dsx);
    dxy[2 * row + 1] = g * ((tvy - sky * tay) - A * dsy);
  }
  float* dp = fr.dpix;
  if (!dp) { wave_lds_sync(); return; }

  // ---- pass 3: scatter dL/dv (whole pixels, then the cut ones) ---------
  const double ks = Wt > 0.0 ? -g * A / Wt : 0.0;
  WinWalk W1;
  W1.init(fr, xa, xb, ya, yb, lane);
  for (int e0 = 0; e0 < W1.npx; e0 += kWave) {
    const bool live = e0 + lane < W1.npx;
    const int px = xa + W1.wc, py = ya + W1.wr;
    float I, B;
    bool inside;
    W1.load(live, &I, &B, &inside);
    double near2, far2;
    pixel_dist2(cx, cy, px, py, &near2, &far2);
    W1.advance();
    const bool ok = live & inside & isfinite(I);
    const double v = (double)I - (double)B;
    const bool ap_whole = ok & (near2 < ra2) & (far2 <= ra2);
    const bool ann_whole = ok & (near2 < ro2) & !(far2 <= ri2) &
                           (v >= vlo) & (v <= vhi) & (far2 <= ro2) &
                           !(near2 < ri2);
    const double gd = (ap_whole ? g : 0.0) + (ann_whole ? ks : 0.0);
    if (gd != 0.0) atomicAdd(&dp[(int64_t)py * fr.w + px], (float)gd);
  }
  for (int j = lane; j < ntk; j += kWave) {
    const int t = L.tk[j];
    const int px = xa + (t & 63), py = ya + ((t >> 6) & 63);
    const double k = (t >> 28) == 0 ? g : ks;
    atomicAdd(&dp[(int64_t)py * fr.w + px], (float)(k * L.tw[j]));
  }
  wave_lds_sync();
}

}  // namespace

template <int NS>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(NS <= 512 ? 3 : 1))) void k_aperture_bwd_t(
    Work wk, ipp_params p, ipp_sources src, const double* sky_lohi,
    const double* gF, double* dxy) {
  __shared__ BwLds<NS> L[kWaves];
  __shared__ double atan_lds[kAtanTerms];
  if (threadIdx.x < kAtanTerms) atan_lds[threadIdx.x] = atan_coef(threadIdx.x);
  __syncthreads();
  long long nrows = src.capacity;
  if (src.n_total && *src.n_total < nrows) nrows = *src.n_total;
  // wave index made provably uniform, so per-row loads are scalar
  const long long wid =
      blockIdx.x * (long long)kWaves +
      __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const long long nw = (long long)gridDim.x * kWaves;
  BwLds<NS>& mine = L[threadIdx.x / kWave];
  for (long long row = wid; row < nrows; row += nw)
    aperture_bwd_one<NS>(wk, p, src, sky_lohi, gF, dxy, row, mine,
                         atan_lds);
}

// ---------------------------------------------------------------------
// Centroid refinement around the photometry and its backward: maximise
// J(c) = F_rc(c) / F_ap(c0) by plain ascent c <- c + eta dJ/dc.  The
// backward is given dL/dF = g = 1 / F_ap(c0), so it returns dJ/dc; rows
// with F_ap(c0) <= 0 (or not a number) get g = 0 and stay in place.
// ---------------------------------------------------------------------
namespace {
__device__ __forceinline__ long long refine_rows(const int64_t* n_total,
                                                 int64_t cap) {
  long long n = cap;
  if (n_total && *n_total < n) n = *n_total;
  return n;
}
}  // namespace

__global__ __launch_bounds__(kBlock) void k_refine_start(
    const double* x, const double* y, double* xo, double* yo,
    uint32_t* flags, const int64_t* n_total, int64_t cap) {
  const long long n = refine_rows(n_total, cap);
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock) {
    const double a = x[i], b = y[i];    // read both before any write
    xo[i] = a;
    yo[i] = b;
    flags[i] = 0u;
  }
}

__global__ __launch_bounds__(kBlock) void k_refine_norm(
    const double* flux, double* g, const int64_t* n_total, int64_t cap) {
  const long long n = refine_rows(n_total, cap);
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock) {
    const double f = flux[i];
    g[i] = f > 0.0 ? 1.0 / f : 0.0;
  }
}

__global__ __launch_bounds__(kBlock) void k_refine_step(
    const double* dxy, const double* g, double* xo, double* yo, double eta,
    const int64_t* n_total, int64_t cap) {
  const long long n = refine_rows(n_total, cap);
  for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock) {
    if (g[i] != 0.0) {
      xo[i] = xo[i] + eta * dxy[2 * i];
      yo[i] = yo[i] + eta * dxy[2 * i + 1];
    }
  }
}

template __global__ void k_aperture_bwd_t<256>(
    Work, ipp_params, ipp_sources, const double*, const double*, double*);
template __global__ void k_aperture_bwd_t<512>(
    Work, ipp_params, ipp_sources, const double*, const double*, double*);
template __global__ void k_aperture_bwd_t<1024>(
    Work, ipp_params, ipp_sources, const double*, const double*, double*);

}  // namespace ipp
