// Aperture photometry with a local sky annulus (Sec. 2.2.5: per-object
// aperture photometry).
//
// One wavefront per source, four sources per workgroup, no workgroup
// barriers.  The wave walks the source's window with the exact membership
// predicates (from per-column and per-row distance tables), sums the
// pixels wholly inside the aperture, appends every annulus value to its
// LDS slice and lists every pixel cut by one of the three circles as one
// task per circle.  The annulus values are sorted in registers with a
// bitonic network and the k-sigma clipping of the sky works on contiguous
// ranges of the sorted values.  Only then are the exact overlap areas
// (binary64) computed, one uniform code path over the dense task list with
// every lane busy: each cut pixel adds its overlap (aperture) or the
// difference of its annulus weight from 1 (annulus survivors) to the sums.
#include <type_traits>

#include "ipp_internal.h"
#include "kernels.h"
#include "phot_geom.h"

namespace ipp {

namespace {

constexpr int kEdges = 36;      // pixel edges per axis of a window, r <= 16
// Pixels cut by one circle of radius r <= 16: a cut pixel's square holds
// points inside and outside the circle, so the circle crosses it; each of
// the circle's four monotone quarter arcs crosses at most r + 1 column and
// r + 1 row lines, so it passes through at most 2r + 3 squares.
constexpr int kCutCap = 8 * 16 + 16;
constexpr int kTaskCap = 3 * kCutCap;
constexpr int kTaskCapF = 4 * kCutCap;   // the forward's list (4 circles)

// A source's window of pixels: columns [xa, xa + nwx), rows [ya, ya + nwy).
// Loads take 32-bit byte offsets from a wave-uniform row base (the window's
// first in-frame row; pitch <= 2^24 and at most 35 rows).  A window wholly
// inside the frame needs neither clamping nor an inside test: its offsets
// advance by constant steps.
struct Window {
  int xa, ya, nwx, nwy, npx, ry0, fw, fh;
  bool interior;
  const char* wpix;
  const char* wbkg;
  uint32_t pitchB, wB;

  __device__ void init(const FrameDev& fr, int xa_, int xb, int ya_, int yb) {
    xa = xa_;
    ya = ya_;
    nwx = xb - xa + 1;
    nwy = yb - ya + 1;
    npx = nwx * nwy;
    fw = fr.w;
    fh = fr.h;
    ry0 = min(max(ya, 0), fr.h - 1);
    wpix = uniform_ptr((const char*)(fr.pix + (int64_t)ry0 * fr.pitch));
    wbkg = uniform_ptr((const char*)(fr.bkg + (int64_t)ry0 * fr.w));
    pitchB = (uint32_t)fr.pitch * 4u;
    wB = (uint32_t)fr.w * 4u;
    interior = xa >= 0 && ya >= 0 && xb < fr.w && yb < fr.h;
  }
  // v = I - B of the in-frame pixel (px, py)
  __device__ double value_at(int px, int py) const {
    const uint32_t qr = (uint32_t)(py - ry0);
    return (double)gld((const float*)(wpix + (qr * pitchB + (uint32_t)px * 4u))) -
           (double)gld((const float*)(wbkg + (qr * wB + (uint32_t)px * 4u)));
  }
  // Every pixel of the window, 64 a round: visit(live, pos, ok, v, mok,
  // mlive) with pos = wy << 6 | wx, ok = the pixel lies in the frame and I
  // is finite, v = I - B, mok and mlive = the wave's lanes with ok and with
  // live.  Lanes past the
  // window's end visit with live = false (a valid position, ok = false).
  // The loads of kChunk rounds are issued before any is used, so their
  // latencies overlap.  Lane masks are formed as products of ballots of
  // single comparisons (each ballot is that comparison's own result): a
  // ballot of a compound predicate costs two vector instructions more.
  template <int kChunk, bool EDGE, typename F>
  __device__ void walk_t(int lane, F&& visit) const {
    const int dwr = kWave / nwx, dwc = kWave - (kWave / nwx) * nwx;
    int wr = lane / nwx, wc = lane - (lane / nwx) * nwx;  // window row, col
    uint32_t offp = (uint32_t)wr * pitchB + (uint32_t)(xa + wc) * 4u;
    uint32_t offb = (uint32_t)wr * wB + (uint32_t)(xa + wc) * 4u;
    const uint32_t stepP = (uint32_t)dwr * pitchB + (uint32_t)dwc * 4u;
    const uint32_t stepB = (uint32_t)dwr * wB + (uint32_t)dwc * 4u;
    const uint32_t wrapP = pitchB - (uint32_t)nwx * 4u;
    const uint32_t wrapB = wB - (uint32_t)nwx * 4u;
    for (int e0 = 0; e0 < npx; e0 += kChunk * kWave) {
      float Iv[kChunk], Bv[kChunk];
      int pos[kChunk];
      bool ins[kChunk];
      uint64_t mins[kChunk];
#pragma unroll
      for (int c = 0; c < kChunk; ++c) {
        if (e0 + c * kWave >= npx) break;            // wave-uniform
        const bool live = e0 + c * kWave + lane < npx;
        pos[c] = (wr << 6) | wc;
        if constexpr (EDGE) {
          // loads clamped into the frame: every lane loads, no branches
          const int px = xa + wc, py = ya + wr;
          ins[c] = live & (px >= 0) & (px < fw) & (py >= 0) & (py < fh);
          mins[c] = ballot(live) & ballot(px >= 0) & ballot(px < fw) &
                    ballot(py >= 0) & ballot(py < fh);
          const uint32_t qx = (uint32_t)min(max(px, 0), fw - 1);
          const uint32_t qr = (uint32_t)(min(max(py, 0), fh - 1) - ry0);
          Iv[c] = gld((const float*)(wpix + (qr * pitchB + qx * 4u)));
          Bv[c] = gld((const float*)(wbkg + (qr * wB + qx * 4u)));
        } else {
          // a lane past the window end loads the window's first pixel
          ins[c] = live;
          Iv[c] = gld((const float*)(wpix + (live ? offp : 0u)));
          Bv[c] = gld((const float*)(wbkg + (live ? offb : 0u)));
        }
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
        const bool live = e0 + c * kWave + lane < npx;
        // finite: |I| at most the largest float (false for NaN)
        const bool fin = fabsf(Iv[c]) <= 3.40282347e38f;
        // the live lanes as a scalar mask: the first npx - e lanes
        const int rem = npx - (e0 + c * kWave);
        const uint64_t mlive = rem >= kWave ? ~0ull : (1ull << rem) - 1ull;
        visit(live, pos[c], ins[c] & fin, (double)Iv[c] - (double)Bv[c],
              (EDGE ? mins[c] : mlive) & ballot(fin), mlive);
      }
    }
  }
  template <int kChunk, typename F>
  __device__ void walk(int lane, F&& visit) const {
    if (interior) walk_t<kChunk, false>(lane, visit);
    else walk_t<kChunk, true>(lane, visit);
  }
};

// Per window column and row: the squared nearest and farthest offsets from
// the centre (a pixel's distances are sums of one of each: the same two
// rounded squares and the same addition as computing them per pixel) and,
// at every column (row) edge q, the roots sqrt(r^2 - min(|q|, r)^2) of the
// NC circles (aperture, outer, inner, and a second aperture r_x when NC is
// 4), for the exact overlaps.
template <int NC>
struct WinTablesT {
  double2 colT[kEdges];
  double2 rowT[kEdges];
  double sq[NC * 2 * kEdges];      // [circle][axis][edge]

  __device__ void fill(const Window& W, double cx, double cy, double r_ap,
                       double r_in, double r_out, int lane,
                       double r_x = 0.0) {
    const double ra2 = r_ap * r_ap, ri2 = r_in * r_in;
    const double ro2 = r_out * r_out, rx2 = r_x * r_x;
    const int ne = (W.nwx > W.nwy ? W.nwx : W.nwy) + 1;   // <= kEdges
    for (int e = lane; e < 2 * ne; e += kWave) {
      const bool col = e < ne;
      const int j = col ? e : e - ne;
      const double a = col ? fabs((double)(W.xa + j) - cx)
                           : fabs((double)(W.ya + j) - cy);
      const double n = fmax(a - 0.5, 0.0), fo = a + 0.5;
      double2 t;
      t.x = n * n;
      t.y = fo * fo;
      const double q = col ? ((double)(W.xa + j) - 0.5) - cx
                           : ((double)(W.ya + j) - 0.5) - cy;
      const int ax = col ? 0 : kEdges;
      if (j < kEdges) {
        (col ? colT : rowT)[j] = t;
        sq[ax + j] = edge_root(q, r_ap, ra2);
        sq[2 * kEdges + ax + j] = edge_root(q, r_out, ro2);
        sq[4 * kEdges + ax + j] = edge_root(q, r_in, ri2);
        if constexpr (NC > 3) sq[6 * kEdges + ax + j] = edge_root(q, r_x, rx2);
      }
    }
  }
  // squared nearest and farthest distance of the pixel at pos (a position
  // past the window's end reads a valid row of the table)
  __device__ void dist2(int pos, double* near2, double* far2) const {
    const double2 tc = colT[pos & 63];
    const double2 tr = rowT[min(pos >> 6, kEdges - 1)];
    *near2 = tc.x + tr.x;
    *far2 = tc.y + tr.y;
  }
};
using WinTables = WinTablesT<3>;

// Circle of a task: 0 the aperture, 1 the outer, 2 the inner annulus circle.
__device__ __forceinline__ void task_circle(double r_ap, double r_in,
                                            double r_out, int c, double* r,
                                            double* r2) {
  const double rr = c == 0 ? r_ap : (c == 1 ? r_out : r_in);
  *r = rr;
  *r2 = rr * rr;
}
// The same with circle 3, a second aperture r_x.
__device__ __forceinline__ void task_circle4(double r_ap, double r_in,
                                             double r_out, double r_x, int c,
                                             double* r, double* r2) {
  const double rr = c == 0 ? r_ap : (c == 1 ? r_out : (c == 2 ? r_in : r_x));
  *r = rr;
  *r2 = rr * rr;
}

// NC: circles of the window tables (4 with a second aperture).
template <int NS, int NC = 3>
struct ApLds {
  static constexpr int kCap = NC > 3 ? kTaskCapF : kTaskCap;
  // the annulus values as they are found; once read into registers, the
  // sort's transposes and then the sorted values
  double xs[NS + kWave];
  // pixels cut by a circle: circle << 12 | wy << 6 | wx (circle 0: the
  // aperture, 1: the outer and 2: the inner annulus circle, 3: the second
  // aperture).  The lists start kWave slots in from either end and their
  // counts are clamped round by round, so a round's appends stay inside the
  // array without a bound test per lane (the values lists likewise: the
  // count stays at most NS, and xs has kWave slots more).
  int tk[kCap + 2 * kWave];
  WinTablesT<NC> T;
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

// Photometry of one source whose frame and centre are valid: the sums of
// the aperture flux and the sky, and with GRAD the centre derivative of
// the flux with the sky clip mask held fixed (as the backward below).
struct ApOut {
  double raw;          // sum of w v over the aperture
  double a_ap;         // aperture area (sum of w)
  double num, den;     // sum of m w v and of m w over the annulus
  double vlo, vhi;     // the sky survivors' value range (empty: vlo > vhi)
  uint32_t flags;
  double dfx, dfy;     // dF/dcx, dF/dcy (GRAD)
  double raw_x, a_x;   // raw and a_ap of the second aperture (r_x > 0)
  uint32_t flags_x;    // flags of the second aperture's photometry
};

// With GRAD, `norm` (wave-uniform) asks for the flux sums only (raw, not
// the derivative sums) and its absence for the derivative only (no raw).
// r_x > 0 (wave-uniform) adds the flux sums of a second aperture of that
// radius about the same centre, over the same sky: the refinement's
// normaliser taken in the evaluation of its first step.
template <int NS, bool GRAD, int NC = 3, bool XFLAGS = false>
__device__ ApOut aperture_eval(const FrameDev& fr, const ipp_params& p,
                               double r_ap, double cx, double cy,
                               ApLds<NS, NC>& L, const double* atan_lds,
                               int lane, bool norm = true,
                               double r_x = 0.0) {
  constexpr int kCapT = ApLds<NS, NC>::kCap;
  constexpr int PL = NS / kWave;
  constexpr int P = PL == 4 ? 2 : (PL == 8 ? 3 : 4);
  static_assert((1 << P) == PL, "NS is 256, 512 or 1024");
  const bool dual = NC > 3 && r_x > 0.0;
  double R = r_ap > p.r_out ? r_ap : p.r_out;
  R = r_x > R ? r_x : R;
  // window bounds: wave-uniform values, kept in scalar registers
  Window W;
  W.init(fr, __builtin_amdgcn_readfirstlane((int)ceil(cx - R - 0.5)),
         __builtin_amdgcn_readfirstlane((int)floor(cx + R + 0.5)),
         __builtin_amdgcn_readfirstlane((int)ceil(cy - R - 0.5)),
         __builtin_amdgcn_readfirstlane((int)floor(cy + R + 0.5)));
  // squared radii as the membership predicates form them
  const double ra2 = r_ap * r_ap, ri2 = p.r_in * p.r_in;
  const double ro2 = p.r_out * p.r_out, rx2 = r_x * r_x;
  L.T.fill(W, cx, cy, r_ap, p.r_in, p.r_out, lane, r_x);
  wave_lds_sync();

  // ---- walk the window: sums, annulus values, cut pixels ---------------
  // Aperture tasks are listed from the front of the task list, annulus
  // tasks from its back, so that the few rounds of aperture tasks (whose
  // angles may need the general path) are not spread over the list.
  int nfull = 0;                       // pixels wholly inside the aperture
  int nann = 0, nt0 = 0, nt1 = 0;      // wave-uniform list lengths
  double raw = 0.0;                    // per lane: sum of v over them
  int nfull_x = 0;                     // the same for the second aperture
  double raw_x = 0.0;
  uint64_t bad_x = 0;
  uint64_t bad_ap = 0, bad_ann = 0;    // lanes of members not ok
  W.walk<4>(lane, [&](bool live, int q, bool ok, double v, uint64_t mok,
                      uint64_t mlive) {
    double near2, far2;
    L.T.dist2(q, &near2, &far2);
    const bool in_ap = live & (near2 < ra2);
    const bool in_ann = live & (near2 < ro2) & !(far2 <= ri2);
    const bool ap_whole = far2 <= ra2;
    const uint64_t m_ap = mlive & ballot(near2 < ra2);
    const uint64_t m_ann =
        mlive & ballot(near2 < ro2) & ~ballot(far2 <= ri2);
    const uint64_t m_whole = ballot(ap_whole);
    bad_ap |= m_ap & ~mok;
    bad_ann |= m_ann & ~mok;
    const bool full = in_ap & ok & ap_whole;
    nfull += __popcll(m_ap & mok & m_whole);
    if (full) raw += v;
    const bool ann = in_ann & ok;
    const uint64_t ba = m_ann & mok;
    if (ann) L.xs[nann + lanes_before(ba)] = v;
    nann = min(nann + (int)__popcll(ba), NS);
    // one task per circle that cuts the pixel
    const bool c0 = in_ap & ok & !ap_whole;
    const bool c1 = ann & !(far2 <= ro2);
    const bool c2 = ann & (near2 < ri2);
    const uint64_t b0 = m_ap & mok & ~m_whole;
    const uint64_t b1 = ba & ~ballot(far2 <= ro2);
    const uint64_t b2 = ba & ballot(near2 < ri2);
    if (c0) L.tk[kWave + nt0 + lanes_before(b0)] = q;
    nt0 = min(nt0 + (int)__popcll(b0), kCapT);
    if (c1)
      L.tk[kWave + kCapT - 1 - (nt1 + lanes_before(b1))] = (1 << 12) | q;
    nt1 = min(nt1 + (int)__popcll(b1), kCapT);
    if (c2)
      L.tk[kWave + kCapT - 1 - (nt1 + lanes_before(b2))] = (2 << 12) | q;
    nt1 = min(nt1 + (int)__popcll(b2), kCapT);
    if (dual) {
      // the second aperture: whole pixels summed, cut ones listed with
      // the aperture's from the front
      const bool x_whole = far2 <= rx2;
      const uint64_t m_xa = mlive & ballot(near2 < rx2);
      if constexpr (XFLAGS) bad_x |= m_xa & ~mok;
      const uint64_t m_x = m_xa & mok;
      const uint64_t m_xw = ballot(x_whole);
      nfull_x += __popcll(m_x & m_xw);
      if (live & ok & (near2 < rx2) & x_whole) raw_x += v;
      const uint64_t b3 = m_x & ~m_xw;
      if (live & ok & (near2 < rx2) & !x_whole)
        L.tk[kWave + nt0 + lanes_before(b3)] = (3 << 12) | q;
      nt0 = min(nt0 + (int)__popcll(b3), kCapT);
    }
  });
  // not reachable: NS bounds the ring, and the task lists cannot meet
  if (nt0 + nt1 > kCapT) { nt0 = min(nt0, kCapT); nt1 = kCapT - nt0; }
  ApOut o;
  o.flags = 0;                         // wave-uniform
  if (bad_ap) o.flags |= IPP_SRC_APERTURE_OFF_EDGE;
  if (bad_ann) o.flags |= IPP_SRC_ANNULUS_OFF_EDGE;
  o.flags_x = (bad_x ? IPP_SRC_APERTURE_OFF_EDGE : 0u) |
              (bad_ann ? IPP_SRC_ANNULUS_OFF_EDGE : 0u);
  wave_lds_sync();

  // ---- sort the annulus values ------------------------------------------
  double sv[PL];
#pragma unroll
  for (int k = 0; k < PL; ++k) {
    const int e = lane * PL + k;
    sv[k] = e < nann ? L.xs[e] : __builtin_inf();
  }
  wave_lds_sync();                     // read before the network writes
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
#pragma clang fp contract(fast)
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
    const double inv_n = 1.0 / (double)n;
    const double dm = S1 * inv_n;
    const double var = S2 * inv_n - dm * dm;
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
    // the removed values are the sorted ranges [a, a + cl) and
    // [bnd - ch, bnd): one lane reads each from LDS (usually one round)
    double r1 = 0.0, r2 = 0.0;
    for (int j = lane; j < cl + ch; j += kWave) {
#pragma clang fp contract(fast)
      const int e = j < cl ? a + j : bnd - ch + (j - cl);
      const double d = sorted_at<P>(L.xs, e) - c0;
      r1 += d;
      r2 += d * d;
    }
    S1 -= wave_sum(r1);
    S2 -= wave_sum(r2);
    a += cl;
    bnd -= ch;
  }
  // the survivors are the values in [vlo, vhi] (clipping is by value);
  // with weight 1 each they sum to su
  o.vlo = 0.0;
  o.vhi = -1.0;
  if (bnd > a) {
    o.vlo = sorted_at<P>(L.xs, a);
    o.vhi = sorted_at<P>(L.xs, bnd - 1);
  }
  const double vlo = o.vlo, vhi = o.vhi;
  double su = 0.0;
#pragma unroll
  for (int k = 0; k < PL; ++k) {
    const int e = lane * PL + k;
    su += (e >= a && e < bnd) ? sv[k] : 0.0;
  }
  su = wave_sum(su);                   // before the sorted registers die

  // ---- exact overlaps of the cut pixels ----------------------------------
  // One overlap per task, whatever circle it belongs to.  An aperture task
  // adds w and w v; an annulus task of a survivor corrects its weight 1:
  // by w - 1 for the outer circle and by -w for the inner one (a pixel cut
  // by both gets w_out - w_in).  With GRAD the centre derivatives of the
  // same overlaps (chords at the pixel's corners) are summed alongside.
  double acut = 0.0, dnum = 0.0, dden = 0.0, acut_x = 0.0;
  double tvx = 0.0, tvy = 0.0, tax = 0.0, tay = 0.0;   // aperture terms
  double svx = 0.0, svy = 0.0, swx = 0.0, swy = 0.0;   // sky terms
  const int ntk = nt0 + nt1;
  for (int j = lane; j < ntk; j += kWave) {
#pragma clang fp contract(fast)
    // the series coefficients are read where they are used (an offset the
    // compiler cannot hoist keeps them out of registers across the loop)
    int co = 0;
    asm volatile("" : "+s"(co));
    const double* coef = atan_lds + co;
    const int t = L.tk[kWave + (j < nt0 ? j : kCapT - nt1 + (j - nt0))];
    const int c = t >> 12, wx = t & 63, wy = (t >> 6) & 63;
    const int px = W.xa + wx, py = W.ya + wy;
    double r, r2;
    if constexpr (NC > 3) task_circle4(r_ap, p.r_in, p.r_out, r_x, c, &r, &r2);
    else task_circle(r_ap, p.r_in, p.r_out, c, &r, &r2);
    const double* sq = L.T.sq + c * 2 * kEdges;
    const double hx0 = sq[wx], hx1 = sq[wx + 1];
    const double xs0 = sq[kEdges + wy], xs1 = sq[kEdges + wy + 1];
    const double w = overlap_cut(cx, cy, r, r2, px, py, hx0, hx1, xs0, xs1,
                                 coef);
    const double v = W.value_at(px, py);
    double gx = 0.0, gy = 0.0;
    if constexpr (GRAD)
      overlap_grad_roots(cx, cy, px, py, hx0, hx1, xs0, xs1, &gx, &gy);
    if (c == 0) {
      acut += w;
      raw += w * v;
      if constexpr (GRAD) {
        tvx += v * gx; tvy += v * gy;
        tax += gx; tay += gy;
      }
    } else if (c == 3) {
      acut_x += w;
      raw_x += w * v;
    } else if (v >= vlo && v <= vhi) {
      const double dw = c == 1 ? w - 1.0 : -w;
      dden += dw;
      dnum += dw * v;
      if constexpr (GRAD) {
        // the inner circle's overlap enters negated
        if (c == 2) { gx = -gx; gy = -gy; }
        svx += v * gx; svy += v * gy;
        swx += gx; swy += gy;
      }
    }
  }
  o.a_ap = (double)nfull + wave_sum(acut);
  o.raw = !GRAD || norm ? wave_sum(raw) : 0.0;
  o.raw_x = o.a_x = 0.0;
  if (dual) {
    o.a_x = (double)nfull_x + wave_sum(acut_x);
    o.raw_x = wave_sum(raw_x);
  }
  o.num = su + wave_sum(dnum);
  o.den = (double)(bnd - a) + wave_sum(dden);
  o.dfx = o.dfy = 0.0;
  if (GRAD && !norm) {
    tvx = wave_sum(tvx); tvy = wave_sum(tvy);
    tax = wave_sum(tax); tay = wave_sum(tay);
    svx = wave_sum(svx); svy = wave_sum(svy);
    swx = wave_sum(swx); swy = wave_sum(swy);
    const double sky = o.den > 0.0 ? o.num / o.den : 0.0;
    double dsx = 0.0, dsy = 0.0;
    if (o.den > 0.0) {
      dsx = (svx - sky * swx) / o.den;
      dsy = (svy - sky * swy) / o.den;
    }
    o.dfx = (tvx - sky * tax) - o.a_ap * dsx;
    o.dfy = (tvy - sky * tay) - o.a_ap * dsy;
  }
  wave_lds_sync();                     // the slice is reused next
  return o;
}

__device__ __forceinline__ bool centre_ok(double cx, double cy) {
  return isfinite(cx) && isfinite(cy) && fabs(cx) <= 1e9 && fabs(cy) <= 1e9;
}

template <int NS>
__device__ void aperture_one(const Work& wk, const ipp_params& p,
                             ipp_sources& src, double* sky_lohi,
                             long long row, ApLds<NS>& L,
                             const double* atan_lds) {
  // the lane number made opaque to the compiler at every row: addresses
  // derived from it are formed where they are used instead of being kept
  // in registers across the whole row loop
  int lane = threadIdx.x & (kWave - 1);
  asm volatile("" : "+v"(lane));
  const int f = src.frame[row];
  const double cx = src.x[row], cy = src.y[row];
  if (!(f >= 0 && f < wk.nframes) || !centre_ok(cx, cy)) {
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
  const ApOut o =
      aperture_eval<NS, false>(fr, p, p.r_ap, cx, cy, L, atan_lds, lane);
  if (lane == 0) {
    uint32_t flags = o.flags;
    double sky = 0.0;
    if (o.den > 0.0) sky = o.num / o.den; else flags |= IPP_SRC_NO_SKY;
    src.flux_ap[row] = o.raw - sky * o.a_ap;
    src.sky[row] = sky;
    src.area_ap[row] = o.a_ap;
    src.area_ann[row] = o.den;
    src.flags[row] |= flags;
    if (sky_lohi) { sky_lohi[2 * row] = o.vlo; sky_lohi[2 * row + 1] = o.vhi; }
  }
}

// Centroid refinement of one source: the normaliser F_ap(c0) with p's
// aperture, then `steps` ascent steps c <- c + eta g dF_rc/dc (g =
// 1 / F_ap(c0)), each step's derivative taken with that step's sky clip
// mask, all in this wave.  The first step's evaluation (at c0) also takes
// the normaliser, as the flux of a second aperture over the same sky; with
// `phot` that evaluation's photometry (p's aperture at c0) is written to
// the row as aperture_one writes it.  Sources with g = 0 (F_ap(c0) <= 0 or
// not a number) stay in place, and so does a centre that leaves the valid
// range.
template <int NS, bool PHOT>
__device__ void refine_one(const Work& wk, const ipp_params& p,
                           double r_c, double eta, int steps,
                           const ipp_sources& src, double* xo, double* yo,
                           long long row, ApLds<NS, 4>& L,
                           const double* atan_lds, void* const* cols) {
  int lane = threadIdx.x & (kWave - 1);
  asm volatile("" : "+v"(lane));
  const int f = src.frame[row];
  double cx = src.x[row], cy = src.y[row];
  if ((f >= 0 && f < wk.nframes) && centre_ok(cx, cy)) {
    const FrameDev fr = wk.frames[f];   // f is wave-uniform: SGPRs
    // one call site, so that the photometry is inlined once; with phot
    // and no steps the first evaluation is still taken
    double g = 0.0;
    const int nev = steps > 0 ? steps : (PHOT ? 1 : 0);
    for (int k = 0; k < nev; ++k) {
      const ApOut o = aperture_eval<NS, true, 4, PHOT>(
          fr, p, r_c, cx, cy, L, atan_lds, lane, false,
          k == 0 ? p.r_ap : 0.0);
      if (k == 0) {
        const double sky0 = o.den > 0.0 ? o.num / o.den : 0.0;
        const double F0 = o.raw_x - sky0 * o.a_x;
        if (PHOT && lane == 0) {
          ((double*)cols[0])[row] = F0;
          ((double*)cols[1])[row] = sky0;
          ((double*)cols[2])[row] = o.a_x;
          ((double*)cols[3])[row] = o.den;
          ((uint32_t*)cols[4])[row] |=
              o.flags_x | (o.den > 0.0 ? 0u : IPP_SRC_NO_SKY);
        }
        if (k == steps) break;
        g = F0 > 0.0 ? 1.0 / F0 : 0.0;
        if (g == 0.0) break;
      }
      const double dx = g * o.dfx, dy = g * o.dfy;
      cx = cx + eta * dx;
      cy = cy + eta * dy;
      if (!centre_ok(cx, cy)) break;
    }
  } else if (PHOT && lane == 0) {
    ((double*)cols[0])[row] = __builtin_nan("");
    ((double*)cols[1])[row] = __builtin_nan("");
    ((double*)cols[2])[row] = 0.0;
    ((double*)cols[3])[row] = 0.0;
    ((uint32_t*)cols[4])[row] |= IPP_SRC_APERTURE_OFF_EDGE | IPP_SRC_NO_SKY;
  }
  if (lane == 0) {
    xo[row] = cx;
    yo[row] = cy;
  }
}

}  // namespace

// NS: sort size (>= the annulus pixel count bound).
template <int NS>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(NS <= 512 ? 4 : 1))) void k_aperture_t(
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

// Centroid refinement: one wavefront per row, every step in the wave
// (PHOT: the photometry of the first evaluation is written too; a
// variant of its own, so that the plain refinement keeps its registers).
template <int NS, bool PHOT>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(NS <= 512 ? 3 : 1))) void k_refine_t(
    Work wk, ipp_params p, double r_c, double eta, int steps,
    ipp_sources src, double* xo, double* yo) {
  __shared__ ApLds<NS, 4> L[kWaves];
  __shared__ double atan_lds[kAtanTerms];
  // the photometry columns' addresses, read from LDS where they are
  // written: kept in scalar registers across the row loop they would push
  // the kernel's scalar registers into spills
  __shared__ void* cols[5];
  if (threadIdx.x < kAtanTerms) atan_lds[threadIdx.x] = atan_coef(threadIdx.x);
  if (PHOT && threadIdx.x == 0) {
    cols[0] = src.flux_ap;
    cols[1] = src.sky;
    cols[2] = src.area_ap;
    cols[3] = src.area_ann;
    cols[4] = src.flags;
  }
  __syncthreads();
  long long nrows = src.capacity;
  if (src.n_total && *src.n_total < nrows) nrows = *src.n_total;
  const long long wid =
      blockIdx.x * (long long)kWaves +
      __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const long long nw = (long long)gridDim.x * kWaves;
  ApLds<NS, 4>& mine = L[threadIdx.x / kWave];
  for (long long row = wid; row < nrows; row += nw)
    refine_one<NS, PHOT>(wk, p, r_c, eta, steps, src, xo, yo, row, mine,
                         atan_lds, cols);
}

template __global__ void k_refine_t<256, false>(Work, ipp_params, double,
    double, int, ipp_sources, double*, double*);
template __global__ void k_refine_t<256, true>(Work, ipp_params, double,
    double, int, ipp_sources, double*, double*);
template __global__ void k_refine_t<512, false>(Work, ipp_params, double,
    double, int, ipp_sources, double*, double*);
template __global__ void k_refine_t<512, true>(Work, ipp_params, double,
    double, int, ipp_sources, double*, double*);
template __global__ void k_refine_t<1024, false>(Work, ipp_params, double,
    double, int, ipp_sources, double*, double*);
template __global__ void k_refine_t<1024, true>(Work, ipp_params, double,
    double, int, ipp_sources, double*, double*);
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
  // pixels cut by a circle: circle << 12 | wy << 6 | wx (circle 0: the
  // aperture, 1: the outer and 2: the inner circle of a survivor), and the
  // pixel weight each adds (w, w - 1, -w)
  int tk[kTaskCap];
  double tw[kTaskCap];
  WinTables T;
};

template <int NS>
__device__ void aperture_bwd_one(const Work& wk, const ipp_params& p,
                                 const ipp_sources& src,
                                 const double* sky_lohi, const double* gF,
                                 double* dxy, long long row, BwLds<NS>& L,
                                 const double* atan_lds) {
  int lane = threadIdx.x & (kWave - 1);
  asm volatile("" : "+v"(lane));
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
  Window W;
  W.init(fr, __builtin_amdgcn_readfirstlane((int)ceil(cx - R - 0.5)),
         __builtin_amdgcn_readfirstlane((int)floor(cx + R + 0.5)),
         __builtin_amdgcn_readfirstlane((int)ceil(cy - R - 0.5)),
         __builtin_amdgcn_readfirstlane((int)floor(cy + R + 0.5)));
  const double ra2 = p.r_ap * p.r_ap, ri2 = p.r_in * p.r_in;
  const double ro2 = p.r_out * p.r_out;
  L.T.fill(W, cx, cy, p.r_ap, p.r_in, p.r_out, lane);
  wave_lds_sync();

  // ---- pass 1: whole pixels summed, cut pixels listed ------------------
  // Aperture members: the square meets the disk; annulus survivors: it
  // meets the outer disk, is not inside the inner one, and its value lies
  // in the forward's [vlo, vhi].  Every survivor counts with weight 1 here;
  // its cut tasks correct that weight.
  int nwhole = 0, nsurv = 0, ntk = 0;  // wave-uniform
  double Sv = 0.0;                     // per lane: sum of survivor values
  W.walk<4>(lane, [&](bool live, int q, bool ok, double v, uint64_t mok,
                      uint64_t) {
    double near2, far2;
    L.T.dist2(q, &near2, &far2);
    const bool in_ap = live & ok & (near2 < ra2);
    const bool surv = live & ok & (near2 < ro2) & !(far2 <= ri2) &
                      (v >= vlo) & (v <= vhi);
    const bool ap_whole = far2 <= ra2;
    const uint64_t m_ap = mok & ballot(near2 < ra2);
    const uint64_t m_surv = mok & ballot(near2 < ro2) & ~ballot(far2 <= ri2) &
                            ballot(v >= vlo) & ballot(v <= vhi);
    const uint64_t m_whole = ballot(ap_whole);
    nwhole += __popcll(m_ap & m_whole);
    nsurv += __popcll(m_surv);
    if (surv) Sv += v;
    const bool c0 = in_ap & !ap_whole;
    const bool c1 = surv & !(far2 <= ro2);
    const bool c2 = surv & (near2 < ri2);
    const uint64_t b0 = m_ap & ~m_whole;
    const uint64_t b1 = m_surv & ~ballot(far2 <= ro2);
    const uint64_t b2 = m_surv & ballot(near2 < ri2);
    if (c0) {
      const int s = ntk + lanes_before(b0);
      if (s < kTaskCap) L.tk[s] = q;
    }
    ntk += __popcll(b0);
    if (c1) {
      const int s = ntk + lanes_before(b1);
      if (s < kTaskCap) L.tk[s] = (1 << 12) | q;
    }
    ntk += __popcll(b1);
    if (c2) {
      const int s = ntk + lanes_before(b2);
      if (s < kTaskCap) L.tk[s] = (2 << 12) | q;
    }
    ntk += __popcll(b2);
  });
  if (ntk > kTaskCap) ntk = kTaskCap;   // not reachable
  wave_lds_sync();

  // ---- pass 2: the cut pixels' weights and centre derivatives ----------
  double A = 0.0, Wt = 0.0;                            // cut-pixel parts
  double tvx = 0.0, tvy = 0.0, tax = 0.0, tay = 0.0;   // aperture terms
  double svx = 0.0, svy = 0.0, swx = 0.0, swy = 0.0;   // sky terms
  for (int j = lane; j < ntk; j += kWave) {
    int co = 0;
    asm volatile("" : "+s"(co));
    const double* coef = atan_lds + co;
    const int t = L.tk[j];
    const int c = t >> 12, wx = t & 63, wy = (t >> 6) & 63;
    const int px = W.xa + wx, py = W.ya + wy;
    double r, r2;
    task_circle(p.r_ap, p.r_in, p.r_out, c, &r, &r2);
    const double* sq = L.T.sq + c * 2 * kEdges;
    const double hx0 = sq[wx], hx1 = sq[wx + 1];
    const double xs0 = sq[kEdges + wy], xs1 = sq[kEdges + wy + 1];
    double gx, gy;
    overlap_grad_roots(cx, cy, px, py, hx0, hx1, xs0, xs1, &gx, &gy);
    const double w = overlap_cut(cx, cy, r, r2, px, py, hx0, hx1, xs0, xs1,
                                 coef);
    const double v = W.value_at(px, py);
    double tw;
    if (c == 0) {
      A += w;
      tvx += v * gx; tvy += v * gy;
      tax += gx; tay += gy;
      tw = w;
    } else {
      // the inner circle's overlap and its derivative enter negated
      const double s = c == 1 ? 1.0 : -1.0;
      tw = c == 1 ? w - 1.0 : -w;
      gx *= s;
      gy *= s;
      Wt += tw;
      Sv += tw * v;
      svx += v * gx; svy += v * gy;
      swx += gx; swy += gy;
    }
    L.tw[j] = tw;
  }
  A = (double)nwhole + wave_sum(A);
  Wt = (double)nsurv + wave_sum(Wt);
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

  // ---- pass 3: scatter dL/dv ---------------------------------------------
  // whole aperture pixels get g, every survivor ks (its weight 1); the cut
  // tasks add g w, ks (w - 1) or -ks w
  const double ks = Wt > 0.0 ? -g * A / Wt : 0.0;
  W.walk<4>(lane, [&](bool live, int q, bool ok, double v, uint64_t,
                      uint64_t) {
    double near2, far2;
    L.T.dist2(q, &near2, &far2);
    const bool ap_whole = live & ok & (near2 < ra2) & (far2 <= ra2);
    const bool surv = live & ok & (near2 < ro2) & !(far2 <= ri2) &
                      (v >= vlo) & (v <= vhi);
    const double gd = (ap_whole ? g : 0.0) + (surv ? ks : 0.0);
    if (gd != 0.0)
      atomicAdd(&dp[(int64_t)(W.ya + (q >> 6)) * fr.w + W.xa + (q & 63)],
                (float)gd);
  });
  for (int j = lane; j < ntk; j += kWave) {
    const int t = L.tk[j];
    const int px = W.xa + (t & 63), py = W.ya + ((t >> 6) & 63);
    const double k = (t >> 12) == 0 ? g : ks;
    atomicAdd(&dp[(int64_t)py * fr.w + px], (float)(k * L.tw[j]));
  }
  wave_lds_sync();
}

}  // namespace

template <int NS>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(3))) void k_aperture_bwd_t(
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

template __global__ void k_aperture_bwd_t<256>(
    Work, ipp_params, ipp_sources, const double*, const double*, double*);
template __global__ void k_aperture_bwd_t<512>(
    Work, ipp_params, ipp_sources, const double*, const double*, double*);
template __global__ void k_aperture_bwd_t<1024>(
    Work, ipp_params, ipp_sources, const double*, const double*, double*);

}  // namespace ipp
