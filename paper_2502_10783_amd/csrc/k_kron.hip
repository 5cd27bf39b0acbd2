// AUTO (Kron) photometry (Sec. 2.2.5 lists auto photometry among the
// per-object measurements; Sec. 3.3 compares its magnitudes).
//
// One wavefront per object, four objects per workgroup.  The object's
// second moments (x2, y2, xy), regularised by the variance 1/12 of a
// uniform unit pixel on each axis, give the quadratic form
//   q(dx, dy) = (Y dx^2 + X dy^2 - 2 xy dx dy) / det,  det = X Y - xy^2,
// (q = 1 on the one-sigma ellipse).  Pass 1: over the pixel centres with
// q <= search^2, r1 = sum sqrt(q) v / sum v (v = I - B32); the Kron radius
// is R = max(k r1, R_min), or R_min when the sums are unusable.  Pass 2:
// over the pixels of the ellipse q <= R^2, the AUTO flux sum w v and area
// sum w, w the exact pixel overlap: u = L d (L the upper Cholesky factor
// of the form / R^2) maps the ellipse onto the unit disk and the pixel
// onto a parallelogram, whose intersection with the disk is summed edge by
// edge (a triangle where an edge piece lies inside the disk, a circular
// sector where it lies outside), then divided by det L.  A pixel whose
// four corners lie inside the ellipse (q <= R^2 with a relative margin of
// 1e-12) is wholly inside it, its area exactly 1; only the other member
// pixels are listed (LDS) and then computed, every lane busy.  A window of
// more than kKronBigPx pixels (wide moments, or a large R where the first
// moment's weights nearly cancel) would hold one wavefront for hundreds or
// thousands of rounds: such a pass (with its pass 1 when the search window
// is the large one) is left to k_kron_big, which splits the window over a
// workgroup's waves and adds their sums in a fixed order.
//
// The membership tests (q against search^2, the frame bounds) use the
// same binary64 operations as the oracle; the sums are taken over the
// wavefront in a fixed order (deterministic, equal to the oracle's
// sequential sums to rounding).
#include "ipp_internal.h"
#include "kernels.h"
#include "phot_geom.h"

namespace ipp {

namespace {

__device__ __forceinline__ double qform(double X, double Y, double xy,
                                        double det, double dx, double dy) {
  return (Y * dx * dx + X * dy * dy - 2.0 * xy * dx * dy) / det;
}

// Smallest q over the square [x0, x1] x [y0, y1] of offsets: 0 when the
// centre lies in it, else the smallest edge minimum (the stationary point
// of q along the edge, clamped to it).
__device__ double min_q(double X, double Y, double xy, double det, double x0,
                        double x1, double y0, double y1) {
  if (x0 <= 0.0 && 0.0 <= x1 && y0 <= 0.0 && 0.0 <= y1) return 0.0;
  double best = __builtin_inf();
  const double xs[2] = {x0, x1}, ys[2] = {y0, y1};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double dx = xs[k];
    const double dy = fmin(fmax(xy * dx / X, y0), y1);
    best = fmin(best, qform(X, Y, xy, det, dx, dy));
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double dy = ys[k];
    const double dx = fmin(fmax(xy * dy / Y, x0), x1);
    best = fmin(best, qform(X, Y, xy, det, dx, dy));
  }
  return best;
}

// Signed area of the unit disk inside the triangle (0, a, b); sector
// angles from the atan series table coef.
__device__ double disk_tri(double ax, double ay, double bx, double by,
                           const double* coef) {
  const double dx = bx - ax, dy = by - ay;
  const double A = dx * dx + dy * dy;
  if (A == 0.0) return 0.0;
  const double B = ax * dx + ay * dy;
  const double C = ax * ax + ay * ay - 1.0;
  const double disc = B * B - A * C;
  double ts[4];
  int nt = 0;
  ts[nt++] = 0.0;
  if (disc > 0.0) {
    const double s = sqrt(disc);
    const double t0 = (-B - s) / A, t1 = (-B + s) / A;
    if (t0 > 0.0 && t0 < 1.0) ts[nt++] = t0;
    if (t1 > 0.0 && t1 < 1.0) ts[nt++] = t1;
  }
  ts[nt++] = 1.0;
  // (t0 <= t1 already, so the list is sorted)
  double area = 0.0;
  for (int k = 0; k + 1 < nt; ++k) {
    const double u0 = ts[k], u1 = ts[k + 1];
    const double px = ax + u0 * dx, py = ay + u0 * dy;
    const double qx = ax + u1 * dx, qy = ay + u1 * dy;
    const double mx = ax + 0.5 * (u0 + u1) * dx;
    const double my = ay + 0.5 * (u0 + u1) * dy;
    const double cr = px * qy - qx * py;
    if (mx * mx + my * my <= 1.0)
      area += 0.5 * cr;
    else
      area += 0.5 * angle_of(px * qx + py * qy, cr, coef);
  }
  return area;
}

struct Ell {
  double l11, l12, l22, inv_det;   // unit-disk map and 1 / det L
};

__device__ __forceinline__ Ell ell_map(double X, double Y, double xy,
                                       double det, double R) {
  const double s = det * R * R;
  const double a = Y / s, b = -xy / s, c = X / s;
  Ell e;
  e.l11 = sqrt(a);
  e.l12 = b / e.l11;
  e.l22 = sqrt(c - e.l12 * e.l12);
  e.inv_det = 1.0 / (e.l11 * e.l22);
  return e;
}

// Exact area of pixel (px, py) inside the ellipse centred at (cx, cy).
__device__ double ell_overlap(const Ell& e, double cx, double cy, int px,
                              int py, const double* coef) {
  const double x0 = (double)px - 0.5 - cx, x1 = (double)px + 0.5 - cx;
  const double y0 = (double)py - 0.5 - cy, y1 = (double)py + 0.5 - cy;
  // corners in counter-clockwise order for x right, y up: a positive sum
  const double ux[4] = {e.l11 * x0 + e.l12 * y0, e.l11 * x1 + e.l12 * y0,
                        e.l11 * x1 + e.l12 * y1, e.l11 * x0 + e.l12 * y1};
  const double uy[4] = {e.l22 * y0, e.l22 * y0, e.l22 * y1, e.l22 * y1};
  double a = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    a += disk_tri(ux[k], uy[k], ux[(k + 1) & 3], uy[(k + 1) & 3], coef);
  return a * e.inv_det;
}

constexpr int kCut = 1024;     // listed pixels per flush (a multiple of 64)
constexpr int kChunk = 4;      // rounds whose loads are issued together

__device__ __forceinline__ int lo_px(double v, int a) {
  return (int)fmax(ceil(v), (double)a);
}
__device__ __forceinline__ int hi_px(double v, int b) {
  return (int)fmin(floor(v), (double)b);
}

// A row's inputs: frame, centre and the moments regularised by the
// variance 1/12 of a uniform unit pixel; ok = all usable.
struct KronRow {
  int f;
  double cx, cy, X, Y, xy, det;
  bool ok;
};

__device__ __forceinline__ KronRow kron_row(const Work& wk,
                                            const ipp_sources& src,
                                            const double* mom,
                                            long long row) {
  KronRow r;
  r.f = src.frame[row];
  r.cx = src.x[row];
  r.cy = src.y[row];
  r.X = mom[6 * row] + 1.0 / 12.0;
  r.Y = mom[6 * row + 1] + 1.0 / 12.0;
  r.xy = mom[6 * row + 2];
  r.det = r.X * r.Y - r.xy * r.xy;
  r.ok = r.f >= 0 && r.f < wk.nframes && isfinite(r.X) && isfinite(r.Y) &&
         isfinite(r.xy) && r.det > 0.0 && isfinite(r.cx) && isfinite(r.cy) &&
         fabs(r.cx) < 1e9 && fabs(r.cy) < 1e9;
  return r;
}

// Pass-2 window: the Kron ellipse's bounding box within the frame and a
// ring of one pixel around it (an ellipse centred in the frame that reaches
// outside meets the ring: it is convex).
struct KronWin {
  int xa, ya, nwx, npx;
};

__device__ __forceinline__ KronWin kron_window(const FrameDev& fr,
                                               const KronRow& r, double R) {
  const double gx = R * sqrt(r.X), gy = R * sqrt(r.Y);
  const int xa = lo_px(r.cx - gx - 0.5, -1), xb = hi_px(r.cx + gx + 0.5, fr.w);
  const int ya = lo_px(r.cy - gy - 0.5, -1), yb = hi_px(r.cy + gy + 0.5, fr.h);
  KronWin k;
  k.xa = xa;
  k.ya = ya;
  k.nwx = max(xb - xa + 1, 0);
  k.npx = yb >= ya ? k.nwx * (yb - ya + 1) : 0;
  return k;
}

// Pass-1 window: the search ellipse's box within the frame.
__device__ __forceinline__ KronWin search_window(const FrameDev& fr,
                                                 const KronRow& r,
                                                 double search) {
  // bounds clamped in binary64 before the conversion to int
  const double hx = search * sqrt(r.X), hy = search * sqrt(r.Y);
  const int xa = lo_px(r.cx - hx - 0.5, 0), xb = hi_px(r.cx + hx + 0.5, fr.w - 1);
  const int ya = lo_px(r.cy - hy - 0.5, 0), yb = hi_px(r.cy + hy + 0.5, fr.h - 1);
  KronWin k;
  k.xa = xa;
  k.ya = ya;
  k.nwx = xb >= xa ? xb - xa + 1 : 0;
  k.npx = (xb >= xa && yb >= ya) ? k.nwx * (yb - ya + 1) : 0;
  return k;
}

// Pass 1 over search-window pixels [e_begin, e_end) (raster order): the
// sums sqrt(q) v and v over the pixel centres with q <= search^2 and a
// finite I; each lane sums its pixels in window order, the loads of kChunk
// rounds issued before any is used.
__device__ void kron_pass1(const FrameDev& fr, const KronRow& r,
                           double search, const KronWin& kw, int e_begin,
                           int e_end, int lane, double& num, double& den) {
  const int nwx = kw.nwx;
  if (nwx <= 0 || e_end <= e_begin) return;
  const double s2 = search * search;
  const int dwr = kWave / nwx, dwc = kWave - dwr * nwx;
  const int el0 = e_begin + lane;
  int wr = el0 / nwx, wc = el0 - (el0 / nwx) * nwx;
  for (int e0 = e_begin; e0 < e_end; e0 += kChunk * kWave) {
    float Iv[kChunk], Bv[kChunk];
    int pxs[kChunk], pys[kChunk];
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      const bool live = e0 + c * kWave + lane < e_end;
      pxs[c] = live ? kw.xa + wc : -1;
      pys[c] = kw.ya + wr;
      const int qx = live ? kw.xa + wc : kw.xa, qy = live ? kw.ya + wr : kw.ya;
      Iv[c] = fr.pix[(int64_t)qy * fr.pitch + qx];
      Bv[c] = fr.bkg[(int64_t)qy * fr.w + qx];
      wr += dwr;
      wc += dwc;
      if (wc >= nwx) {
        wc -= nwx;
        ++wr;
      }
    }
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      if (pxs[c] < 0) continue;
      const double q = qform(r.X, r.Y, r.xy, r.det, (double)pxs[c] - r.cx,
                             (double)pys[c] - r.cy);
      if (!(q <= s2)) continue;
      if (!isfinite(Iv[c])) continue;
      const double v = (double)Iv[c] - (double)Bv[c];
      num += sqrt(q) * v;
      den += v;
    }
  }
}

// The Kron radius from the first-moment sums (flag 2: R_min used).
__device__ __forceinline__ double kron_radius(double num, double den,
                                              double kfac, double rmin,
                                              uint32_t* fl) {
  const double r1 = den > 0.0 ? num / den : __builtin_nan("");
  if (den > 0.0 && isfinite(r1)) {
    const double R = kfac * r1;
    return R > rmin ? R : rmin;
  }
  *fl |= 2u;
  return rmin;
}

// Pass 2 over window pixels [e_begin, e_end) (raster order): members of
// the open ellipse whose four corners lie inside it add v and area 1, the
// other members are listed and add w v and w, w the exact overlap; a
// member off the frame or not finite sets edge.  Membership is the exact
// predicate min_q < R^2, but most pixels are settled by their centre
// without it: min_q <= q(centre), and sqrt(min_q) >= sqrt(q(centre)) - m
// with m the largest sqrt(q) of a half-pixel corner offset, so a centre
// with q below R^2 (1 - 1e-9) is a member and one above (R + m)^2
// (1 + 1e-9) is not (margins no rounding here can cross); the pixels in
// between (a band along the boundary) are listed and tested exactly, all
// lanes busy.  Per chunk of kCut / 2 window pixels the band is listed
// from the back of `cut`, the cut members from its front.  Each lane
// accumulates the settled members in window order, then the band's, then
// the cut ones; the pixel loads of kChunk rounds are issued before any is
// used (clamped into the frame; only members use them).
__device__ void kron_pass2(const FrameDev& fr, const KronRow& r,
                           const Ell& el, double R, const KronWin& kw,
                           int e_begin, int e_end, int lane, int* cut,
                           const double* atan_lds, double& fs, double& as,
                           bool& edge) {
  const double X = r.X, Y = r.Y, xy = r.xy, det = r.det;
  const double cx = r.cx, cy = r.cy;
  const double R2 = R * R;
  // corners inside: q det <= R^2 det (1 - 1e-12), no division
  const double lim = R2 * det * (1.0 - 1e-12);
  const double m = sqrt(0.25 * (X + Y + 2.0 * fabs(xy)) / det);
  const double lim_in = R2 * det * (1.0 - 1e-9);
  const double lim_out = (R + m) * (R + m) * det * (1.0 + 1e-9);
  auto qd = [&](double dx, double dy) {
    return Y * dx * dx + X * dy * dy - 2.0 * xy * dx * dy;
  };
  // a member pixel with its loaded values: edge, a whole pixel, or listed
  auto member = [&](int px, int py, float I, float B, int pos, bool* listed,
                    int* lpos) {
    const bool in = px >= 0 && px < fr.w && py >= 0 && py < fr.h;
    if (!in || !isfinite(I)) {
      edge = true;
      return;
    }
    const double x0 = (double)px - 0.5 - cx, x1 = (double)px + 0.5 - cx;
    const double y0 = (double)py - 0.5 - cy, y1 = (double)py + 0.5 - cy;
    if (qd(x0, y0) <= lim && qd(x1, y0) <= lim && qd(x0, y1) <= lim &&
        qd(x1, y1) <= lim) {
      fs += (double)I - (double)B;
      as += 1.0;
    } else {
      *listed = true;
      *lpos = pos;
    }
  };
  const int nwx = kw.nwx;
  if (nwx <= 0 || e_end <= e_begin) return;
  // window positions stepped round by round without division
  const int dwr = kWave / nwx, dwc = kWave - dwr * nwx;
  const int el0 = e_begin + lane;
  int sy = el0 / nwx, sx = el0 - (el0 / nwx) * nwx;
  constexpr int kPart = kCut / 2;      // window pixels per chunk
  for (int e0 = e_begin; e0 < e_end; e0 += kPart) {
    int ncut = 0, nband = 0;
    const int e1 = min(e_end, e0 + kPart);
    for (int eb = e0; eb < e1; eb += kChunk * kWave) {
      float Iv[kChunk], Bv[kChunk];
      int wys[kChunk], wxs[kChunk];
#pragma unroll
      for (int c = 0; c < kChunk; ++c) {
        if (eb + c * kWave >= e1) break;             // wave-uniform
        wys[c] = sy;
        wxs[c] = sx;
        const int qx = min(max(kw.xa + sx, 0), fr.w - 1);
        const int qy = min(max(kw.ya + sy, 0), fr.h - 1);
        Iv[c] = fr.pix[(int64_t)qy * fr.pitch + qx];
        Bv[c] = fr.bkg[(int64_t)qy * fr.w + qx];
        sy += dwr;
        sx += dwc;
        if (sx >= nwx) {
          sx -= nwx;
          ++sy;
        }
      }
#pragma unroll
      for (int c = 0; c < kChunk; ++c) {
        if (eb + c * kWave >= e1) break;             // wave-uniform
        const int e = eb + c * kWave + lane;
        bool listed = false, band = false;
        int pos = 0;
        if (e < e1) {
          const int wy = wys[c], wx = wxs[c];
          const int py = kw.ya + wy, px = kw.xa + wx;
          pos = (wy << 16) | wx;
          const double qc = qd((double)px - cx, (double)py - cy);
          if (qc <= lim_in) {
            int lp = 0;
            member(px, py, Iv[c], Bv[c], pos, &listed, &lp);
          } else {
            band = !(qc >= lim_out);
          }
        }
        const uint64_t bb = ballot(band);
        if (band) cut[kCut - 1 - (nband + lanes_before(bb))] = pos;
        nband += __popcll(bb);
        const uint64_t b = ballot(listed);
        if (listed) cut[ncut + lanes_before(b)] = pos;
        ncut += __popcll(b);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the band: the exact predicate, then as any member
    for (int j0 = 0; j0 < nband; j0 += kWave) {
      const int j = j0 + lane;
      bool listed = false;
      int pos = 0;
      if (j < nband) {
        const int t = cut[kCut - 1 - j];
        const int wx = t & 0xFFFF, wy = t >> 16;
        const int px = kw.xa + wx, py = kw.ya + wy;
        const double x0 = (double)px - 0.5 - cx, x1 = (double)px + 0.5 - cx;
        const double y0 = (double)py - 0.5 - cy, y1 = (double)py + 0.5 - cy;
        if (min_q(X, Y, xy, det, x0, x1, y0, y1) < R2) {
          const bool in = px >= 0 && px < fr.w && py >= 0 && py < fr.h;
          float I = 0.0f, B = 0.0f;
          if (in) {
            I = fr.pix[(int64_t)py * fr.pitch + px];
            B = fr.bkg[(int64_t)py * fr.w + px];
          }
          member(px, py, I, B, t, &listed, &pos);
        }
      }
      const uint64_t b = ballot(listed);
      if (listed) cut[ncut + lanes_before(b)] = pos;
      ncut += __popcll(b);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int j = lane; j < ncut; j += kWave) {
      int co = 0;
      asm volatile("" : "+s"(co));
      const double* coef = atan_lds + co;
      const int t = cut[j];
      const int px = kw.xa + (t & 0xFFFF), py = kw.ya + (t >> 16);
      const double w = ell_overlap(el, cx, cy, px, py, coef);
      const double v = (double)fr.pix[(int64_t)py * fr.pitch + px] -
                       (double)fr.bkg[(int64_t)py * fr.w + px];
      fs += w * v;
      as += w;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_kron(Work wk, ipp_sources src,
                                                 const double* mom,
                                                 double kfac, double rmin,
                                                 double search, double* kron,
                                                 double* flux, double* area,
                                                 uint32_t* flags) {
  // pixels of the Kron ellipse cut by its boundary: py << 16 | px offsets
  // from the window corner, per wave
  __shared__ int cut_lds[kWaves][kCut];
  __shared__ double atan_lds[kAtanTerms];
  if (threadIdx.x < kAtanTerms) atan_lds[threadIdx.x] = atan_coef(threadIdx.x);
  __syncthreads();
  int* cut = cut_lds[threadIdx.x / kWave];
  const int lane = threadIdx.x & (kWave - 1);
  long long nrows = src.capacity;
  if (src.n_total && *src.n_total < nrows) nrows = *src.n_total;
  const long long wid =
      blockIdx.x * (long long)kWaves +
      __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const long long nw = (long long)gridDim.x * kWaves;
  for (long long row = wid; row < nrows; row += nw) {
    const KronRow r = kron_row(wk, src, mom, row);
    if (!r.ok) {
      if (lane == 0) {
        kron[row] = __builtin_nan("");
        flux[row] = __builtin_nan("");
        area[row] = 0.0;
        flags[row] = 1u;                               // bad shape
      }
      continue;
    }
    const double cx = r.cx, cy = r.cy, X = r.X, Y = r.Y, xy = r.xy;
    const double det = r.det;
    const FrameDev fr = wk.frames[r.f];
    uint32_t fl = 0;
    // ---- pass 1: first moment over the search ellipse ------------------
    const KronWin sw = search_window(fr, r, search);
    if (sw.npx > kKronBigPx) continue;     // the whole row is k_kron_big's
    double num = 0.0, den = 0.0;
    kron_pass1(fr, r, search, sw, 0, sw.npx, lane, num, den);
    num = wave_sum(num);
    den = wave_sum(den);
    const double R = kron_radius(num, den, kfac, rmin, &fl);
    // ---- pass 2: exact overlaps with the Kron ellipse -------------------
    // (one centred outside the frame is flagged outright)
    if (!(cx >= -0.5 && cx <= (double)fr.w - 0.5 && cy >= -0.5 &&
          cy <= (double)fr.h - 0.5))
      fl |= 4u;
    const KronWin kw = kron_window(fr, r, R);
    if (kw.npx > kKronBigPx) {
      // a window this large is summed by k_kron_big, a workgroup at once
      if (lane == 0) {
        kron[row] = R;
        flags[row] = fl;
      }
      continue;
    }
    const Ell el = ell_map(X, Y, xy, det, R);
    double fs = 0.0, as = 0.0;
    bool edge = false;
    kron_pass2(fr, r, el, R, kw, 0, kw.npx, lane, cut, atan_lds, fs, as,
               edge);
    fs = wave_sum(fs);
    as = wave_sum(as);
    if (__builtin_amdgcn_ballot_w64(edge)) fl |= 4u;    // off the frame
    if (lane == 0) {
      kron[row] = R;
      flux[row] = fs;
      area[row] = as;
      flags[row] = fl;
    }
  }
}

// The rows k_kron left: those whose search window holds more than
// kKronBigPx pixels (both passes here) and those whose Kron ellipse window
// does (pass 2 here, with the radius k_kron wrote).  Each workgroup checks
// kBigThreads rows at once (one per thread), then takes each such row with
// all its waves, wave k summing the k-th of kBigWaves equal parts of a
// window; the parts' sums are added in wave order.
__global__ __launch_bounds__(kBigThreads) void k_kron_big(
    Work wk, ipp_sources src, const double* mom, double kfac, double rmin,
    double search, double* kron, double* flux, double* area,
    uint32_t* flags) {
  constexpr int kBigWaves = kBigThreads / kWave;
  __shared__ int cut_lds[kBigWaves][kCut];
  __shared__ double atan_lds[kAtanTerms];
  __shared__ int list[kBigThreads];
  __shared__ int nlist;
  __shared__ double part[kBigWaves][2];
  __shared__ int pedge[kBigWaves];
  if (threadIdx.x < kAtanTerms) atan_lds[threadIdx.x] = atan_coef(threadIdx.x);
  if (threadIdx.x == 0) nlist = 0;
  __syncthreads();
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = threadIdx.x & (kWave - 1);
  int* cut = cut_lds[wv];
  long long nrows = src.capacity;
  if (src.n_total && *src.n_total < nrows) nrows = *src.n_total;
  // the parts of a window: [eb, ee) of its npx pixels for this wave, and
  // the sum of two per-wave values over the waves in wave order
  auto share = [&](int npx, int* eb, int* ee) {
    const int per = (npx + kBigWaves - 1) / kBigWaves;
    *eb = min(npx, wv * per);
    *ee = min(npx, *eb + per);
  };
  auto combine = [&](double p0, double p1, bool e, double* s0, double* s1,
                     bool* any) {
    p0 = wave_sum(p0);
    p1 = wave_sum(p1);
    const bool ae = __builtin_amdgcn_ballot_w64(e) != 0;
    if (lane == 0) {
      part[wv][0] = p0;
      part[wv][1] = p1;
      pedge[wv] = ae ? 1 : 0;
    }
    __syncthreads();
    double t0 = 0.0, t1 = 0.0;
    int ed = 0;
    for (int k = 0; k < kBigWaves; ++k) {
      t0 += part[k][0];
      t1 += part[k][1];
      ed |= pedge[k];
    }
    __syncthreads();                  // read before the next use
    *s0 = t0;
    *s1 = t1;
    *any = ed != 0;
  };
  for (long long base = blockIdx.x * (long long)kBigThreads; base < nrows;
       base += (long long)gridDim.x * kBigThreads) {
    {
      const long long row = base + threadIdx.x;
      bool big = false;
      if (row < nrows) {
        const KronRow r = kron_row(wk, src, mom, row);
        if (r.ok) {
          const FrameDev& fr = wk.frames[r.f];
          big = search_window(fr, r, search).npx > kKronBigPx ||
                kron_window(fr, r, kron[row]).npx > kKronBigPx;
        }
      }
      if (big) list[atomicAdd(&nlist, 1)] = (int)threadIdx.x;
    }
    __syncthreads();
    const int nb = nlist;
    __syncthreads();                  // every thread has read the count
    for (int i = 0; i < nb; ++i) {
      const long long row = base + list[i];
      const KronRow r = kron_row(wk, src, mom, row);
      const FrameDev fr = wk.frames[r.f];
      const KronWin sw = search_window(fr, r, search);
      const bool both = sw.npx > kKronBigPx;
      uint32_t fl = 0;
      double R;
      int eb, ee;
      bool e_unused;
      if (both) {
        double num = 0.0, den = 0.0;
        share(sw.npx, &eb, &ee);
        kron_pass1(fr, r, search, sw, eb, ee, lane, num, den);
        combine(num, den, false, &num, &den, &e_unused);
        R = kron_radius(num, den, kfac, rmin, &fl);
        if (!(r.cx >= -0.5 && r.cx <= (double)fr.w - 0.5 && r.cy >= -0.5 &&
              r.cy <= (double)fr.h - 0.5))
          fl |= 4u;
      } else {
        R = kron[row];                 // k_kron wrote R and the flags
      }
      const KronWin kw = kron_window(fr, r, R);
      const Ell el = ell_map(r.X, r.Y, r.xy, r.det, R);
      double fs = 0.0, as = 0.0;
      bool edge = false;
      share(kw.npx, &eb, &ee);
      kron_pass2(fr, r, el, R, kw, eb, ee, lane, cut, atan_lds, fs, as,
                 edge);
      bool any_edge;
      combine(fs, as, edge, &fs, &as, &any_edge);
      if (threadIdx.x == 0) {
        if (any_edge) fl |= 4u;                         // off the frame
        if (both) {
          kron[row] = R;
          flags[row] = fl;
        } else {
          flags[row] |= fl;
        }
        flux[row] = fs;
        area[row] = as;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) nlist = 0;
    __syncthreads();
  }
}

}  // namespace ipp
