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
// pixels are listed (LDS) and then computed, every lane busy.
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

}  // namespace

__global__ __launch_bounds__(kBlock) void k_kron(Work wk, ipp_sources src,
                                                 const double* mom,
                                                 double kfac, double rmin,
                                                 double search, double* kron,
                                                 double* flux, double* area,
                                                 uint32_t* flags) {
  // pixels of the Kron ellipse cut by its boundary: py << 16 | px offsets
  // from the window corner, per wave
  constexpr int kCut = 1024;            // a multiple of 64
  constexpr int kChunk = 4;
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
    const int f = src.frame[row];
    const double cx = src.x[row], cy = src.y[row];
    const double X = mom[6 * row] + 1.0 / 12.0;
    const double Y = mom[6 * row + 1] + 1.0 / 12.0;
    const double xy = mom[6 * row + 2];
    const double det = X * Y - xy * xy;
    const bool ok = f >= 0 && f < wk.nframes && isfinite(X) &&
                    isfinite(Y) && isfinite(xy) && det > 0.0 &&
                    isfinite(cx) && isfinite(cy) && fabs(cx) < 1e9 &&
                    fabs(cy) < 1e9;
    if (!ok) {
      if (lane == 0) {
        kron[row] = __builtin_nan("");
        flux[row] = __builtin_nan("");
        area[row] = 0.0;
        flags[row] = 1u;                               // bad shape
      }
      continue;
    }
    const FrameDev fr = wk.frames[f];
    uint32_t fl = 0;
    // ---- pass 1: first moment over the search ellipse ------------------
    // window bounds clamped in binary64 before the conversion to int
    auto lo = [](double v, int a) { return (int)fmax(ceil(v), (double)a); };
    auto hi = [](double v, int b) { return (int)fmin(floor(v), (double)b); };
    const double hx = search * sqrt(X), hy = search * sqrt(Y);
    const int xa = lo(cx - hx - 0.5, 0), xb = hi(cx + hx + 0.5, fr.w - 1);
    const int ya = lo(cy - hy - 0.5, 0), yb = hi(cy + hy + 0.5, fr.h - 1);
    double num = 0.0, den = 0.0;
    const double s2 = search * search;
    if (xb >= xa && yb >= ya) {
      // the window (inside the frame) in rounds of 64 pixels, positions
      // stepped without division, the loads of kChunk rounds issued before
      // any is used; each lane sums its pixels in window order
      const int nwx = xb - xa + 1;
      const int npx = nwx * (yb - ya + 1);
      const int dwr = kWave / nwx, dwc = kWave - dwr * nwx;
      int wr = lane / nwx, wc = lane - (lane / nwx) * nwx;
      for (int e0 = 0; e0 < npx; e0 += kChunk * kWave) {
        float Iv[kChunk], Bv[kChunk];
        int pxs[kChunk], pys[kChunk];
#pragma unroll
        for (int c = 0; c < kChunk; ++c) {
          const bool live = e0 + c * kWave + lane < npx;
          pxs[c] = live ? xa + wc : -1;
          pys[c] = ya + wr;
          const int qx = live ? xa + wc : xa, qy = live ? ya + wr : ya;
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
          const double q = qform(X, Y, xy, det, (double)pxs[c] - cx,
                                 (double)pys[c] - cy);
          if (!(q <= s2)) continue;
          if (!isfinite(Iv[c])) continue;
          const double v = (double)Iv[c] - (double)Bv[c];
          num += sqrt(q) * v;
          den += v;
        }
      }
    }
    num = wave_sum(num);
    den = wave_sum(den);
    const double r1 = den > 0.0 ? num / den : __builtin_nan("");
    double R;
    if (den > 0.0 && isfinite(r1)) {
      R = kfac * r1;
      R = R > rmin ? R : rmin;
    } else {
      R = rmin;
      fl |= 2u;                                        // R_min used
    }
    // ---- pass 2: exact overlaps with the Kron ellipse -------------------
    const Ell el = ell_map(X, Y, xy, det, R);
    // the frame and a ring of one pixel around it: an ellipse centred in
    // the frame that reaches outside meets the ring (it is convex); one
    // centred outside is flagged outright
    const double gx = R * sqrt(X), gy = R * sqrt(Y);
    const int xa2 = lo(cx - gx - 0.5, -1), xb2 = hi(cx + gx + 0.5, fr.w);
    const int ya2 = lo(cy - gy - 0.5, -1), yb2 = hi(cy + gy + 0.5, fr.h);
    if (!(cx >= -0.5 && cx <= (double)fr.w - 0.5 && cy >= -0.5 &&
          cy <= (double)fr.h - 0.5))
      fl |= 4u;
    const int nwx2 = max(xb2 - xa2 + 1, 0);
    const int npx2 = yb2 >= ya2 ? nwx2 * (yb2 - ya2 + 1) : 0;
    double fs = 0.0, as = 0.0;
    bool edge = false;
    const double R2 = R * R;
    // corners inside: q det <= R^2 det (1 - 1e-12), no division
    const double lim = R2 * det * (1.0 - 1e-12);
    // members wholly inside are summed here, the others listed, in chunks
    // of kCut pixels of the window (so that the list cannot overflow)
    // window positions stepped round by round without division
    const int dwr2 = nwx2 > 0 ? kWave / nwx2 : 0;
    const int dwc2 = kWave - dwr2 * nwx2;
    int sy = nwx2 > 0 ? lane / nwx2 : 0, sx = lane - sy * nwx2;
    for (int e0 = 0; e0 < npx2; e0 += kCut) {
      int ncut = 0;
      const int e1 = min(npx2, e0 + kCut);
      for (int eb = e0; eb < e1; eb += kWave) {
        const int e = eb + lane;
        bool listed = false;
        int pos = 0;
        const int wy = sy, wx = sx;          // this round's position
        sy += dwr2;
        sx += dwc2;
        if (sx >= nwx2) {
          sx -= nwx2;
          ++sy;
        }
        if (e < e1) {
          const int py = ya2 + wy, px = xa2 + wx;
          const double x0 = (double)px - 0.5 - cx, x1 = (double)px + 0.5 - cx;
          const double y0 = (double)py - 0.5 - cy, y1 = (double)py + 0.5 - cy;
          // the pixel meets the open ellipse: an exact predicate
          if (min_q(X, Y, xy, det, x0, x1, y0, y1) < R2) {
            const bool in = px >= 0 && px < fr.w && py >= 0 && py < fr.h;
            float I = 0.0f;
            if (in) I = fr.pix[(int64_t)py * fr.pitch + px];
            if (!in || !isfinite(I)) {
              edge = true;
            } else {
              auto qd = [&](double dx, double dy) {
                return Y * dx * dx + X * dy * dy - 2.0 * xy * dx * dy;
              };
              if (qd(x0, y0) <= lim && qd(x1, y0) <= lim &&
                  qd(x0, y1) <= lim && qd(x1, y1) <= lim) {
                const double v =
                    (double)I - (double)fr.bkg[(int64_t)py * fr.w + px];
                fs += v;
                as += 1.0;
              } else {
                listed = true;
                pos = (wy << 16) | wx;
              }
            }
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
        const int px = xa2 + (t & 0xFFFF), py = ya2 + (t >> 16);
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

}  // namespace ipp
