// Exact circle/pixel overlap geometry in binary64 for aperture photometry.
//
// The signed corner integral G(x, y) = int_0^x int_0^y [s^2+t^2 <= r^2] of
// a disk of radius r about the origin is odd in x and in y; for
// 0 <= x, y <= r it is x*y when the corner lies in the circle and otherwise
// y*xs + P(x) - P(xs) with xs = sqrt(r^2 - y^2) and
// P(s) = int_0^s sqrt(r^2 - u^2) du = (s sqrt(r^2 - s^2) + r^2 asin(s/r))/2
// (its angle term evaluated as the angle of a rotation, see corner_g).
// A pixel's overlap is the inclusion-exclusion of G over its corners; for
// r >= 3/4 the four angle terms are summed as one rotation and recovered by
// a single angle evaluation (see corner_rot).  Angles come from the
// Maclaurin series of atan, its coefficients read from a table in LDS, after
// argument halvings where the argument is large: no library call, so no
// constant of a library routine is kept in registers.
// Inside the overlap formulas products may fuse with the additions that
// take them (one rounding fewer; the corner's in/out choice there selects
// between two forms of G that agree on the circle).  Membership (the pixel
// square meets the open disk) and full containment are decided by the
// exact predicates below, formed as written, so that every pixel that a
// rounding residue could move in or out is classified the same way on
// every device.  dG/dx(x, y) = sign(y) min(|y|, sqrt(r^2 - x^2)) gives the
// derivative of an overlap with respect to the disk centre.
#pragma once

#include <hip/hip_runtime.h>

namespace ipp {

__device__ __forceinline__ bool touches(double cx, double cy, double r,
                                        int px, int py) {
  const double dx = fmax(fabs((double)px - cx) - 0.5, 0.0);
  const double dy = fmax(fabs((double)py - cy) - 0.5, 0.0);
  return dx * dx + dy * dy < r * r;
}

__device__ __forceinline__ bool within(double cx, double cy, double r,
                                       int px, int py) {
  const double fx = fabs((double)px - cx) + 0.5;
  const double fy = fabs((double)py - cy) + 0.5;
  return fx * fx + fy * fy <= r * r;
}

// Coefficients of the Maclaurin series of atan through the power 33:
// (-1)^k / (2k + 1), k = 0..16.
constexpr int kAtanTerms = 17;
__device__ __forceinline__ double atan_coef(int k) {
  return (k & 1 ? -1.0 : 1.0) / (double)(2 * k + 1);
}

// atan(t) for |t| <= 0.3 from the series (coefficient table coef): the
// first term left out is below 2e-20 relative.
__device__ __forceinline__ double atan_series(double t, const double* coef) {
  // all coefficients requested before the first is used: one wait for the
  // table instead of one per term
  double c[kAtanTerms];
#pragma unroll
  for (int k = 0; k < kAtanTerms; ++k) c[k] = coef[k];
  const double t2 = t * t;
  double s = c[kAtanTerms - 1];
#pragma unroll
  for (int k = kAtanTerms - 2; k >= 0; --k) s = fma(s, t2, c[k]);
  return t * s;
}

// atan(t) for |t| <= 1: two halvings atan t = 2 atan(t / (1 + sqrt(1 + t^2)))
// bring the argument below tan(pi/16) < 0.2, then the series.
__device__ __forceinline__ double atan_unit(double t, const double* coef) {
  t = t / (1.0 + sqrt(fma(t, t, 1.0)));
  t = t / (1.0 + sqrt(fma(t, t, 1.0)));
  return 4.0 * atan_series(t, coef);
}

// Angle in (-pi, pi] of the direction (c, s), c and s not both zero.
__device__ __forceinline__ double angle_of(double c, double s,
                                           const double* coef) {
  constexpr double kHalfPi = 1.5707963267948966;
  constexpr double kPi = 3.141592653589793;
  const double ac = fabs(c), as = fabs(s);
  double a = as <= ac ? atan_unit(as / ac, coef)
                      : kHalfPi - atan_unit(ac / as, coef);
  if (c < 0.0) a = kPi - a;
  return s < 0.0 ? -a : a;
}

// G for a corner (x, y) outside the circle, 0 <= x, y <= r, with
// xs = sqrt(r^2 - y^2) and hx = sqrt(r^2 - x^2):
//   G = y xs + P(x) - P(xs)
//     = (y xs + x hx + r^2 (asin(x/r) - asin(xs/r))) / 2.
// With a = asin(x/r) and b = asin(y/r) the angle asin(x/r) - asin(xs/r) is
// a + b - pi/2, whose direction (cos, sin) is proportional to
// (hx y + x xs, x y - xs hx): the cosine is a sum of non-negative products,
// so the angle of the pair is accurate up to the right angle, where asin of
// the sine alone would lose half its digits.  The two square roots depend
// on one coordinate each, so a pixel needs four.
__device__ __forceinline__ double corner_g(double ax, double ay, double hx,
                                           double xs, double r2,
                                           const double* coef) {
#pragma clang fp contract(fast)
  if (ax * ax + ay * ay <= r2) return ax * ay;
  const double c = hx * ay + ax * xs;
  const double s = ax * ay - xs * hx;
  return 0.5 * ((ay * xs + ax * hx) + r2 * angle_of(c, s, coef));
}

// The same corner as a rotation: corner_rot adds the corner's non-angular
// part to lin and turns (re, im) by the corner's signed angle; a corner in
// the circle has no angle term.  After all four corners the summed angle is
// the arc of the circle that lies inside the pixel, and lin plus r^2/2 times
// that angle is the overlap.  The factors are left unnormalised (length
// r^2 each); the angle does not depend on the length.
__device__ __forceinline__ void corner_rot(double ax, double ay, double hx,
                                           double xs, double sig, double r2,
                                           double& lin, double& re,
                                           double& im) {
#pragma clang fp contract(fast)
  const bool out = ax * ax + ay * ay > r2;
  const double c = hx * ay + ax * xs;
  const double s = sig * (ax * ay - xs * hx);
  lin = fma(sig, out ? 0.5 * (ay * xs + ax * hx) : ax * ay, lin);
  const double cc = out ? c : 1.0, ss = out ? s : 0.0;
  const double nre = re * cc - im * ss;
  im = fma(re, ss, im * cc);
  re = nre;
}

// Angle in [0, pi) of the rotation (re, im) (im >= 0, not both zero): the
// series of atan(im / re) once |im| <= 0.3 re, which holds at once for
// every cut pixel of a circle of radius 5 or more.  A larger angle is
// first turned back by a right angle if it exceeds one ((re, im) ->
// (im, -re), so that re > 0), then halved until it qualifies: (re, im) ->
// (re + |(re, im)|, im) halves the angle of a vector with re > 0 without
// cancellation (at most four halvings from below a right angle).  Every
// lane evaluates the series once, whichever path it took.
__device__ __forceinline__ double rotor_angle(double re, double im,
                                              const double* coef) {
  constexpr double kHalfPi = 1.5707963267948966;
  double base = 0.0, scale = 1.0;
  if (!(fabs(im) <= 0.3 * re)) {
    if (re < 0.0) {
      const double t = re;
      re = im;
      im = -t;
      base = kHalfPi;
    }
    do {
      re = re + sqrt(fma(re, re, im * im));
      scale = 2.0 * scale;
    } while (!(fabs(im) <= 0.3 * re));
  }
  return fma(scale, atan_series(im / re, coef), base);
}

// Overlap of the pixel square [px-1/2, px+1/2] x [py-1/2, py+1/2] with the
// disk of radius r about (cx, cy), for a square that meets the disk and is
// not inside it: inclusion-exclusion of G over the square's corners, given
// the four square roots hx0/hx1 = sqrt(r^2 - min(|x|, r)^2) at the left /
// right edge and xs0/xs1 likewise at the bottom / top edge.
// The arc of a circle inside a unit square is below half the circle once
// 2r exceeds the square's diagonal (an arc of half the circle or more holds
// two antipodal points), so for r >= 3/4 the summed corner angle lies in
// [0, pi) and one angle of the composed rotation returns it; smaller
// circles, whose arc inside one pixel can reach the whole circle, take one
// angle per corner.  coef: the atan series coefficients (atan_coef).
__device__ __forceinline__ double overlap_cut(double cx, double cy, double r,
                                              double r2, int px, int py,
                                              double hx0, double hx1,
                                              double xs0, double xs1,
                                              const double* coef) {
#pragma clang fp contract(fast)
  const double x0 = ((double)px - 0.5) - cx, x1 = ((double)px + 0.5) - cx;
  const double y0 = ((double)py - 0.5) - cy, y1 = ((double)py + 0.5) - cy;
  const double ax0 = fmin(fabs(x0), r), ax1 = fmin(fabs(x1), r);
  const double ay0 = fmin(fabs(y0), r), ay1 = fmin(fabs(y1), r);
  const double sx0 = x0 < 0.0 ? -1.0 : 1.0, sx1 = x1 < 0.0 ? -1.0 : 1.0;
  const double sy0 = y0 < 0.0 ? -1.0 : 1.0, sy1 = y1 < 0.0 ? -1.0 : 1.0;
  if (r >= 0.75) {
    // the first corner's rotation is the corner's own (1 times it)
    double lin, re, im;
    {
      const double sig = sx1 * sy1;
      const bool out = ax1 * ax1 + ay1 * ay1 > r2;
      lin = sig * (out ? 0.5 * (ay1 * xs1 + ax1 * hx1) : ax1 * ay1);
      re = out ? hx1 * ay1 + ax1 * xs1 : 1.0;
      im = out ? sig * (ax1 * ay1 - xs1 * hx1) : 0.0;
    }
    corner_rot(ax0, ay1, hx0, xs1, -(sx0 * sy1), r2, lin, re, im);
    corner_rot(ax1, ay0, hx1, xs0, -(sx1 * sy0), r2, lin, re, im);
    corner_rot(ax0, ay0, hx0, xs0, sx0 * sy0, r2, lin, re, im);
    return fma(0.5 * r2, rotor_angle(re, im, coef), lin);
  }
  return sx1 * sy1 * corner_g(ax1, ay1, hx1, xs1, r2, coef) -
         sx0 * sy1 * corner_g(ax0, ay1, hx0, xs1, r2, coef) -
         sx1 * sy0 * corner_g(ax1, ay0, hx1, xs0, r2, coef) +
         sx0 * sy0 * corner_g(ax0, ay0, hx0, xs0, r2, coef);
}

// Square root term of one pixel edge at offset q from the centre.
__device__ __forceinline__ double edge_root(double q, double r, double r2) {
  const double a = fmin(fabs(q), r);
  return sqrt(fmax(r2 - a * a, 0.0));
}

// (d/dcx, d/dcy) of the overlap of pixel (px, py) with the disk of radius
// r about (cx, cy), from the pixel's four edge roots (as for overlap_cut):
// the chord at an edge x is sign(y) min(|y|, sqrt(r^2 - x^2)).
__device__ __forceinline__ void overlap_grad_roots(double cx, double cy,
                                                   int px, int py,
                                                   double hx0, double hx1,
                                                   double xs0, double xs1,
                                                   double* gx, double* gy) {
  const double x0 = ((double)px - 0.5) - cx, x1 = ((double)px + 0.5) - cx;
  const double y0 = ((double)py - 0.5) - cy, y1 = ((double)py + 0.5) - cy;
  auto ch = [](double h, double y) { return copysign(fmin(fabs(y), h), y); };
  *gx = -(ch(hx1, y1) - ch(hx0, y1) - ch(hx1, y0) + ch(hx0, y0));
  *gy = -(ch(xs1, x1) - ch(xs0, x1) - ch(xs1, x0) + ch(xs0, x0));
}

}  // namespace ipp
