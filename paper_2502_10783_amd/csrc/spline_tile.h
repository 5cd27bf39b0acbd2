// Evaluation of the tensor-product natural cubic spline background and rms
// (Sec. 2.2.2: spline interpolation of the filtered mesh back to the full
// resolution) over one detection tile.
//
// With per-node tables f, fxx (second derivative along x), fyy and fxxyy,
// the spline restricted to an image row y is a 1-D natural spline in x
// through the values g_i(y) with second derivatives g''_i(y), where g_i and
// g''_i are 1-D splines in y of the node columns of (f, fyy) and
// (fxx, fxxyy).  The tile prologue stages the few mesh nodes the tile
// spans in LDS, evaluates g and g'' per tile row for those mesh columns,
// and the per-column x weights; each pixel is then four multiply-adds per
// map.
#pragma once

#include "ipp_internal.h"

namespace ipp {

// A tile of TW columns spans at most (TW-1)/16 + 2 mesh intervals for
// meshes >= 16 px (only the last interval of a frame is shorter than the
// mesh, and it is at least half a mesh long), so its columns use mesh
// columns ilo .. ilo + TW/16 + 2; likewise for rows.
template <int TH, int TW>
struct SplineLds {
  static constexpr int NC = TW / 16 + 3;
  static constexpr int NR = TH / 16 + 3;
  double gB[TH][NC];
  double gBpp[TH][NC];
  double gR[TH][NC];
  double gRpp[TH][NC];
  double wx[4][TW];            // x weights, structure of arrays
  int cx[TW];
  double wy[TH][4];
  int ry[TH];
  double node[8][NR][NC];      // tb[0..3], tr[0..3] of the spanned nodes
};

template <int TH, int TW, int NT = kBlock>
__device__ __forceinline__ void spline_prologue(const Work& wk,
                                                const FrameDev& fr,
                                                const ipp_params& p, int y0,
                                                int x0,
                                                SplineLds<TH, TW>& S) {
  constexpr int NC = SplineLds<TH, TW>::NC;
  constexpr int NR = SplineLds<TH, TW>::NR;
  int ilo, jlo;
  {
    double w4[4];
    spline_weights((double)x0, p.mesh_w, fr.w, fr.nx, &ilo, w4);
    spline_weights((double)y0, p.mesh_h, fr.h, fr.ny, &jlo, w4);
  }
  for (int c = threadIdx.x; c < TW + TH; c += NT) {
    double w4[4];
    int j;
    if (c < TW) {
      spline_weights((double)(x0 + c), p.mesh_w, fr.w, fr.nx, &j, w4);
      S.cx[c] = min(j - ilo, NC - 2);
#pragma unroll
      for (int k = 0; k < 4; ++k) S.wx[k][c] = w4[k];
    } else {
      const int r = c - TW;
      const int y = min(y0 + r, fr.h - 1);
      spline_weights((double)y, p.mesh_h, fr.h, fr.ny, &j, w4);
      S.ry[r] = min(j - jlo, NR - 2);
#pragma unroll
      for (int k = 0; k < 4; ++k) S.wy[r][k] = w4[k];
    }
  }
  const int nx = fr.nx, ny = fr.ny;
  for (int e = threadIdx.x; e < 8 * NR * NC; e += NT) {
    const int t = e / (NR * NC), rc = e - t * (NR * NC);
    const int r = rc / NC, c = rc - r * NC;
    const int j = min(jlo + r, ny - 1), i = min(ilo + c, nx - 1);
    const double* tab = t < 4 ? wk.tb[t] : wk.tr[t - 4];
    S.node[t][r][c] = tab[fr.node0 + j * nx + i];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TH * NC; e += NT) {
    const int r = e / NC, c = e - (e / NC) * NC;
    const int j = S.ry[r];
    const int j1 = ny == 1 ? j : j + 1;
    const double a0 = S.wy[r][0], a1 = S.wy[r][1];
    const double a2 = S.wy[r][2], a3 = S.wy[r][3];
    auto comb = [&](int tv, int tm) {
      return ((a0 * S.node[tv][j][c] + a1 * S.node[tv][j1][c]) +
              a2 * S.node[tm][j][c]) + a3 * S.node[tm][j1][c];
    };
    S.gB[r][c] = comb(0, 2);        // f with fyy
    S.gBpp[r][c] = comb(1, 3);      // fxx with fxxyy
    S.gR[r][c] = comb(4, 6);
    S.gRpp[r][c] = comb(5, 7);
  }
  __syncthreads();
}

// The x part of a tile column's spline evaluation: its mesh interval and
// four weights, the same for every row.
struct SplineX {
  int k;
  double w0, w1, w2, w3;
};

template <int TH, int TW>
__device__ __forceinline__ SplineX spline_x(const SplineLds<TH, TW>& S,
                                            int c) {
  SplineX x;
  x.k = S.cx[c];
  x.w0 = S.wx[0][c];
  x.w1 = S.wx[1][c];
  x.w2 = S.wx[2][c];
  x.w3 = S.wx[3][c];
  return x;
}

// Background and rms (binary64) of tile pixel (r, c) after the prologue,
// from the column's x part.
template <int TH, int TW>
__device__ __forceinline__ void spline_at(const SplineLds<TH, TW>& S,
                                          const SplineX& x, int r, double* b,
                                          double* rr) {
  const int k = x.k;
  // fused multiply-adds: four FP64 operations per map
  *b = fma(x.w3, S.gBpp[r][k + 1],
           fma(x.w2, S.gBpp[r][k],
               fma(x.w1, S.gB[r][k + 1], x.w0 * S.gB[r][k])));
  *rr = fma(x.w3, S.gRpp[r][k + 1],
            fma(x.w2, S.gRpp[r][k],
                fma(x.w1, S.gR[r][k + 1], x.w0 * S.gR[r][k])));
}

template <int TH, int TW>
__device__ __forceinline__ void spline_pixel(const SplineLds<TH, TW>& S,
                                             int r, int c, double* b,
                                             double* rr) {
  spline_at<TH, TW>(S, spline_x<TH, TW>(S, c), r, b, rr);
}

}  // namespace ipp
