// Evaluation of the tensor-product natural cubic spline background and rms
// (Sec. 2.2.2: spline interpolation of the filtered mesh back to the full
// resolution) over one detection tile.
//
// With per-node tables f, fxx (second derivative along x), fyy and fxxyy,
// the spline restricted to an image row y is a 1-D natural spline in x
// through the values g_i(y) with second derivatives g''_i(y), where g_i and
// g''_i are 1-D splines in y of the node columns of (f, fyy) and
// (fxx, fxxyy).  The tile prologue evaluates those per row for the few
// mesh columns the tile spans, and the per-column x weights; each pixel is
// then four multiply-adds per map.
#pragma once

#include "ipp_internal.h"

namespace ipp {

template <int TH, int TW>
struct SplineLds {
  // mesh columns a tile can span (mesh >= 16), with one of slack
  static constexpr int NC = TW / 16 + 4;
  double gB[TH][NC];
  double gBpp[TH][NC];
  double gR[TH][NC];
  double gRpp[TH][NC];
  double wx[TW][4];
  int cx[TW];
};

template <int TH, int TW>
__device__ __forceinline__ void spline_prologue(const Work& wk,
                                                const FrameDev& fr,
                                                const ipp_params& p, int y0,
                                                int x0,
                                                SplineLds<TH, TW>& S) {
  constexpr int NC = SplineLds<TH, TW>::NC;
  int ilo;
  {
    double w4[4];
    spline_weights((double)x0, p.mesh_w, fr.w, fr.nx, &ilo, w4);
  }
  for (int c = threadIdx.x; c < TW; c += kBlock) {
    double w4[4];
    int j;
    spline_weights((double)(x0 + c), p.mesh_w, fr.w, fr.nx, &j, w4);
    S.cx[c] = j - ilo;
#pragma unroll
    for (int k = 0; k < 4; ++k) S.wx[c][k] = w4[k];
  }
  const int nx = fr.nx;
  for (int e = threadIdx.x; e < TH * NC; e += kBlock) {
    const int r = e / NC, c = e - (e / NC) * NC;
    const int i = min(ilo + c, nx - 1);
    const int y = min(y0 + r, fr.h - 1);
    double w4[4];
    int j;
    spline_weights((double)y, p.mesh_h, fr.h, fr.ny, &j, w4);
    const int j1 = (fr.ny == 1) ? j : j + 1;
    const int n0 = fr.node0 + j * nx + i, n1 = fr.node0 + j1 * nx + i;
    S.gB[r][c] = ((w4[0] * wk.tb[0][n0] + w4[1] * wk.tb[0][n1])
                  + w4[2] * wk.tb[2][n0]) + w4[3] * wk.tb[2][n1];
    S.gBpp[r][c] = ((w4[0] * wk.tb[1][n0] + w4[1] * wk.tb[1][n1])
                    + w4[2] * wk.tb[3][n0]) + w4[3] * wk.tb[3][n1];
    S.gR[r][c] = ((w4[0] * wk.tr[0][n0] + w4[1] * wk.tr[0][n1])
                  + w4[2] * wk.tr[2][n0]) + w4[3] * wk.tr[2][n1];
    S.gRpp[r][c] = ((w4[0] * wk.tr[1][n0] + w4[1] * wk.tr[1][n1])
                    + w4[2] * wk.tr[3][n0]) + w4[3] * wk.tr[3][n1];
  }
  __syncthreads();
}

// Background and rms (binary64) of tile pixel (r, c) after the prologue.
template <int TH, int TW>
__device__ __forceinline__ void spline_pixel(const SplineLds<TH, TW>& S,
                                             int r, int c, double* b,
                                             double* rr) {
  const int k = S.cx[c];
  const double w0 = S.wx[c][0], w1 = S.wx[c][1];
  const double w2 = S.wx[c][2], w3 = S.wx[c][3];
  *b = ((w0 * S.gB[r][k] + w1 * S.gB[r][k + 1]) + w2 * S.gBpp[r][k])
       + w3 * S.gBpp[r][k + 1];
  *rr = ((w0 * S.gR[r][k] + w1 * S.gR[r][k + 1]) + w2 * S.gRpp[r][k])
        + w3 * S.gRpp[r][k + 1];
}

}  // namespace ipp
