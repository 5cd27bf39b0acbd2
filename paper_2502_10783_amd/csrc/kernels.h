// Kernel declarations of libipp (definitions in k_*.hip).
#pragma once

#include "ipp_internal.h"

namespace ipp {

template <int PPT>
__global__ void k_mesh_stats(Work wk, ipp_params p);
template <int PPL>
__global__ void k_mesh_stats_w(Work wk, ipp_params p);
__global__ void k_mesh_fill(Work wk, ipp_params p);
template <int F>
__global__ void k_mesh_filter(Work wk, ipp_params p);
template <int PASS>
__global__ void k_mesh_spline(Work wk, ipp_params p);

template <int TH, int TW>
__global__ void k_bkg_maps(Work wk, ipp_params p);
// threads per detection tile (4096 pixels: 8 per thread)
constexpr int kTileThreads = 512;
template <int TH, int TW, bool FUSED, bool CONN8, int NT>
__global__ void k_tile_ccl(Work wk, ipp_params p, int write_rms);
// threads of k_border: one per right-border and bottom-border pixel of a
// tile, in whole waves
template <int TH, int TW>
constexpr int border_threads() { return (TH + TW + 63) / 64 * 64; }
template <int TH, int TW>
__global__ void k_border(Work wk, ipp_params p);
template <int TH, int TW>
__global__ void k_relabel(Work wk, ipp_params p);

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v);
__global__ void k_fill_i64(int64_t* a, int64_t n, int64_t v);
__global__ void k_resolve(Work wk, ipp_params p);
__global__ void k_heads(Work wk, ipp_params p);
__global__ void k_scan_blocks(const int32_t* in, int32_t* blocks, int n);
__global__ void k_scan_top(int32_t* blocks, int nblocks, int64_t* total);
__global__ void k_scan_apply(const int32_t* in, const int32_t* blocks,
                             int32_t* out, int n);
__global__ void k_frame_offsets(Work wk, ipp_sources src);
__global__ void k_scatter(Work wk, ipp_params p);
__global__ void k_rank(Work wk, ipp_params p, ipp_sources src);
__global__ void k_reclabel(Work wk);
__global__ void k_source_stats(Work wk, ipp_sources src);
__global__ void k_source_moments(Work wk, ipp_sources src, double* mom);

template <int NS>
__global__ void k_aperture_t(Work wk, ipp_params p, ipp_sources src,
                             double* sky_lohi);

template <int NS>
__global__ void k_aperture_bwd_t(Work wk, ipp_params p, ipp_sources src,
                                 const double* sky_lohi, const double* gF,
                                 double* dxy);

// Centroid refinement, every step of a row in one wavefront: xo, yo get
// the refined centres; PHOT: the photometry columns of the first
// evaluation as well.  Rows: min(capacity, *n_total).
template <int NS, bool PHOT>
__global__ void k_refine_t(Work wk, ipp_params p, double r_c, double eta,
                           int steps, ipp_sources src, double* xo,
                           double* yo);

// ab (nullable): device (a, b) used in place of the value arguments
__global__ void k_asinh_fwd(const float* v, float* y, int64_t n, float inv_a,
                            float b, const double* ab);
__global__ void k_asinh_bwd(const float* v, const float* dy, float* dv,
                            int64_t n, double a, double b, const double* ab,
                            double* partial);
__global__ void k_asinh_bwd_final(const double* partial, int nb,
                                  double* out);
// Device address of the file-scope scratch of the asinh backward on
// `device` (2 * kAsinhMaxBlocks doubles), looked up on first use with that
// device current and kept per device.  hipSuccess or the lookup's error.
hipError_t asinh_scratch(int device, double** ptr);

// Deblending (k_deblend.hip): see that file for the sequence.
// need: scratch units per row; big / nbig: the rows of boxes over
// kDbSmallBox pixels, those over kDbBigBox from the front (nbig[0]), the
// others from the back (nbig[1]); nbig zeroed by the caller.
__global__ void k_db_need(ipp_sources cand, int64_t* need, int32_t* big,
                          int64_t* nbig);
__global__ void k_scan64_blocks(const int64_t* in, int64_t* blocks,
                                int64_t n);
__global__ void k_scan64_top(int64_t* blocks, int64_t nblocks,
                             int64_t* total);
__global__ void k_scan64_apply(const int64_t* in, const int64_t* blocks,
                               int64_t* out, int64_t n);
// Bounding boxes up to this many pixels take a wavefront, larger ones a
// workgroup.
constexpr int kDbSmallBox = 512;
// Resident workgroups per compute unit of the two kernels (LDS and
// register limits); queue: a zeroed counter of taken rows.
constexpr int kDbSmallPerCu = 3, kDbLargePerCu = 2;
// Boxes over this many pixels are taken first by the workgroup kernel.
constexpr int kDbBigBox = 2048;
__global__ void k_db_small(Work wk, ipp_sources cand, const int64_t* off,
                           const int64_t* tot, char* pool,
                           int64_t pool_units, double nsigma, int conn,
                           int nthresh, int clean, double mincont, double kc,
                           int64_t* cnt, int64_t* queue);
__global__ void k_db_large(Work wk, ipp_sources cand, const int64_t* off,
                           const int64_t* tot, char* pool,
                           int64_t pool_units, double nsigma, int conn,
                           int nthresh, int clean, double mincont, double kc,
                           int64_t* cnt, int64_t* queue, const int32_t* big,
                           const int64_t* nbig);
__global__ void k_db_zero(Work wk);
__global__ void k_db_write(Work wk, ipp_sources cand, const int64_t* off,
                           const int64_t* tot, const char* pool,
                           int64_t pool_units, const int64_t* cnt,
                           const int64_t* ooff, ipp_sources obj,
                           int32_t* parent);
__global__ void k_db_offsets(Work wk, ipp_sources cand, const int64_t* ooff,
                             const int64_t* total, ipp_sources obj);
__global__ void k_db_flags(ipp_sources cand, const int64_t* cnt,
                           const int64_t* total, ipp_sources obj,
                           const int32_t* parent);
__global__ void k_db_diag(const int64_t* tot, int64_t pool_units,
                          const int64_t* counters, int64_t* diag);

// AUTO (Kron) photometry: one wavefront per row (k_kron.hip); rows whose
// search or ellipse window holds more than kKronBigPx pixels are finished
// by k_kron_big, kBigThreads threads per workgroup, launched after k_kron.
constexpr int kKronBigPx = 16384;
constexpr int kBigThreads = 512;
__global__ void k_kron(Work wk, ipp_sources src, const double* mom,
                       double kfac, double rmin, double search, double* kron,
                       double* flux, double* area, uint32_t* flags);
__global__ void k_kron_big(Work wk, ipp_sources src, const double* mom,
                           double kfac, double rmin, double search,
                           double* kron, double* flux, double* area,
                           uint32_t* flags);

// Stamp convolution and subtraction: one workgroup per stamp, HW = the
// kernel half-width; launched with sub_threads(stamp) threads and
// sub_lds_bytes(stamp, HW) bytes of dynamic LDS.
template <int HW>
__global__ void k_subtract_t(const SubFrame* frames, int nframes,
                             SubBasis bs, int64_t total_stamps);
size_t sub_lds_bytes(int stamp, int hw);
int sub_threads(int stamp);

__global__ void k_zscale(const GrayFrame* frames, double contrast,
                         double krej, int max_iter, double* z1z2,
                         double* info);
__global__ void k_gray_map(const GrayFrame* frames, int nframes,
                           int total_rows, int kind, float a, float c,
                           float lna, const double* lohi);
__global__ void k_eq_minmax(const GrayFrame* frames, int nframes,
                            int total_rows, uint32_t* mm);
__global__ void k_eq_hist(const GrayFrame* frames, int nframes,
                          int total_rows, int nbins, const uint32_t* mm,
                          uint32_t* counts);
__global__ void k_eq_cdf(const uint32_t* counts, int nbins, double* cdf);
__global__ void k_eq_map(const GrayFrame* frames, int nframes, int total_rows,
                         int nbins, const uint32_t* mm, const double* cdf);

}  // namespace ipp
