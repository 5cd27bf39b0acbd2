/*
 * ipp.h -- C ABI of the astronomical image pre-processing hot path on
 * AMD Instinct MI355X (gfx950).
 *
 * The calls follow the steps of the GPU pre-processing framework of
 * arXiv 2502.10783 (Cao, Jia et al., "Image Pre-Processing Framework for
 * Time-Domain Astronomy in the Artificial Intelligence Era"):
 *
 *   ipp_background   Sec. 2.2.2 -- mesh of sigma-clipped region statistics
 *                    (Eq. 1-4), median filter, spline interpolation.
 *   ipp_detect       Sec. 2.2.5 -- background removal, threshold detection,
 *                    connection of pixels into candidates, pre-analysis
 *                    (peak value, total flux, barycentre).
 *   ipp_photometry   Sec. 2.2.5 -- per-object circular aperture photometry.
 *   ipp_process_batch Sec. 2.1 pipeline mode -- all of the above for a batch
 *                    of frames with one fixed parameter set.
 *   ipp_photometry_backward, ipp_asinh, ipp_asinh_backward -- gradients of the
 *                    photometry and a gray-scale stretch (Sec. 2.2.6) so the
 *                    pre-processing can sit inside a training graph.
 *
 * Conventions (all calls):
 *  - Image, map, mesh and table arrays are DEVICE pointers owned by the
 *    caller.  Descriptor arrays (ipp_frame[], ipp_maps[], ipp_mesh[]) and
 *    ipp_params are HOST memory read during the call only.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t passed as
 *    void*, NULL = the null stream).  Results are valid once the stream has
 *    reached the point of the call.  Calls on one context must not overlap
 *    (one stream per context): they share the context's workspace.
 *  - Every argument is validated on the host before anything is enqueued.
 *    A failed check returns IPP_E_INVALID_ARG (or IPP_E_UNSUPPORTED /
 *    IPP_E_WORKSPACE) and enqueues nothing; ipp_last_error() describes it.
 *    No call aborts the process or lets an exception cross the ABI.
 *  - Pixel (x, y) is column x, row y of a row-major frame; its centre is at
 *    (x, y) and it covers [x-1/2, x+1/2] x [y-1/2, y+1/2].
 *  - Problems in the data (NaN pixels, no valid mesh node, apertures off the
 *    frame) do not fail a call; they set flags (IPP_FRAME_*, IPP_SRC_*).
 */
#ifndef IPP_H
#define IPP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IPP_API_VERSION 1

typedef enum ipp_status {
  IPP_OK = 0,
  IPP_E_INVALID_ARG = -1,   /* bad pointer, size or parameter            */
  IPP_E_UNSUPPORTED = -2,   /* valid but not implemented (e.g. mesh < 16) */
  IPP_E_CAPACITY = -3,      /* a caller-sized output is too small         */
  IPP_E_DEVICE = -4,        /* a HIP runtime call failed                  */
  IPP_E_WORKSPACE = -5      /* context workspace too small: reserve more  */
} ipp_status;

/* Background estimators, Sec. 2.2.2 Eq. 1-4. */
enum {
  IPP_EST_SEXTRACTOR = 0,   /* Eq. 3: 2.5*median - 1.5*mean (default)     */
  IPP_EST_MEDIAN = 1,       /* Eq. 1                                      */
  IPP_EST_MEAN = 2,         /* Eq. 2                                      */
  IPP_EST_MODE = 3          /* Eq. 4, read as median_factor*median
                               - mean_factor*mean                          */
};

/* ipp_params.flags */
#define IPP_F_WRITE_RMS 1u  /* ipp_process_batch also writes the rms maps  */
#define IPP_F_NO_GRAPH 2u   /* ipp_process_batch and ipp_refine_centroids
                               launch their kernels one by one instead of
                               capturing and replaying a HIP graph         */
#define IPP_F_NO_PHOTOMETRY 4u      /* ipp_process_batch stops after the
                                       source table: the photometry columns
                                       are left to ipp_photometry or to
                                       ipp_refine_centroids with the next
                                       flag                                */
#define IPP_F_REFINE_PHOTOMETRY 8u  /* ipp_refine_centroids also writes the
                                       photometry of ipp_photometry at the
                                       starting centres (flux_ap, sky,
                                       area_ap, area_ann; flags or'ed in),
                                       taken in its first evaluation       */

/* Per-frame flags (uint32 per frame). */
#define IPP_FRAME_NO_VALID_MESH 1u  /* no node had min_valid pixels: every
                                       node with >= 1 pixel was used        */
#define IPP_FRAME_EMPTY_MESH 2u     /* no node had any usable pixel: the
                                       background and rms are 0             */

/* Per-source flags (uint32 per table row). */
#define IPP_SRC_APERTURE_OFF_EDGE 1u  /* an aperture pixel is off the frame
                                         or not finite                      */
#define IPP_SRC_ANNULUS_OFF_EDGE 2u   /* same for the sky annulus           */
#define IPP_SRC_NO_SKY 4u             /* no annulus pixel: sky taken as 0   */
#define IPP_SRC_INEXACT_SUM_RANGE 8u  /* a pixel of the candidate lies
                                         outside the exact-sum range        */
#define IPP_SRC_NONPOSITIVE_FLUX 16u  /* isophotal flux <= 0: unweighted
                                         centroid                           */
#define IPP_SRC_BLENDED 32u           /* an object of a candidate that
                                         deblending split                   */

/*
 * Method parameters.  Defaults (ipp_params_default) are the settings of
 * Sec. 2.2.2 and 2.2.5: 64x64 regions, 3x3 median filter, 3 clip passes at
 * 3 sigma, at least 100 pixels per valid region, 1.5 sigma detection,
 * minimum area 5, 8-connectivity, aperture radius 5 px, annulus 8-12 px.
 */
typedef struct ipp_params {
  int32_t mesh_h, mesh_w;        /* region size in pixels, 16..128         */
  int32_t filter_h, filter_w;    /* median filter size in nodes (odd)      */
  int32_t clip_iters;            /* max rejection passes (0..16)           */
  int32_t estimator;             /* IPP_EST_*                              */
  double clip_sigma;             /* k of the k-sigma bounds (> 0)          */
  double median_factor;          /* Eq. 4 weights                          */
  double mean_factor;
  int32_t min_valid;             /* pixels for a valid region (>= 1)       */
  int32_t min_area;              /* pixels for a kept candidate (>= 1)     */
  double det_nsigma;             /* detection threshold in rms units       */
  int32_t connectivity;          /* 8 or 4                                 */
  int32_t sky_clip_iters;        /* annulus clip passes (0..16)            */
  double sky_clip_sigma;         /* annulus clip k (> 0)                   */
  double r_ap, r_in, r_out;      /* aperture and annulus radii in px,
                                    0 < r_ap <= 16, 0 <= r_in < r_out <= 16 */
  int32_t tile_h, tile_w;        /* detection tile shape; 0 = default.
                                    Supported: 64x64, 32x128, 128x32       */
  uint32_t flags;                /* IPP_F_*                                */
  int32_t reserved;
} ipp_params;

/* One input frame: h rows of w float32 pixels, row stride `pitch`
 * elements (w <= pitch <= 2^24).  `mask` (nullable) is h x w bytes with the
 * same pitch; a nonzero byte excludes the pixel from the background
 * statistics.  Frames up to 32767 x 32767 pixels. */
typedef struct ipp_frame {
  const float* pix;
  const uint8_t* mask;
  int64_t pitch;
  int32_t h, w;
} ipp_frame;

/* Full-resolution maps of one frame, dense h x w (row stride w). */
typedef struct ipp_maps {
  float* bkg;        /* background B32                                     */
  float* rms;        /* background rms R32                                 */
  int32_t* labels;   /* candidate labels: 0 = none, 1..K in raster order of
                        each candidate's first pixel                       */
} ipp_maps;

/* Mesh of one frame, ny x nx row-major with ny = ceil(h/mesh_h),
 * nx = ceil(w/mesh_w).  Every member is nullable. */
typedef struct ipp_mesh {
  double* bkg_raw;   /* estimator of each region's clipped pixels          */
  double* rms_raw;   /* population sigma of the clipped pixels             */
  int32_t* n_used;   /* surviving pixel count                              */
  double* bkg;       /* after invalid-node fill and median filter          */
  double* rms;
} ipp_mesh;

/* Source table: struct of arrays with `capacity` rows, DEVICE memory.
 * Rows are ordered by frame, then by label; frame f owns rows
 * [frame_offsets[f], frame_offsets[f+1]).  In ipp_photometry the columns
 * frame, x, y and the device scalar n_total (nullable: then `capacity`
 * rows) are inputs. */
typedef struct ipp_sources {
  int64_t capacity;
  int64_t* n_total;          /* device scalar: rows found (may exceed
                                capacity: then rows >= capacity are lost)  */
  int64_t* frame_offsets;    /* device [n_frames + 1]                      */
  int32_t* frame;
  int32_t* label;
  int32_t* npix;
  int32_t *xmin, *xmax, *ymin, *ymax;
  int32_t *peak_x, *peak_y;
  double* peak;              /* max of I - B32 over the candidate          */
  double* flux_iso;          /* sum of I - B32 over the candidate          */
  double *x, *y;             /* flux-weighted barycentre                   */
  double* flux_ap;           /* aperture flux minus sky * aperture area    */
  double* sky;               /* local sky per pixel                        */
  double* area_ap;           /* sum of aperture weights                    */
  double* area_ann;          /* sum of weights of the surviving annulus px */
  uint32_t* flags;           /* IPP_SRC_*                                  */
} ipp_sources;

/* Library version (IPP_API_VERSION). */
int32_t ipp_version(void);
/* Static text for a status code. */
const char* ipp_status_string(int32_t status);

/* Fill *p with the defaults listed above. */
void ipp_params_default(ipp_params* p);
/* Host-only check of a parameter set; no device is touched. */
ipp_status ipp_params_validate(const ipp_params* p);

/* Context: owns a device workspace and the last error message.
 * ipp_ctx_create makes `device` current and allocates nothing;
 * ipp_ctx_reserve (re)allocates the workspace to at least `bytes` (call it
 * before any ipp_* call that needs more; never during stream capture). */
ipp_status ipp_ctx_create(void** ctx, int32_t device);
ipp_status ipp_ctx_destroy(void* ctx);
ipp_status ipp_ctx_reserve(void* ctx, size_t bytes);
/* Message of the last failed call on ctx ("" if none); owned by ctx. */
const char* ipp_last_error(void* ctx);

/* Kernel timing: with `on` != 0 every kernel a call enqueues is bracketed
 * by a pair of HIP events recorded on the call's stream (this also clears
 * the totals); 0 stops recording.  ipp_ctx_profile_read waits for the
 * recorded events and returns the number of distinct kernels; for the
 * first `max` of them it writes the name (32 bytes each, NUL-terminated,
 * into names[32*max]), the summed milliseconds and the launch count.
 * All three output arrays are host memory and nullable.  Returns -1 for a
 * NULL ctx. */
ipp_status ipp_ctx_profile(void* ctx, int32_t on);
int32_t ipp_ctx_profile_read(void* ctx, int32_t max, char* names,
                             double* total_ms, int32_t* count);

/* Workspace bytes the calls below need for this batch, with room for
 * `record_capacity` partial candidates (a candidate cut by detection-tile
 * borders counts once per tile piece; 0 = a default of one per 16 pixels).
 * Host-only: returns 0 for invalid arguments. */
size_t ipp_workspace_bytes(const ipp_frame* frames, int32_t n,
                           const ipp_params* p, int64_t record_capacity);

/*
 * Background estimation (Sec. 2.2.2) of n frames: writes maps[f].bkg and
 * maps[f].rms (both required), and the mesh arrays given in mesh[f]
 * (mesh may be NULL).  frame_flags: device uint32[n], nullable.
 */
ipp_status ipp_background(void* ctx, const ipp_frame* frames, int32_t n,
                          const ipp_params* p, const ipp_maps* maps,
                          const ipp_mesh* mesh, uint32_t* frame_flags,
                          void* stream);

/*
 * Detection and pre-analysis (Sec. 2.2.5) of n frames against the given
 * background maps[f].bkg and rms maps[f].rms (inputs); writes
 * maps[f].labels and the table columns frame, label, npix, bbox, peak,
 * peak_x, peak_y, flux_iso, x, y, flags plus n_total and frame_offsets.
 * diag: device int64[4], nullable: [0] partial candidates used,
 * [1] their capacity, [2] nonzero if it overflowed (labels then invalid).
 */
ipp_status ipp_detect(void* ctx, const ipp_frame* frames, int32_t n,
                      const ipp_params* p, const ipp_maps* maps,
                      ipp_sources* src, int64_t* diag, void* stream);

/*
 * Aperture photometry (Sec. 2.2.5) of the table rows against the frames
 * and their background maps[f].bkg: reads frame, x, y; writes flux_ap,
 * sky, area_ap, area_ann and ORs IPP_SRC_* edge/sky bits into flags.
 * sky_lohi: device double[2*capacity], nullable: the value range of the
 * surviving annulus pixels of each row, kept for ipp_photometry_backward.
 */
ipp_status ipp_photometry(void* ctx, const ipp_frame* frames, int32_t n,
                          const ipp_maps* maps, const ipp_params* p,
                          ipp_sources* src, double* sky_lohi, void* stream);

/*
 * Pipeline mode (Sec. 2.1): background, detection and photometry of a
 * batch of frames of any sizes, fused (the background is evaluated inside
 * the detection kernel) and replayed from a captured HIP graph when the
 * same batch is seen again.  Writes maps[f].bkg and maps[f].labels
 * (required) and maps[f].rms if IPP_F_WRITE_RMS is set.
 */
ipp_status ipp_process_batch(void* ctx, const ipp_frame* frames, int32_t n,
                             const ipp_params* p, const ipp_maps* maps,
                             ipp_sources* src, uint32_t* frame_flags,
                             int64_t* diag, void* stream);

/*
 * Backward of ipp_photometry (the annulus clip mask of the forward held
 * fixed).  Inputs as for ipp_photometry plus sky_lohi (device
 * double[2*rows], written by the forward) and dL_dflux (device
 * double[rows], upstream gradient of flux_ap).  dL_dpix: HOST array of n
 * device pointers (nullable, entries nullable), each a dense h x w float32
 * map to which dL/dI is ADDED with float atomics (summation order, hence
 * the last bits, may vary from run to run); dL/dB32 is its negative.
 * dL_dxy: device double[2*rows] (nullable), overwritten with
 * (dL/dx, dL/dy) per row.  Rows: min(capacity, *n_total).
 */
ipp_status ipp_photometry_backward(void* ctx, const ipp_frame* frames,
                                   int32_t n, const ipp_maps* maps,
                                   const ipp_params* p,
                                   const ipp_sources* src,
                                   const double* sky_lohi,
                                   const double* dL_dflux,
                                   float* const* dL_dpix, double* dL_dxy,
                                   void* stream);

/*
 * Gradient centroid refinement on the photometry of Sec. 2.2.5 and its
 * backward (this library's addition; the paper measures objects at their
 * detected positions).  Each row's centre c (columns frame, x, y of src;
 * rows min(capacity, *n_total), or capacity when n_total is NULL) climbs
 * J(c) = F_rc(c) / F_ap(c0): F_rc is the sky-subtracted flux of
 * ipp_photometry with the aperture radius r_c (annulus and clipping from
 * p), F_ap(c0) the flux with p's own aperture at the start.  `steps`
 * plain ascent steps c <- c + eta dJ/dc follow, the gradient taken by
 * ipp_photometry_backward with each step's annulus clip mask held fixed.
 * Rows with F_ap(c0) <= 0 (or not a number) stay where they are.
 * x_out, y_out: device double[capacity], the refined centres (they may be
 * src->x and src->y themselves); the table's other columns are untouched
 * unless IPP_F_REFINE_PHOTOMETRY is set (below).
 * r_c in (0, 16], eta finite, steps in [0, 1000].  One kernel launch: a
 * wavefront takes each row through the normaliser and every step (forward
 * and gradient from the same exact overlaps; the normaliser is the flux
 * of a second aperture in the first step's evaluation, over that step's
 * sky).  With IPP_F_REFINE_PHOTOMETRY in p->flags that evaluation's
 * photometry with p's aperture at the starting centre is also written to
 * the table's flux_ap, sky, area_ap, area_ann and flags (which must then
 * be given), equal to ipp_photometry's up to the order of binary64 sums,
 * also when steps is 0.  Needs
 * ipp_refine_workspace_bytes of workspace (the frame descriptors; rows is
 * checked, not counted).  The launch is replayed from a captured HIP graph
 * when called again with the same signature.
 */
size_t ipp_refine_workspace_bytes(const ipp_frame* frames, int32_t n,
                                  int64_t rows);
ipp_status ipp_refine_centroids(void* ctx, const ipp_frame* frames,
                                int32_t n, const ipp_maps* maps,
                                const ipp_params* p, const ipp_sources* src,
                                double r_c, double eta, int32_t steps,
                                double* x_out, double* y_out, void* stream);

/*
 * asinh gray-scale stretch (Sec. 2.2.6 gray-scale transformations):
 * y[i] = b * asinh(v[i] / a), float32 arrays of n elements (device),
 * a > 0 (softening), b (scale).
 */
ipp_status ipp_asinh(void* ctx, const float* v, float* y, int64_t n,
                     double a, double b, void* stream);
/* Backward: dv[i] = dy[i] * b / sqrt(a^2 + v[i]^2) (dv nullable; written,
 * not accumulated); dL_dab (device double[2], nullable) =
 * (sum dy * -b v / (a sqrt(a^2+v^2)), sum dy * asinh(v/a)), accumulated in
 * binary64 in a fixed order (deterministic).  Needs 32 KiB of workspace
 * when dL_dab is given. */
ipp_status ipp_asinh_backward(void* ctx, const float* v, const float* dy,
                              float* dv, double* dL_dab, int64_t n, double a,
                              double b, void* stream);

/*
 * ipp_asinh and ipp_asinh_backward with the parameters in device memory:
 * ab is a device double[2] = (a, b), read by the kernels, so a caller's
 * parameter tensors need no host round trip (and the calls can be captured
 * into a graph).  The host cannot check values it does not read: with
 * a <= 0, a or b not finite, every output (y, dv, dL_dab) is NaN.
 */
ipp_status ipp_asinh_dev(void* ctx, const float* v, float* y, int64_t n,
                         const double* ab, void* stream);
ipp_status ipp_asinh_backward_dev(void* ctx, const float* v, const float* dy,
                                  float* dv, double* dL_dab, int64_t n,
                                  const double* ab, void* stream);

/*
 * ipp_asinh_backward without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): same arguments, results and
 * error checks as ipp_asinh_backward, but the block partials of dL_dab live
 * in a static device array of the library (2 * 2048 doubles = 32 KiB per
 * GPU, held until the process ends) instead of the context workspace, so
 * no ipp_ctx_reserve is needed.  Any n is accepted: at most 2048
 * grid-stride workgroups write partials, each its own slot, before the
 * final reduction reads them (nothing must start at zero).  Calls that
 * overlap on one GPU share that array and race: serialise them (one
 * stream, or events between streams).  IPP_E_CAPACITY if the partials
 * would not fit the array.
 */
ipp_status ipp_asinh_backward_noalloc(void* ctx, const float* v,
                                      const float* dy, float* dv,
                                      double* dL_dab, int64_t n, double a,
                                      double b, void* stream);

/*
 * Deblending and cleaning (Sec. 2.2.5, the phases between detection and
 * photometry): every candidate of a detection (label map + table) is split
 * into objects by multi-threshold deblending, and objects that cleaning
 * finds to be light of a brighter neighbour are merged back.
 *
 *  - Levels: t0 = det_nsigma R32 at the candidate's peak pixel;
 *    q = (peak / t0)^(1/nthresh) by log2(nthresh) square roots;
 *    t_i = t_{i-1} q, i = 1 .. nthresh-1 (binary64).  Candidates of one
 *    pixel, or with t0 <= 0, stay whole.
 *  - Tree: at each level the candidate's pixels with v = I - B32 above it
 *    form components (p->connectivity), nested in the level below.
 *  - Contrast: a node is significant iff fl(S 2^-28) - n t_i (S the exact
 *    sum of the source table's weights D over its n pixels) exceeds
 *    mincont times the candidate's flux.
 *  - Pruning, bottom up: a leaf is one object; a node with two or more
 *    significant children stands for their objects, with one for that
 *    child's objects when it has two or more, else for itself.
 *  - The object nodes' pixels are seeds, numbered in raster order of their
 *    first pixels; every other pixel goes to the seed whose model
 *    F s2 / (s2 + d^2)^2 is largest (F, barycentre and s2 = x2 + y2 + 1/6
 *    from the seed's exact moments; ties to the lower index).
 *  - Cleaning (clean != 0): an object whose mean value minus
 *    clean_param F s2 / (pi (s2 + d^2)^2) summed over the brighter objects
 *    of its candidate (at its seed barycentre) falls below t0 joins the
 *    brightest contributor.
 *
 * Inputs: frames; maps[f].bkg, .rms and .labels (the detection's); cand,
 * the detection table (frame, label, npix, bounding box, peak, peak_x,
 * peak_y, frame_offsets; rows min(capacity, *n_total)); p (det_nsigma,
 * connectivity).  Outputs: objects[f], device int32 h x w per frame:
 * 0 outside the candidates, objects numbered 1..K per frame candidate by
 * candidate and within a candidate in seed order; obj, the object table:
 * frame, label (the object number), npix, bounding box, then the
 * pre-analysis of ipp_detect over the object map (peak, peak_x, peak_y,
 * flux_iso, x, y, flags, with IPP_SRC_BLENDED on objects of split
 * candidates), n_total, frame_offsets; parent, device int32[obj capacity]:
 * the candidate label of each object.  Rows beyond obj->capacity are not
 * written (n_total still counts them).  Scratch: the workspace beyond the
 * fixed part (ipp_deblend_workspace_bytes with scratch_bytes); a candidate
 * needs 48 B per bounding-box pixel plus 368 B per pixel.  diag
 * (device int64[4], nullable): [0] scratch bytes needed, [1] available,
 * [2] nonzero if candidates were left whole for lack of scratch, [3]
 * objects found.
 */
typedef struct ipp_deblend_params {
  int32_t nthresh;        /* levels: a power of two in [2, 64] (32)       */
  int32_t clean;          /* cleaning pass (1)                            */
  double mincont;         /* contrast fraction, >= 0 (0.005)              */
  double clean_param;     /* scale of the neighbours' light, >= 0 (1.0)   */
} ipp_deblend_params;

void ipp_deblend_params_default(ipp_deblend_params* d);
size_t ipp_deblend_workspace_bytes(const ipp_frame* frames, int32_t n,
                                   int64_t cand_capacity,
                                   int64_t scratch_bytes);
ipp_status ipp_deblend(void* ctx, const ipp_frame* frames, int32_t n,
                       const ipp_params* p, const ipp_deblend_params* dp,
                       const ipp_maps* maps, const ipp_sources* cand,
                       int32_t* const* objects, ipp_sources* obj,
                       int32_t* parent, int64_t* diag, void* stream);

/*
 * Second-order moments of each table row's footprint (the pre-analysis of
 * Sec. 2.2.5 carried to second order, as SExtractor's X2, Y2, XY and the
 * ellipse A, B, THETA): over the bounding-box pixels whose label is the
 * row's, with the integer weights D = (I - B32) 2^28 of the source table,
 * exact sums of D, D dx, D dy, D dx^2, D dy^2, D dx dy (dx, dy from the
 * bounding-box corner), each rounded once to binary64; then
 * mx = Sx/S, my = Sy/S, x2 = Sxx/S - mx^2, y2 = Syy/S - my^2,
 * xy = Sxy/S - mx my, t = (x2 + y2)/2, r = sqrt(((x2 - y2)/2)^2 + xy^2),
 * a = sqrt(t + r), b = sqrt(max(t - r, 0)), theta = atan2(2 xy, x2 - y2)/2.
 * Reads the table's frame, label and bounding box (rows: min(capacity,
 * *n_total)) and maps[f].bkg and maps[f].labels; writes mom, device
 * double[6 * capacity]: (x2, y2, xy, a, b, theta) per row, NaN where the
 * weights do not sum to a positive value.
 */
ipp_status ipp_source_moments(void* ctx, const ipp_frame* frames, int32_t n,
                              const ipp_maps* maps, const ipp_sources* src,
                              double* mom, void* stream);

/*
 * AUTO (Kron) photometry (Sec. 2.2.5 lists auto photometry among the
 * per-object measurements; Sec. 3.3 compares auto magnitudes): for each
 * table row (frame, x, y; rows min(capacity, *n_total)) with the second
 * moments mom[6 row + 0..2] = (x2, y2, xy) of ipp_source_moments:
 *  - X = x2 + 1/12, Y = y2 + 1/12, det = X Y - xy^2 (the moments
 *    regularised by a uniform unit pixel); q(dx, dy) = (Y dx^2 + X dy^2
 *    - 2 xy dx dy) / det is 1 on the one-sigma ellipse;
 *  - Kron radius: r1 = sum sqrt(q) v / sum v over the in-frame pixel
 *    centres with q <= search^2 (v = I - B32), R = max(kron_factor r1,
 *    kron_min), or kron_min when sum v <= 0 (flag 2);
 *  - AUTO flux = sum of v times the exact area of each pixel inside the
 *    ellipse q <= R^2 around (x, y), area = the sum of those areas; a
 *    pixel belongs to the ellipse iff the smallest q over its square is
 *    below R^2; ellipse pixels off the frame or not finite are skipped
 *    (flag 4; the frame's one-pixel surround is examined, and an ellipse
 *    centred off the frame is flagged);
 *  - rows with unusable moments (det <= 0 or not finite) get NaN (flag 1).
 * Outputs (device, per row): kron (R), flux, area, flags.  ap nullable:
 * defaults kron_factor 2.5, kron_min 3.5, search 6.
 */
typedef struct ipp_auto_params {
  double kron_factor;     /* k in R = k r1 (2.5)                          */
  double kron_min;        /* smallest R (3.5)                             */
  double search;          /* search ellipse for r1, in sigmas (6)         */
} ipp_auto_params;

void ipp_auto_params_default(ipp_auto_params* a);
ipp_status ipp_photometry_auto(void* ctx, const ipp_frame* frames, int32_t n,
                               const ipp_maps* maps, const ipp_sources* src,
                               const double* mom, const ipp_auto_params* ap,
                               double* kron, double* flux, double* area,
                               uint32_t* flags, void* stream);

/*
 * Stamp convolution and image subtraction (Sec. 2.2.4, Eq. 8-10).  The
 * template frames R (aligned with the science frames I, same shapes) are
 * convolved with the kernel
 *   K(u, v) = sum_n a_n(x, y) exp(-(u^2 + v^2) / (2 sigma_k^2)) u^i v^j,
 * the basis ordered by Gaussian (as given), then i = 0..order_k, then
 * j = 0..order_k - i, u (columns) and v (rows) in [-hw, hw]; and
 * D = (I + B) - R (x) K is written (zero where Eq. 10 holds).  a_n and the
 * background difference B are polynomials in xn = (2x - (W-1)) / (W-1),
 * yn likewise (0 on a one-pixel axis): sum over p = 0..d, q = 0..d-p of
 * c_pq xn^p yn^q, coefficients in that order; each stamp (stamp x stamp
 * pixels, partial at the right and bottom edges) uses them at its centre
 * (the centre of its actual extent).  R is zero outside the frame.  coef:
 * device double array, per frame nbasis * P(spatial_order) coefficients
 * (basis by basis) then P(bkg_order), P(d) = (d+1)(d+2)/2, frames one
 * after another.  diff[f]: device float32 h x w.  The kernel fit itself
 * is not part of this call.  Products are summed in binary32 per kernel
 * row and the rows in binary64.
 */
#define IPP_SUB_MAX_GAUSS 4
typedef struct ipp_subtract_params {
  int32_t half_width;         /* hw, 1..15 (10: 21 x 21 kernels)          */
  int32_t stamp;              /* stamp size, 1..32 (21)                    */
  int32_t n_gauss;            /* 1..4 (3)                                  */
  int32_t spatial_order;      /* degree of a_n(x, y), 0..4 (2)             */
  int32_t bkg_order;          /* degree of B(x, y), 0..4 (1)               */
  int32_t order[IPP_SUB_MAX_GAUSS];  /* max i + j per Gaussian, 0..7
                                        (6, 4, 2)                          */
  double sigma[IPP_SUB_MAX_GAUSS];   /* widths > 0 (0.7, 1.5, 3.0)         */
} ipp_subtract_params;

void ipp_subtract_params_default(ipp_subtract_params* sp);
/* Coefficients per frame (nbasis * P(spatial) + P(bkg)); 0 if invalid. */
int64_t ipp_subtract_coef_count(const ipp_subtract_params* sp);
ipp_status ipp_subtract(void* ctx, const ipp_frame* sci,
                        const ipp_frame* tmpl, int32_t n,
                        const ipp_subtract_params* sp, const double* coef,
                        float* const* diff, void* stream);

/*
 * Gray-scale transformations (Sec. 2.2.6): the zscale display range, point
 * maps and histogram equalization.  Frames as elsewhere (mask ignored);
 * outputs out[f] are device float32 h x w arrays with row pitch w.
 */
#define IPP_MAP_LINEAR 0  /* y = x                                         */
#define IPP_MAP_LOG 1     /* y = ln(1 + a x) / ln(1 + a), a > 0            */
#define IPP_MAP_EXP 2     /* y = (a^x - 1) / (a - 1), a > 0, a != 1        */
#define IPP_MAP_POWER 3   /* y = x^a, a > 0                                */
#define IPP_ZSCALE_MAX_SAMPLES 1000
#define IPP_EQ_MAX_BINS 4096

/* Workspace bytes the gray-scale calls need for n frames and nbins
 * histogram bins (ipp_zscale and ipp_gray_map: nbins 0).  Host-only;
 * 0 for invalid arguments. */
size_t ipp_gray_workspace_bytes(int32_t n, int32_t nbins);

/*
 * zscale display range of each frame (the SAOimage DS9 / IRAF estimate):
 * the finite pixels on the grid of rows and columns 0, s, 2s, ... (s the
 * smallest step giving at most nsamples points, nsamples in
 * [1, IPP_ZSCALE_MAX_SAMPLES]) are sorted; a straight line is fitted to
 * them against their index with up to 5 fits, rejecting samples beyond
 * 2.5 standard deviations of the residuals and widening each rejection by
 * floor(n/100)/2 samples on either side; while at least half the samples
 * (and 5) remain, the line through the median with its slope divided by
 * contrast (> 0; 0 keeps the slope) gives the range, clamped to the
 * sample's extremes, else the extremes are the range.  z1z2: device
 * double[2n] (z1, z2 per frame; (0, 0) without finite samples).  info:
 * device double[4n], nullable: samples, samples kept, fits, fitted slope.
 */
ipp_status ipp_zscale(void* ctx, const ipp_frame* frames, int32_t n,
                      int32_t nsamples, double contrast, double* z1z2,
                      double* info, void* stream);

/*
 * Point map of every frame: x = (v - lo) / (hi - lo) clipped to [0, 1]
 * (for hi <= lo, 0 where v <= lo and 1 elsewhere), then the IPP_MAP_*
 * function of x with parameter a; non-finite v gives NaN.  lohi: device
 * double[2n] (lo, hi per frame, e.g. the output of ipp_zscale).
 */
ipp_status ipp_gray_map(void* ctx, const ipp_frame* frames, int32_t n,
                        int32_t kind, double a, const double* lohi,
                        float* const* out, void* stream);

/*
 * Histogram equalization of every frame over nbins (2..IPP_EQ_MAX_BINS)
 * equal bins spanning its finite values [lo, hi]: a value's bin is
 * floor(((v - lo) / (hi - lo)) nbins) (binary64; the top value in the last
 * bin), cdf_k = pixels in bins 0..k over the finite pixels, and y is the
 * linear interpolation of (lo + (k + 1/2)(hi - lo)/nbins, cdf_k) at v, held
 * at the end values outside the first and last centre.  A constant frame
 * maps to 1, non-finite pixels to NaN.  counts: device uint32[n * nbins],
 * nullable: the histograms (cleared and written by the call).
 */
ipp_status ipp_equalize(void* ctx, const ipp_frame* frames, int32_t n,
                        int32_t nbins, float* const* out, uint32_t* counts,
                        void* stream);

/* ipp_autotune: what to tune */
#define IPP_TUNE_MESH 1u   /* mesh size from {32, 64, 128} (changes results) */
#define IPP_TUNE_TILE 2u   /* detection tile shape 64x64, 32x128, 128x32
                              (results unchanged)                         */

/*
 * Autotuner of the pipeline mode (Sec. 2.1 runs fixed parameter sets from a
 * configuration file): times ipp_process_batch on the given frames for
 * every candidate mesh size and/or tile shape selected by `what`, keeps
 * the fastest in *p (the other fields are untouched) and its time in
 * *best_ms (nullable).  With cache_path (nullable) the choice is looked up
 * first and stored afterwards in that JSON file, keyed by the device
 * architecture, the multiset of frame shapes and a hash of the remaining
 * parameters.  Allocates its trial outputs with hipMalloc, may grow the
 * context workspace, synchronizes `stream`.  Not for use under capture.
 */
ipp_status ipp_autotune(void* ctx, const ipp_frame* frames, int32_t n,
                        ipp_params* p, uint32_t what, const char* cache_path,
                        double* best_ms, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* IPP_H */
