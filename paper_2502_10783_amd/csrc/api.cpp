// Host side of libipp: argument validation, workspace planning, kernel
// sequencing and the HIP-graph cache of the batched pipeline call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ipp_internal.h"
#include "deblend_core.h"
#include "kernels.h"

using namespace ipp;

// A captured batch pipeline.  The graph bakes in the workspace layout, the
// parameters and the table; the frame descriptors (pixel and map pointers)
// live in the workspace and are uploaded before each launch unless the
// workspace was not touched since the same descriptors were uploaded.
struct IppGraph {
  std::vector<uint8_t> key;       // batch signature
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t ws_gen = 0;            // workspace generation of the last upload
  std::vector<uint8_t> fd;        // descriptors of the last upload
  uint64_t last_use = 0;
};

struct ProfSlot {
  const char* name;
  hipEvent_t a = nullptr, b = nullptr;
};

struct IppCtx {
  bool prof = false;
  std::vector<ProfSlot> pool;     // event pairs (reused)
  size_t used = 0;                // pairs recorded since the last read
  std::vector<std::pair<std::string, std::pair<double, int>>> totals;
  int device = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  uint64_t ws_gen = 1;            // bumped when the workspace is reused
  std::string err;
  std::vector<IppGraph> graphs;   // small LRU cache of captured batches
  uint64_t tick = 0;
  hipStream_t cap = nullptr;      // private stream used only for capture
  bool use_graphs = true;
  int n_cu = 256;                 // compute units of the device
};

namespace {

ProfSlot* prof_begin(IppCtx* c, hipStream_t s, const char* name) {
  if (!c || !c->prof) return nullptr;
  if (c->used == c->pool.size()) {
    ProfSlot ps;
    if (hipEventCreate(&ps.a) != hipSuccess ||
        hipEventCreate(&ps.b) != hipSuccess)
      return nullptr;
    c->pool.push_back(ps);
  }
  ProfSlot* ps = &c->pool[c->used++];
  ps->name = name;
  hipEventRecord(ps->a, s);
  return ps;
}

void prof_end(ProfSlot* ps, hipStream_t s) {
  if (ps) hipEventRecord(ps->b, s);
}

// Fold the recorded event pairs into per-kernel totals (waits for them).
void prof_collect(IppCtx* c) {
  for (size_t i = 0; i < c->used; ++i) {
    ProfSlot& ps = c->pool[i];
    float ms = 0.f;
    hipEventSynchronize(ps.b);
    if (hipEventElapsedTime(&ms, ps.a, ps.b) != hipSuccess) ms = 0.f;
    bool found = false;
    for (auto& t : c->totals)
      if (t.first == ps.name) {
        t.second.first += ms;
        t.second.second += 1;
        found = true;
        break;
      }
    if (!found) c->totals.push_back({ps.name, {(double)ms, 1}});
  }
  c->used = 0;
}

void drop_graphs(IppCtx* c) {
  for (auto& g : c->graphs) {
    if (g.exec) hipGraphExecDestroy(g.exec);
    if (g.graph) hipGraphDestroy(g.graph);
  }
  c->graphs.clear();
}

constexpr int64_t kMaxDim = 32767;
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

ipp_status fail(IppCtx* c, ipp_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

void tile_shape(const ipp_params& p, int* th, int* tw) {
  if (p.tile_h == 32 && p.tile_w == 128) { *th = 32; *tw = 128; return; }
  if (p.tile_h == 128 && p.tile_w == 32) { *th = 128; *tw = 32; return; }
  *th = 64; *tw = 64;
}

std::string check_params(const ipp_params* p) {
  if (!p) return "params is NULL";
  auto bad = [](double v) { return !std::isfinite(v); };
  if (p->mesh_h < 16 || p->mesh_h > 128 || p->mesh_w < 16 || p->mesh_w > 128)
    return "mesh_h and mesh_w must be in [16, 128]";
  if (p->filter_h < 1 || p->filter_h > 7 || !(p->filter_h & 1) ||
      p->filter_w < 1 || p->filter_w > 7 || !(p->filter_w & 1))
    return "filter_h and filter_w must be odd and in [1, 7]";
  if (p->clip_iters < 0 || p->clip_iters > 16)
    return "clip_iters must be in [0, 16]";
  if (bad(p->clip_sigma) || p->clip_sigma <= 0) return "clip_sigma must be > 0";
  if (p->estimator < IPP_EST_SEXTRACTOR || p->estimator > IPP_EST_MODE)
    return "unknown estimator";
  if (bad(p->median_factor) || bad(p->mean_factor))
    return "median_factor and mean_factor must be finite";
  if (p->min_valid < 1) return "min_valid must be >= 1";
  if (p->min_area < 1) return "min_area must be >= 1";
  if (bad(p->det_nsigma)) return "det_nsigma must be finite";
  if (p->connectivity != 4 && p->connectivity != 8)
    return "connectivity must be 4 or 8";
  if (p->sky_clip_iters < 0 || p->sky_clip_iters > 16)
    return "sky_clip_iters must be in [0, 16]";
  if (bad(p->sky_clip_sigma) || p->sky_clip_sigma <= 0)
    return "sky_clip_sigma must be > 0";
  if (bad(p->r_ap) || p->r_ap <= 0 || p->r_ap > 16)
    return "r_ap must be in (0, 16]";
  if (bad(p->r_in) || bad(p->r_out) || p->r_in < 0 || p->r_out <= p->r_in ||
      p->r_out > 16)
    return "annulus radii must satisfy 0 <= r_in < r_out <= 16";
  const bool shape_ok = (p->tile_h == 0 && p->tile_w == 0) ||
                        (p->tile_h == 64 && p->tile_w == 64) ||
                        (p->tile_h == 32 && p->tile_w == 128) ||
                        (p->tile_h == 128 && p->tile_w == 32);
  if (!shape_ok) return "tile shape must be 0x0, 64x64, 32x128 or 128x32";
  return "";
}

std::string check_frames(const ipp_frame* f, int32_t n) {
  if (!f) return "frames is NULL";
  if (n < 1 || n > 65536) return "frame count must be in [1, 65536]";
  for (int i = 0; i < n; ++i) {
    if (!f[i].pix) return "frame " + std::to_string(i) + ": pix is NULL";
    if (f[i].h < 1 || f[i].w < 1 || f[i].h > kMaxDim || f[i].w > kMaxDim)
      return "frame " + std::to_string(i) + ": size must be 1..32767";
    if (f[i].pitch < f[i].w)
      return "frame " + std::to_string(i) + ": pitch < w";
    if (f[i].pitch > (1 << 24))
      return "frame " + std::to_string(i) + ": pitch must be at most 2^24";
  }
  return "";
}

// Workspace layout of one call.
struct Plan {
  std::vector<FrameDev> fd;
  int32_t nodes = 0, dtiles = 0, rows = 0, lines[2] = {0, 0};
  int64_t pix = 0;
  int64_t rec_cap = 0;
  int th = 64, tw = 64;
  // byte offsets
  size_t o_frames, o_mbkg, o_mrms, o_mn, o_fbkg, o_frms, o_fpass, o_tb[4],
      o_tr[4], o_sc0, o_sc1, o_flags, o_tmap, o_tedge, o_rbase, o_recs,
      o_rparent,
      o_rlabel, o_bucket, o_rowc, o_rows, o_rowcur, o_scanb, o_cnt, total;
};

enum PlanMode { kPlanMesh = 0, kPlanDetect = 1, kPlanFrames = 2 };

Plan make_plan(const ipp_frame* f, int32_t n, const ipp_params& p,
               int64_t rec_cap, int mode = kPlanDetect) {
  Plan P;
  tile_shape(p, &P.th, &P.tw);
  P.fd.resize(n);
  for (int i = 0; i < n; ++i) {
    FrameDev& d = P.fd[i];
    std::memset(&d, 0, sizeof(d));
    d.pix = f[i].pix;
    d.mask = f[i].mask;
    d.pitch = f[i].pitch;
    d.h = f[i].h;
    d.w = f[i].w;
    d.ny = (f[i].h + p.mesh_h - 1) / p.mesh_h;
    d.nx = (f[i].w + p.mesh_w - 1) / p.mesh_w;
    d.node0 = P.nodes;
    P.nodes += d.ny * d.nx;
    d.line0[0] = P.lines[0];
    P.lines[0] += 2 * (d.ny + d.nx);
    d.line0[1] = P.lines[1];
    P.lines[1] += 2 * d.nx;
    d.dty = (f[i].h + P.th - 1) / P.th;
    d.dtx = (f[i].w + P.tw - 1) / P.tw;
    d.dtile0 = P.dtiles;
    P.dtiles += d.dty * d.dtx;
    d.row0 = P.rows;
    P.rows += f[i].h;
    d.pix0 = P.pix;
    P.pix += (int64_t)f[i].h * f[i].w;
  }
  P.rec_cap = rec_cap > 0 ? rec_cap : P.pix / 32 + 4096;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += align_up(bytes); return r; };
  const size_t N = mode == kPlanFrames ? 0 : (size_t)P.nodes;
  if (mode != kPlanDetect) {
    P.rec_cap = 0;
    P.rows = mode == kPlanFrames ? 0 : P.rows;
  }
  const int64_t npix = mode == kPlanDetect ? P.pix : 0;
  P.o_frames = take(sizeof(FrameDev) * n);
  P.o_mbkg = take(8 * N);
  P.o_mrms = take(8 * N);
  P.o_mn = take(4 * N);
  P.o_fbkg = take(8 * N);
  P.o_frms = take(8 * N);
  P.o_fpass = take(4 * N);
  for (int k = 0; k < 4; ++k) P.o_tb[k] = take(8 * N);
  for (int k = 0; k < 4; ++k) P.o_tr[k] = take(8 * N);
  P.o_sc0 = take(8 * 4 * N);
  P.o_sc1 = take(8 * 4 * N);
  P.o_flags = take(4 * (size_t)n);
  P.o_tmap = take((size_t)kTmapBytes *
                  (size_t)(mode == kPlanDetect ? P.dtiles : 0));
  P.o_tedge = take(4 * (size_t)kEdgeInts *
                   (size_t)(mode == kPlanDetect ? P.dtiles : 0));
  P.o_rbase = take(4 * (size_t)(mode == kPlanDetect ? P.dtiles : 0));
  P.o_recs = take(sizeof(Rec) * (size_t)P.rec_cap);
  P.o_rparent = take(4 * (size_t)P.rec_cap);
  P.o_rlabel = take(4 * (size_t)P.rec_cap);
  P.o_bucket = take(4 * (size_t)P.rec_cap);
  P.o_rowc = take(4 * (size_t)P.rows);
  P.o_rows = take(4 * (size_t)P.rows);
  P.o_rowcur = take(4 * (size_t)P.rows);
  P.o_scanb = take(4 * (size_t)((P.rows + 1023) / 1024 + 1));
  P.o_cnt = take(8 * 4);
  P.total = o;
  return P;
}

Work make_work(const Plan& P, void* ws, int32_t n) {
  Work w;
  std::memset(&w, 0, sizeof(w));
  char* b = (char*)ws;
  w.frames = (FrameDev*)(b + P.o_frames);
  w.nframes = n;
  w.total_nodes = P.nodes;
  w.total_dtiles = P.dtiles;
  w.total_rows = P.rows;
  w.total_lines[0] = P.lines[0];
  w.total_lines[1] = P.lines[1];
  w.total_pix = P.pix;
  w.m_bkg = (double*)(b + P.o_mbkg);
  w.m_rms = (double*)(b + P.o_mrms);
  w.m_n = (int32_t*)(b + P.o_mn);
  w.f_bkg = (double*)(b + P.o_fbkg);
  w.f_rms = (double*)(b + P.o_frms);
  w.f_pass = (int32_t*)(b + P.o_fpass);
  for (int k = 0; k < 4; ++k) {
    w.tb[k] = (double*)(b + P.o_tb[k]);
    w.tr[k] = (double*)(b + P.o_tr[k]);
  }
  w.sc0 = (double*)(b + P.o_sc0);
  w.sc1 = (double*)(b + P.o_sc1);
  w.frame_flags = (uint32_t*)(b + P.o_flags);
  w.tmap = (uint8_t*)(b + P.o_tmap);
  w.tedge = (int32_t*)(b + P.o_tedge);
  w.tile_rbase = (int32_t*)(b + P.o_rbase);
  w.recs = (Rec*)(b + P.o_recs);
  w.rparent = (int32_t*)(b + P.o_rparent);
  w.rlabel = (int32_t*)(b + P.o_rlabel);
  w.rec_cap = P.rec_cap;
  w.bucket = (int32_t*)(b + P.o_bucket);
  w.row_count = (int32_t*)(b + P.o_rowc);
  w.row_start = (int32_t*)(b + P.o_rows);
  w.row_cursor = (int32_t*)(b + P.o_rowcur);
  w.scan_blocks = (int32_t*)(b + P.o_scanb);
  w.counters = (int64_t*)(b + P.o_cnt);
  return w;
}

// Launch with error check; with profiling on, the launch is bracketed by
// a pair of events recorded on the same stream.
#define IPP_LAUNCH(c, s, name, ...)                                         \
  do {                                                                      \
    ProfSlot* ps_ = prof_begin(c, s, name);                                 \
    __VA_ARGS__;                                                            \
    hipError_t e_ = hipGetLastError();                                      \
    if (e_ != hipSuccess)                                                   \
      return fail(c, IPP_E_DEVICE,                                          \
                  std::string("kernel launch failed: ") +                   \
                      hipGetErrorString(e_));                               \
    prof_end(ps_, s);                                                       \
  } while (0)

int grid_for(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

ipp_status upload(IppCtx* c, const Plan& P, const Work& w,
                  hipStream_t s) {
  hipError_t e = hipMemcpyAsync(w.frames, P.fd.data(),
                                sizeof(FrameDev) * P.fd.size(),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess)
    return fail(c, IPP_E_DEVICE,
                std::string("descriptor upload failed: ") +
                    hipGetErrorString(e));
  return IPP_OK;
}

// Validates and lays out a call.  In detection mode the record capacity
// is the largest that fits in the reserved workspace.
ipp_status prepare(IppCtx* c, const ipp_frame* frames, int32_t n,
                   const ipp_params* p, int mode, Plan* P) {
  if (!c) return IPP_E_INVALID_ARG;
  std::string m = check_params(p);
  if (!m.empty()) return fail(c, IPP_E_INVALID_ARG, m);
  m = check_frames(frames, n);
  if (!m.empty()) return fail(c, IPP_E_INVALID_ARG, m);
  *P = make_plan(frames, n, *p, 1, mode);
  if (mode == kPlanDetect && P->total <= c->ws_bytes) {
    const size_t per = sizeof(Rec) + 3 * sizeof(int32_t);
    int64_t cap = (int64_t)((c->ws_bytes - P->total) / per) + 1;
    if (cap > (1ll << 31) - 1024) cap = (1ll << 31) - 1024;
    for (;;) {
      Plan Q = make_plan(frames, n, *p, cap, mode);
      if (Q.total <= c->ws_bytes || cap <= 1) { *P = Q; break; }
      cap -= 256;
      if (cap < 1) cap = 1;
    }
  }
  if (P->rows > (1 << 20))
    return fail(c, IPP_E_UNSUPPORTED, "more than 2^20 rows in one batch");
  if (P->total > c->ws_bytes)
    return fail(c, IPP_E_WORKSPACE,
                "workspace too small: need " + std::to_string(P->total) +
                    " bytes, have " + std::to_string(c->ws_bytes));
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess)
    return fail(c, IPP_E_DEVICE, std::string("hipSetDevice: ") +
                                     hipGetErrorString(e));
  return IPP_OK;
}


void key_put(std::vector<uint8_t>& key, const void* d, size_t len) {
  const uint8_t* b = (const uint8_t*)d;
  key.insert(key.end(), b, b + len);
}

// Enqueues a kernel sequence through the context's graph cache: the first
// call with a given signature `key` (everything the kernels bake in)
// captures body(stream) into a HIP graph on the private capture stream;
// later calls replay it.  The frame descriptors are uploaded outside the
// graph, and only when they or the workspace changed since the last upload
// for that graph.
template <typename Body>
ipp_status run_cached(IppCtx* c, std::vector<uint8_t> key, const Plan& P,
                      const Work& w, hipStream_t s, Body body) {
  ipp_status st;
  IppGraph* G = nullptr;
  for (auto& g : c->graphs)
    if (g.key == key) G = &g;
  const uint8_t* fdb = (const uint8_t*)P.fd.data();
  std::vector<uint8_t> fdv(fdb, fdb + sizeof(FrameDev) * P.fd.size());
  if (!G) {
    if (c->graphs.size() >= 6) {            // evict the least recently used
      size_t lru = 0;
      for (size_t i = 1; i < c->graphs.size(); ++i)
        if (c->graphs[i].last_use < c->graphs[lru].last_use) lru = i;
      if (c->graphs[lru].exec) hipGraphExecDestroy(c->graphs[lru].exec);
      if (c->graphs[lru].graph) hipGraphDestroy(c->graphs[lru].graph);
      c->graphs.erase(c->graphs.begin() + lru);
    }
    if (!c->cap &&
        hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess)
      return fail(c, IPP_E_DEVICE, "cannot create the capture stream");
    IppGraph g;
    g.key = std::move(key);
    if (hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal) !=
        hipSuccess)
      return fail(c, IPP_E_DEVICE, "hipStreamBeginCapture failed");
    st = body(c->cap);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap, &graph);
    if (st != IPP_OK || e != hipSuccess) {
      if (graph) hipGraphDestroy(graph);
      return st != IPP_OK ? st
                          : fail(c, IPP_E_DEVICE, "hipStreamEndCapture failed");
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) !=
        hipSuccess) {
      hipGraphDestroy(graph);
      return fail(c, IPP_E_DEVICE, "hipGraphInstantiate failed");
    }
    g.graph = graph;
    g.exec = exec;
    c->graphs.push_back(std::move(g));
    G = &c->graphs.back();
  }
  G->last_use = ++c->tick;
  if (G->ws_gen != c->ws_gen || G->fd != fdv) {
    if ((st = upload(c, P, w, s)) != IPP_OK) return st;
    ++c->ws_gen;
    G->ws_gen = c->ws_gen;
    G->fd = fdv;
  }
  const hipError_t e = hipGraphLaunch(G->exec, s);
  if (e != hipSuccess)
    return fail(c, IPP_E_DEVICE, std::string("hipGraphLaunch: ") +
                                     hipGetErrorString(e));
  return IPP_OK;
}

// ---- kernel sequences --------------------------------------------------
ipp_status run_mesh(IppCtx* c, const Plan& P, const Work& w,
                    const ipp_params& p, hipStream_t s) {
  const int area = p.mesh_h * p.mesh_w;
  const dim3 gw((P.nodes + kWaves - 1) / kWaves);
  if (area <= 16 * kWave)
    IPP_LAUNCH(c, s, "k_mesh_stats",
               hipLaunchKernelGGL(k_mesh_stats_w<16>, gw, dim3(kBlock), 0, s,
                                  w, p));
  else if (area <= 64 * kWave)
    IPP_LAUNCH(c, s, "k_mesh_stats",
               hipLaunchKernelGGL(k_mesh_stats_w<64>, gw, dim3(kBlock), 0, s,
                                  w, p));
  else
    IPP_LAUNCH(c, s, "k_mesh_stats",
               hipLaunchKernelGGL(k_mesh_stats<64>, dim3(P.nodes),
                                  dim3(kBlock), 0, s, w, p));
  IPP_LAUNCH(c, s, "k_mesh_fill",
             hipLaunchKernelGGL(k_mesh_fill, dim3((int)P.fd.size()),
                                dim3(kBlock), 0, s, w, p));
  const dim3 gn(grid_for(P.nodes, kBlock, 1 << 30));
  const int fmax = std::max(p.filter_h, p.filter_w) / 2;
  if (fmax <= 1)
    IPP_LAUNCH(c, s, "k_mesh_filter",
               hipLaunchKernelGGL((k_mesh_filter<1>), gn, dim3(kBlock), 0, s,
                                  w, p));
  else if (fmax == 2)
    IPP_LAUNCH(c, s, "k_mesh_filter",
               hipLaunchKernelGGL((k_mesh_filter<2>), gn, dim3(kBlock), 0, s,
                                  w, p));
  else
    IPP_LAUNCH(c, s, "k_mesh_filter",
               hipLaunchKernelGGL((k_mesh_filter<3>), gn, dim3(kBlock), 0, s,
                                  w, p));
  IPP_LAUNCH(c, s, "k_mesh_spline",
             hipLaunchKernelGGL((k_mesh_spline<0>),
                                dim3(grid_for(P.lines[0], 64, 1 << 30)),
                                dim3(64), 0, s, w, p));
  IPP_LAUNCH(c, s, "k_mesh_spline",
             hipLaunchKernelGGL((k_mesh_spline<1>),
                                dim3(grid_for(P.lines[1], 64, 1 << 30)),
                                dim3(64), 0, s, w, p));
  return IPP_OK;
}

template <int TH, int TW>
ipp_status run_bkg_maps(IppCtx* c, const Plan& P, const Work& w,
                        const ipp_params& p, hipStream_t s) {
  IPP_LAUNCH(c, s, "k_bkg_maps", hipLaunchKernelGGL((k_bkg_maps<TH, TW>), dim3(P.dtiles),
                                   dim3(kBlock), 0, s, w, p));
  return IPP_OK;
}

template <int TH, int TW>
ipp_status run_tile(IppCtx* c, const Plan& P, const Work& w,
                    const ipp_params& p, bool fused, int write_rms,
                    hipStream_t s) {
  const dim3 g(P.dtiles), b(kBlock), bt(kTileThreads);
  if (fused && p.connectivity == 8)
    IPP_LAUNCH(c, s, "k_tile_ccl_fused", hipLaunchKernelGGL((k_tile_ccl<TH, TW, true, true, kTileThreads>), g, bt,
                                     0, s, w, p, write_rms));
  else if (fused)
    IPP_LAUNCH(c, s, "k_tile_ccl_fused", hipLaunchKernelGGL((k_tile_ccl<TH, TW, true, false, kTileThreads>), g,
                                     bt, 0, s, w, p, write_rms));
  else if (p.connectivity == 8)
    IPP_LAUNCH(c, s, "k_tile_ccl", hipLaunchKernelGGL((k_tile_ccl<TH, TW, false, true, kTileThreads>), g,
                                     bt, 0, s, w, p, write_rms));
  else
    IPP_LAUNCH(c, s, "k_tile_ccl", hipLaunchKernelGGL((k_tile_ccl<TH, TW, false, false, kTileThreads>), g,
                                     bt, 0, s, w, p, write_rms));
  IPP_LAUNCH(c, s, "k_border", hipLaunchKernelGGL((k_border<TH, TW>), g,
                                   dim3(border_threads<TH, TW>()), 0, s, w, p));
  return IPP_OK;
}

template <int TH, int TW>
ipp_status run_relabel(IppCtx* c, const Plan& P, const Work& w,
                       const ipp_params& p, hipStream_t s) {
  IPP_LAUNCH(c, s, "k_relabel", hipLaunchKernelGGL((k_relabel<TH, TW>), dim3(P.dtiles),
                                   dim3(kBlock), 0, s, w, p));
  return IPP_OK;
}

__global__ void k_diag(Work w, int64_t* diag) {
  if (threadIdx.x == 0) {
    diag[0] = w.counters[0];
    diag[1] = w.rec_cap;
    diag[2] = w.counters[2];
    diag[3] = w.counters[3];
  }
}

// Detection after the tile kernel choice: fill, tiles, merge, number,
// relabel, measure.
ipp_status run_detect(IppCtx* c, const Plan& P, const Work& w,
                      const ipp_params& p, ipp_sources* src, bool fused,
                      int write_rms, int64_t* diag, hipStream_t s) {
  IPP_LAUNCH(c, s, "k_fill_i64", hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, s,
                                   w.counters, (int64_t)4, (int64_t)0));
  IPP_LAUNCH(c, s, "k_fill_i32", hipLaunchKernelGGL(k_fill_i32,
                                   dim3(grid_for(P.rows, kBlock, 4096)),
                                   dim3(kBlock), 0, s, w.row_count,
                                   (int64_t)P.rows, 0));
  IPP_LAUNCH(c, s, "k_fill_i32", hipLaunchKernelGGL(k_fill_i32,
                                   dim3(grid_for(P.rows, kBlock, 4096)),
                                   dim3(kBlock), 0, s, w.row_cursor,
                                   (int64_t)P.rows, 0));
  ipp_status st;
  if (P.th == 32) st = run_tile<32, 128>(c, P, w, p, fused, write_rms, s);
  else if (P.th == 128) st = run_tile<128, 32>(c, P, w, p, fused, write_rms, s);
  else st = run_tile<64, 64>(c, P, w, p, fused, write_rms, s);
  if (st != IPP_OK) return st;
  const int gr = grid_for(P.rec_cap, kBlock, 2048);
  IPP_LAUNCH(c, s, "k_resolve", hipLaunchKernelGGL(k_resolve, dim3(gr), dim3(kBlock), 0, s,
                                   w, p));
  IPP_LAUNCH(c, s, "k_heads", hipLaunchKernelGGL(k_heads, dim3(gr), dim3(kBlock), 0, s, w,
                                   p));
  const int nb = (P.rows + 1023) / 1024;
  IPP_LAUNCH(c, s, "k_scan_blocks", hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(kBlock), 0,
                                   s, w.row_count, w.scan_blocks, P.rows));
  IPP_LAUNCH(c, s, "k_scan_top", hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s,
                                   w.scan_blocks, nb, w.counters + 3));
  IPP_LAUNCH(c, s, "k_scan_apply", hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kBlock), 0,
                                   s, w.row_count, w.scan_blocks,
                                   w.row_start, P.rows));
  IPP_LAUNCH(c, s, "k_frame_offsets", hipLaunchKernelGGL(k_frame_offsets,
                                   dim3(grid_for((int64_t)P.fd.size() + 1,
                                                 kBlock, 4096)),
                                   dim3(kBlock), 0, s, w, *src));
  IPP_LAUNCH(c, s, "k_scatter", hipLaunchKernelGGL(k_scatter, dim3(gr), dim3(kBlock), 0, s,
                                   w, p));
  IPP_LAUNCH(c, s, "k_rank", hipLaunchKernelGGL(k_rank, dim3(gr), dim3(kBlock), 0, s, w,
                                   p, *src));
  IPP_LAUNCH(c, s, "k_reclabel", hipLaunchKernelGGL(k_reclabel, dim3(gr), dim3(kBlock), 0, s,
                                   w));
  if (P.th == 32) st = run_relabel<32, 128>(c, P, w, p, s);
  else if (P.th == 128) st = run_relabel<128, 32>(c, P, w, p, s);
  else st = run_relabel<64, 64>(c, P, w, p, s);
  if (st != IPP_OK) return st;
  IPP_LAUNCH(c, s, "k_source_stats", hipLaunchKernelGGL(k_source_stats,
                                   dim3(grid_for(src->capacity, 4, 4096)),
                                   dim3(kBlock), 0, s, w, *src));
  if (diag)
    IPP_LAUNCH(c, s, "k_diag", hipLaunchKernelGGL(k_diag, dim3(1), dim3(64), 0, s, w,
                                     diag));
  return IPP_OK;
}

// Aperture photometry: one wavefront per source.  NS bounds the annulus
// pixel count: a pixel meeting the disk of radius r_out has its centre
// within r_out + sqrt(2)/2, and every pixel with its centre within
// r_in - sqrt(2)/2 lies inside the disk of radius r_in, so by the lattice
// point bound the ring holds at most pi((r_out+sqrt2)^2 - (r_in-sqrt2)^2).
ipp_status run_aperture(IppCtx* c, const Work& w, const ipp_params& p,
                        ipp_sources* src, double* sky_lohi, hipStream_t s) {
  const double ri = p.r_in > std::sqrt(2.0) ? p.r_in - std::sqrt(2.0) : 0.0;
  const double ro = p.r_out + std::sqrt(2.0);
  const double ring = M_PI * (ro * ro - ri * ri) + 16.0;
  const int grid = grid_for(src->capacity, kWaves, 16384);
  const dim3 g(grid), b(kBlock);
  if (ring <= 256) {
    IPP_LAUNCH(c, s, "k_aperture", hipLaunchKernelGGL((k_aperture_t<256>),
               g, b, 0, s, w, p, *src, sky_lohi));
  } else if (ring <= 512) {
    IPP_LAUNCH(c, s, "k_aperture", hipLaunchKernelGGL((k_aperture_t<512>),
               g, b, 0, s, w, p, *src, sky_lohi));
  } else if (ring <= 1024) {
    IPP_LAUNCH(c, s, "k_aperture", hipLaunchKernelGGL((k_aperture_t<1024>),
               g, b, 0, s, w, p, *src, sky_lohi));
  } else {
    return fail(c, IPP_E_UNSUPPORTED, "aperture radii too large");
  }
  return IPP_OK;
}

// Backward of the aperture photometry: one wavefront per source.
ipp_status run_aperture_bwd(IppCtx* c, const Work& w, const ipp_params& p,
                            const ipp_sources& src, const double* sky_lohi,
                            const double* gF, double* dxy, hipStream_t s) {
  const double ri = p.r_in > std::sqrt(2.0) ? p.r_in - std::sqrt(2.0) : 0.0;
  const double ro = p.r_out + std::sqrt(2.0);
  const double ring = M_PI * (ro * ro - ri * ri) + 16.0;
  const dim3 g(grid_for(src.capacity, kWaves, 16384)), b(kBlock);
  if (ring <= 256)
    IPP_LAUNCH(c, s, "k_aperture_bwd",
               hipLaunchKernelGGL((k_aperture_bwd_t<256>), g, b, 0, s, w, p,
                                  src, sky_lohi, gF, dxy));
  else if (ring <= 512)
    IPP_LAUNCH(c, s, "k_aperture_bwd",
               hipLaunchKernelGGL((k_aperture_bwd_t<512>), g, b, 0, s, w, p,
                                  src, sky_lohi, gF, dxy));
  else if (ring <= 1024)
    IPP_LAUNCH(c, s, "k_aperture_bwd",
               hipLaunchKernelGGL((k_aperture_bwd_t<1024>), g, b, 0, s, w, p,
                                  src, sky_lohi, gF, dxy));
  else
    return fail(c, IPP_E_UNSUPPORTED, "aperture radii too large");
  return IPP_OK;
}

// Centroid refinement: one launch; each wavefront takes a row through the
// normaliser F_ap(c0) and all `steps` forward, gradient and update rounds.
ipp_status run_refine(IppCtx* c, const Work& w, const ipp_params& p,
                      const ipp_sources& src, double r_c, double eta,
                      int steps, double* xo, double* yo, hipStream_t s) {
  const double ri = p.r_in > std::sqrt(2.0) ? p.r_in - std::sqrt(2.0) : 0.0;
  const double ro = p.r_out + std::sqrt(2.0);
  const double ring = M_PI * (ro * ro - ri * ri) + 16.0;
  const dim3 g(grid_for(src.capacity, kWaves, 16384)), b(kBlock);
  const bool phot = (p.flags & IPP_F_REFINE_PHOTOMETRY) != 0;
#define IPP_REFINE(NS)                                                       \
  do {                                                                       \
    if (phot)                                                                \
      IPP_LAUNCH(c, s, "k_refine",                                           \
                 hipLaunchKernelGGL((k_refine_t<NS, true>), g, b, 0, s, w,   \
                                    p, r_c, eta, steps, src, xo, yo));       \
    else                                                                     \
      IPP_LAUNCH(c, s, "k_refine",                                           \
                 hipLaunchKernelGGL((k_refine_t<NS, false>), g, b, 0, s, w,  \
                                    p, r_c, eta, steps, src, xo, yo));       \
  } while (0)
  if (ring <= 256)
    IPP_REFINE(256);
  else if (ring <= 512)
    IPP_REFINE(512);
  else if (ring <= 1024)
    IPP_REFINE(1024);
#undef IPP_REFINE
  else
    return fail(c, IPP_E_UNSUPPORTED, "aperture radii too large");
  return IPP_OK;
}

// Deblending: fixed per-call arrays after the frame descriptors, then the
// scratch pool (the rest of the workspace).
struct DeblendWs {
  size_t o_fd2, o_need, o_off, o_cnt, o_ooff, o_blk, o_tot, o_big, o_pool;
  int64_t nblk;
};

DeblendWs deblend_layout(size_t base, int32_t n, int64_t cap) {
  DeblendWs D;
  size_t o = align_up(base);
  auto take = [&](size_t bytes) { size_t r = o; o += align_up(bytes); return r; };
  const size_t rows = (size_t)cap + 1;
  D.nblk = (int64_t)((rows + 1023) / 1024);
  D.o_fd2 = take(sizeof(FrameDev) * (size_t)n);
  D.o_need = take(8 * rows);
  D.o_off = take(8 * rows);
  D.o_cnt = take(8 * rows);
  D.o_ooff = take(8 * rows);
  D.o_blk = take(8 * (size_t)(D.nblk + 1));
  D.o_tot = take(8 * 8);
  D.o_big = take(4 * rows);
  D.o_pool = o;
  return D;
}

ipp_status scan64(IppCtx* c, const int64_t* in, int64_t* blk, int64_t nblk,
                  int64_t* out, int64_t n, int64_t* total, hipStream_t s) {
  IPP_LAUNCH(c, s, "k_scan64_blocks",
             hipLaunchKernelGGL(k_scan64_blocks, dim3((unsigned)nblk),
                                dim3(kBlock), 0, s, in, blk, n));
  IPP_LAUNCH(c, s, "k_scan64_top",
             hipLaunchKernelGGL(k_scan64_top, dim3(1), dim3(kBlock), 0, s,
                                blk, nblk, total));
  IPP_LAUNCH(c, s, "k_scan64_apply",
             hipLaunchKernelGGL(k_scan64_apply, dim3((unsigned)nblk),
                                dim3(kBlock), 0, s, in, blk, out, n));
  return IPP_OK;
}

// The whole fused batch sequence (also what a captured graph contains).
ipp_status run_batch(IppCtx* c, const Plan& P, const Work& w,
                     const ipp_params& p, ipp_sources* src, int write_rms,
                     int64_t* diag, hipStream_t s) {
  ipp_status st;
  if ((st = run_mesh(c, P, w, p, s)) != IPP_OK) return st;
  if ((st = run_detect(c, P, w, p, src, true, write_rms, diag, s)) != IPP_OK)
    return st;
  if (p.flags & IPP_F_NO_PHOTOMETRY) return IPP_OK;
  return run_aperture(c, w, p, src, nullptr, s);
}

std::string check_sources(const ipp_sources* s, bool detect) {
  if (!s) return "sources is NULL";
  if (s->capacity < 0) return "sources capacity < 0";
  if (!s->frame || !s->x || !s->y || !s->flags)
    return "sources: frame, x, y and flags are required";
  if (detect) {
    if (!s->n_total || !s->frame_offsets || !s->label || !s->npix ||
        !s->xmin || !s->xmax || !s->ymin || !s->ymax || !s->peak_x ||
        !s->peak_y || !s->peak || !s->flux_iso)
      return "sources: every detection column is required";
  } else {
    if (!s->flux_ap || !s->sky || !s->area_ap || !s->area_ann)
      return "sources: flux_ap, sky, area_ap and area_ann are required";
  }
  return "";
}

// ---------------------------------------------------------------------
// Gray-scale calls (Sec. 2.2.6): descriptors and workspace layout.
// ---------------------------------------------------------------------
struct GrayPlan {
  std::vector<GrayFrame> fr;
  int rows = 0;
  size_t o_frames = 0, o_mm = 0, o_counts = 0, o_cdf = 0, total = 0;
};

// Smallest step s >= 1 with ceil(h/s) * ceil(w/s) <= nsamples.
int zscale_step(int h, int w, int nsamples) {
  int s = (int)std::floor(std::sqrt((double)h * (double)w / nsamples)) - 1;
  if (s < 1) s = 1;
  auto pts = [&](int k) {
    return (int64_t)((h + k - 1) / k) * (int64_t)((w + k - 1) / k);
  };
  while (s > 1 && pts(s - 1) <= nsamples) --s;
  while (pts(s) > nsamples) ++s;
  return s;
}

size_t gray_layout(int32_t n, int32_t nbins, GrayPlan* G) {
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += align_up(bytes); return r; };
  G->o_frames = take(sizeof(GrayFrame) * (size_t)n);
  G->o_mm = take(sizeof(uint32_t) * 2 * (size_t)n);
  G->o_counts = take(sizeof(uint32_t) * (size_t)n * (size_t)nbins);
  G->o_cdf = take(sizeof(double) * (size_t)n * (size_t)nbins);
  G->total = o;
  return o;
}

// Validates the frames and outputs, fills the descriptors and uploads them
// into the workspace.
ipp_status gray_prepare(IppCtx* c, const ipp_frame* frames, int32_t n,
                        int32_t nsamples, int32_t nbins, float* const* out,
                        bool need_out, GrayPlan* G, hipStream_t s) {
  if (!c) return IPP_E_INVALID_ARG;
  std::string m = check_frames(frames, n);
  if (!m.empty()) return fail(c, IPP_E_INVALID_ARG, m);
  if (need_out) {
    if (!out) return fail(c, IPP_E_INVALID_ARG, "out is NULL");
    for (int i = 0; i < n; ++i)
      if (!out[i])
        return fail(c, IPP_E_INVALID_ARG,
                    "out[" + std::to_string(i) + "] is NULL");
  }
  gray_layout(n, nbins, G);
  if (G->total > c->ws_bytes)
    return fail(c, IPP_E_WORKSPACE,
                "workspace too small: need " + std::to_string(G->total) +
                    " bytes, have " + std::to_string(c->ws_bytes));
  G->fr.resize(n);
  int64_t rows = 0;
  for (int i = 0; i < n; ++i) {
    GrayFrame& g = G->fr[i];
    g.pix = frames[i].pix;
    g.pitch = frames[i].pitch;
    g.h = frames[i].h;
    g.w = frames[i].w;
    g.s = nsamples > 0 ? zscale_step(g.h, g.w, nsamples) : 1;
    g.sy = (g.h + g.s - 1) / g.s;
    g.sx = (g.w + g.s - 1) / g.s;
    g.row0 = (int32_t)rows;
    g.out = out ? out[i] : nullptr;
    rows += g.h;
    if (nsamples > 0 && (int64_t)g.sy * g.sx > kZMax)
      return fail(c, IPP_E_INVALID_ARG, "zscale sample grid too large");
  }
  if (rows > (1 << 30))
    return fail(c, IPP_E_UNSUPPORTED, "more than 2^30 rows in one batch");
  G->rows = (int)rows;
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess)
    e = hipMemcpyAsync((char*)c->ws + G->o_frames, G->fr.data(),
                       sizeof(GrayFrame) * G->fr.size(),
                       hipMemcpyHostToDevice, s);
  if (e != hipSuccess)
    return fail(c, IPP_E_DEVICE, std::string("descriptor upload failed: ") +
                                     hipGetErrorString(e));
  ++c->ws_gen;
  return IPP_OK;
}

}  // namespace

// ===================================================================== API
extern "C" {

int32_t ipp_version(void) { return IPP_API_VERSION; }

const char* ipp_status_string(int32_t s) {
  switch (s) {
    case IPP_OK: return "ok";
    case IPP_E_INVALID_ARG: return "invalid argument";
    case IPP_E_UNSUPPORTED: return "unsupported";
    case IPP_E_CAPACITY: return "capacity exceeded";
    case IPP_E_DEVICE: return "device error";
    case IPP_E_WORKSPACE: return "workspace too small";
    default: return "unknown status";
  }
}

void ipp_params_default(ipp_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->mesh_h = p->mesh_w = 64;
  p->filter_h = p->filter_w = 3;
  p->clip_iters = 3;
  p->estimator = IPP_EST_SEXTRACTOR;
  p->clip_sigma = 3.0;
  p->median_factor = 3.0;
  p->mean_factor = 2.0;
  p->min_valid = 100;
  p->min_area = 5;
  p->det_nsigma = 1.5;
  p->connectivity = 8;
  p->sky_clip_iters = 3;
  p->sky_clip_sigma = 3.0;
  p->r_ap = 5.0;
  p->r_in = 8.0;
  p->r_out = 12.0;
  p->tile_h = p->tile_w = 0;
  p->flags = 0;
}

ipp_status ipp_params_validate(const ipp_params* p) {
  return check_params(p).empty() ? IPP_OK : IPP_E_INVALID_ARG;
}

ipp_status ipp_ctx_create(void** ctx, int32_t device) {
  if (!ctx) return IPP_E_INVALID_ARG;
  *ctx = nullptr;
  if (device < 0) return IPP_E_INVALID_ARG;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device >= count)
    return IPP_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return IPP_E_DEVICE;
  // the allocation-free calls find their scratch at this device's address
  double* scratch_ptr = nullptr;
  if (asinh_scratch(device, &scratch_ptr) != hipSuccess) return IPP_E_DEVICE;
  IppCtx* c = new (std::nothrow) IppCtx();
  if (!c) return IPP_E_DEVICE;
  c->device = device;
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount,
                            device) == hipSuccess && ncu > 0)
    c->n_cu = ncu;
  *ctx = c;
  return IPP_OK;
}

ipp_status ipp_ctx_destroy(void* ctx) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  hipSetDevice(c->device);
  drop_graphs(c);
  if (c->cap) hipStreamDestroy(c->cap);
  if (c->ws) hipFree(c->ws);
  for (auto& ps : c->pool) {
    hipEventDestroy(ps.a);
    hipEventDestroy(ps.b);
  }
  delete c;
  return IPP_OK;
}

ipp_status ipp_ctx_reserve(void* ctx, size_t bytes) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (bytes <= c->ws_bytes) return IPP_OK;
  hipSetDevice(c->device);
  drop_graphs(c);                   // graphs hold old workspace addresses
  if (c->ws) {
    hipDeviceSynchronize();
    hipFree(c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess)
    return fail(c, IPP_E_DEVICE, std::string("hipMalloc workspace: ") +
                                     hipGetErrorString(e));
  c->ws = p;
  c->ws_bytes = bytes;
  ++c->ws_gen;
  return IPP_OK;
}

ipp_status ipp_ctx_profile(void* ctx, int32_t on) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (c->prof) prof_collect(c);
  c->prof = on != 0;
  if (c->prof) c->totals.clear();
  return IPP_OK;
}

int32_t ipp_ctx_profile_read(void* ctx, int32_t max, char* names,
                             double* total_ms, int32_t* count) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c || max < 0) return -1;
  prof_collect(c);
  const int n = (int)c->totals.size();
  for (int i = 0; i < n && i < max; ++i) {
    if (names) {
      std::strncpy(names + 32 * i, c->totals[i].first.c_str(), 31);
      names[32 * i + 31] = 0;
    }
    if (total_ms) total_ms[i] = c->totals[i].second.first;
    if (count) count[i] = c->totals[i].second.second;
  }
  return n;
}

const char* ipp_last_error(void* ctx) {
  IppCtx* c = (IppCtx*)ctx;
  return c ? c->err.c_str() : "null context";
}

size_t ipp_workspace_bytes(const ipp_frame* frames, int32_t n,
                           const ipp_params* p, int64_t record_capacity) {
  if (!check_params(p).empty() || !check_frames(frames, n).empty()) return 0;
  if (record_capacity < 0 || record_capacity >= (1ll << 31) - 1024) return 0;
  return make_plan(frames, n, *p, record_capacity, kPlanDetect).total;
}

ipp_status ipp_background(void* ctx, const ipp_frame* frames, int32_t n,
                          const ipp_params* p, const ipp_maps* maps,
                          const ipp_mesh* mesh, uint32_t* frame_flags,
                          void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  Plan P;
  ipp_status st = prepare(c, frames, n, p, kPlanMesh, &P);
  if (st != IPP_OK) return st;
  if (!maps) return fail(c, IPP_E_INVALID_ARG, "maps is NULL");
  for (int i = 0; i < n; ++i) {
    if (!maps[i].bkg || !maps[i].rms)
      return fail(c, IPP_E_INVALID_ARG, "maps[f].bkg and .rms are required");
    P.fd[i].bkg = maps[i].bkg;
    P.fd[i].rms = maps[i].rms;
    if (mesh) {
      P.fd[i].o_bkg_raw = mesh[i].bkg_raw;
      P.fd[i].o_rms_raw = mesh[i].rms_raw;
      P.fd[i].o_n = mesh[i].n_used;
      P.fd[i].o_bkg = mesh[i].bkg;
      P.fd[i].o_rms = mesh[i].rms;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  Work w = make_work(P, c->ws, n);
  if (frame_flags) w.frame_flags = frame_flags;
  ++c->ws_gen;
  if ((st = upload(c, P, w, s)) != IPP_OK) return st;
  if ((st = run_mesh(c, P, w, *p, s)) != IPP_OK) return st;
  if (P.th == 32) return run_bkg_maps<32, 128>(c, P, w, *p, s);
  if (P.th == 128) return run_bkg_maps<128, 32>(c, P, w, *p, s);
  return run_bkg_maps<64, 64>(c, P, w, *p, s);
}

ipp_status ipp_detect(void* ctx, const ipp_frame* frames, int32_t n,
                      const ipp_params* p, const ipp_maps* maps,
                      ipp_sources* src, int64_t* diag, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  std::string m = check_sources(src, true);
  if (!m.empty()) return fail(c, IPP_E_INVALID_ARG, m);
  Plan P;
  ipp_status st = prepare(c, frames, n, p, kPlanDetect, &P);
  if (st != IPP_OK) return st;
  if (!maps) return fail(c, IPP_E_INVALID_ARG, "maps is NULL");
  for (int i = 0; i < n; ++i) {
    if (!maps[i].bkg || !maps[i].rms || !maps[i].labels)
      return fail(c, IPP_E_INVALID_ARG,
                  "maps[f].bkg, .rms and .labels are required");
    P.fd[i].bkg = maps[i].bkg;
    P.fd[i].rms = maps[i].rms;
    P.fd[i].labels = maps[i].labels;
  }
  hipStream_t s = (hipStream_t)stream;
  Work w = make_work(P, c->ws, n);
  ++c->ws_gen;
  if ((st = upload(c, P, w, s)) != IPP_OK) return st;
  return run_detect(c, P, w, *p, src, false, 0, diag, s);
}

ipp_status ipp_photometry(void* ctx, const ipp_frame* frames, int32_t n,
                          const ipp_maps* maps, const ipp_params* p,
                          ipp_sources* src, double* sky_lohi, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  std::string m = check_sources(src, false);
  if (!m.empty()) return fail(c, IPP_E_INVALID_ARG, m);
  Plan P;
  ipp_status st = prepare(c, frames, n, p, kPlanFrames, &P);
  if (st != IPP_OK) return st;
  if (!maps) return fail(c, IPP_E_INVALID_ARG, "maps is NULL");
  for (int i = 0; i < n; ++i) {
    if (!maps[i].bkg)
      return fail(c, IPP_E_INVALID_ARG, "maps[f].bkg is required");
    P.fd[i].bkg = maps[i].bkg;
  }
  if (src->capacity == 0) return IPP_OK;
  hipStream_t s = (hipStream_t)stream;
  Work w = make_work(P, c->ws, n);
  ++c->ws_gen;
  if ((st = upload(c, P, w, s)) != IPP_OK) return st;
  return run_aperture(c, w, *p, src, sky_lohi, s);
}

ipp_status ipp_process_batch(void* ctx, const ipp_frame* frames, int32_t n,
                             const ipp_params* p, const ipp_maps* maps,
                             ipp_sources* src, uint32_t* frame_flags,
                             int64_t* diag, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  std::string m = check_sources(src, true);
  if (m.empty()) m = check_sources(src, false);
  if (!m.empty()) return fail(c, IPP_E_INVALID_ARG, m);
  Plan P;
  ipp_status st = prepare(c, frames, n, p, kPlanDetect, &P);
  if (st != IPP_OK) return st;
  if (!maps) return fail(c, IPP_E_INVALID_ARG, "maps is NULL");
  const int write_rms = (p->flags & IPP_F_WRITE_RMS) ? 1 : 0;
  for (int i = 0; i < n; ++i) {
    if (!maps[i].bkg || !maps[i].labels || (write_rms && !maps[i].rms))
      return fail(c, IPP_E_INVALID_ARG,
                  "maps[f].bkg and .labels (and .rms with "
                  "IPP_F_WRITE_RMS) are required");
    P.fd[i].bkg = maps[i].bkg;
    P.fd[i].rms = maps[i].rms;
    P.fd[i].labels = maps[i].labels;
  }
  hipStream_t s = (hipStream_t)stream;
  Work w = make_work(P, c->ws, n);
  if (frame_flags) w.frame_flags = frame_flags;
  if (c->prof || !c->use_graphs || (p->flags & IPP_F_NO_GRAPH)) {  // eager
    ++c->ws_gen;
    if ((st = upload(c, P, w, s)) != IPP_OK) return st;
    return run_batch(c, P, w, *p, src, write_rms, diag, s);
  }
  std::vector<uint8_t> key;
  key_put(key, "batch", 5);
  key_put(key, &n, sizeof(n));
  for (int i = 0; i < n; ++i) {
    key_put(key, &frames[i].h, sizeof(int32_t));
    key_put(key, &frames[i].w, sizeof(int32_t));
  }
  key_put(key, p, sizeof(*p));
  key_put(key, src, sizeof(*src));
  key_put(key, &w, sizeof(w));
  key_put(key, &diag, sizeof(diag));
  const ipp_params pv = *p;
  return run_cached(c, std::move(key), P, w, s, [&](hipStream_t cs) {
    return run_batch(c, P, w, pv, src, write_rms, diag, cs);
  });
}

ipp_status ipp_photometry_backward(void* ctx, const ipp_frame* frames,
                                   int32_t n, const ipp_maps* maps,
                                   const ipp_params* p,
                                   const ipp_sources* src,
                                   const double* sky_lohi,
                                   const double* dL_dflux,
                                   float* const* dL_dpix, double* dL_dxy,
                                   void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (!src || src->capacity < 0 || !src->frame || !src->x || !src->y)
    return fail(c, IPP_E_INVALID_ARG, "sources: frame, x and y are required");
  if (!sky_lohi || !dL_dflux)
    return fail(c, IPP_E_INVALID_ARG, "sky_lohi and dL_dflux are required");
  Plan P;
  ipp_status st = prepare(c, frames, n, p, kPlanFrames, &P);
  if (st != IPP_OK) return st;
  if (!maps) return fail(c, IPP_E_INVALID_ARG, "maps is NULL");
  for (int i = 0; i < n; ++i) {
    if (!maps[i].bkg)
      return fail(c, IPP_E_INVALID_ARG, "maps[f].bkg is required");
    P.fd[i].bkg = maps[i].bkg;
    P.fd[i].dpix = dL_dpix ? dL_dpix[i] : nullptr;
  }
  if (src->capacity == 0) return IPP_OK;
  hipStream_t s = (hipStream_t)stream;
  Work w = make_work(P, c->ws, n);
  ++c->ws_gen;
  if ((st = upload(c, P, w, s)) != IPP_OK) return st;
  return run_aperture_bwd(c, w, *p, *src, sky_lohi, dL_dflux, dL_dxy, s);
}

size_t ipp_refine_workspace_bytes(const ipp_frame* frames, int32_t n,
                                  int64_t rows) {
  if (!check_frames(frames, n).empty() || rows < 0) return 0;
  ipp_params pd;
  ipp_params_default(&pd);
  // the frame descriptors only: every step of a row lives in its wavefront
  return make_plan(frames, n, pd, 1, kPlanFrames).total;
}

ipp_status ipp_refine_centroids(void* ctx, const ipp_frame* frames,
                                int32_t n, const ipp_maps* maps,
                                const ipp_params* p, const ipp_sources* src,
                                double r_c, double eta, int32_t steps,
                                double* x_out, double* y_out, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (!src || src->capacity < 0 || !src->frame || !src->x || !src->y)
    return fail(c, IPP_E_INVALID_ARG, "sources: frame, x and y are required");
  if (!x_out || !y_out)
    return fail(c, IPP_E_INVALID_ARG, "x_out and y_out are required");
  if (!std::isfinite(r_c) || r_c <= 0 || r_c > 16)
    return fail(c, IPP_E_INVALID_ARG, "r_c must be in (0, 16]");
  if (!std::isfinite(eta)) return fail(c, IPP_E_INVALID_ARG,
                                       "eta must be finite");
  if (steps < 0 || steps > 1000)
    return fail(c, IPP_E_INVALID_ARG, "steps must be in [0, 1000]");
  if (p && (p->flags & IPP_F_REFINE_PHOTOMETRY) &&
      (!src->flux_ap || !src->sky || !src->area_ap || !src->area_ann ||
       !src->flags))
    return fail(c, IPP_E_INVALID_ARG,
                "IPP_F_REFINE_PHOTOMETRY: flux_ap, sky, area_ap, area_ann "
                "and flags are required");
  Plan P;
  ipp_status st = prepare(c, frames, n, p, kPlanFrames, &P);
  if (st != IPP_OK) return st;
  if (!maps) return fail(c, IPP_E_INVALID_ARG, "maps is NULL");
  for (int i = 0; i < n; ++i) {
    if (!maps[i].bkg)
      return fail(c, IPP_E_INVALID_ARG, "maps[f].bkg is required");
    P.fd[i].bkg = maps[i].bkg;
  }
  if (P.total > c->ws_bytes)
    return fail(c, IPP_E_WORKSPACE,
                "workspace too small: need " + std::to_string(P.total) +
                    " bytes, have " + std::to_string(c->ws_bytes));
  if (src->capacity == 0) return IPP_OK;
  hipStream_t s = (hipStream_t)stream;
  Work w = make_work(P, c->ws, n);
  if (c->prof || !c->use_graphs || (p->flags & IPP_F_NO_GRAPH)) {  // eager
    ++c->ws_gen;
    if ((st = upload(c, P, w, s)) != IPP_OK) return st;
    return run_refine(c, w, *p, *src, r_c, eta, steps, x_out, y_out, s);
  }
  std::vector<uint8_t> key;
  key_put(key, "refine", 6);
  key_put(key, &n, sizeof(n));
  for (int i = 0; i < n; ++i) {
    key_put(key, &frames[i].h, sizeof(int32_t));
    key_put(key, &frames[i].w, sizeof(int32_t));
  }
  key_put(key, p, sizeof(*p));
  key_put(key, src, sizeof(*src));
  key_put(key, &w, sizeof(w));
  key_put(key, &r_c, sizeof(r_c));
  key_put(key, &eta, sizeof(eta));
  key_put(key, &steps, sizeof(steps));
  key_put(key, &x_out, sizeof(x_out));
  key_put(key, &y_out, sizeof(y_out));
  const ipp_params pv = *p;
  const ipp_sources sv = *src;
  return run_cached(c, std::move(key), P, w, s, [&](hipStream_t cs) {
    return run_refine(c, w, pv, sv, r_c, eta, steps, x_out, y_out, cs);
  });
}

ipp_status ipp_asinh(void* ctx, const float* v, float* y, int64_t n,
                     double a, double b, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (n < 0 || (n > 0 && (!v || !y)))
    return fail(c, IPP_E_INVALID_ARG, "v and y are required, n >= 0");
  if (!std::isfinite(a) || a <= 0 || !std::isfinite(b))
    return fail(c, IPP_E_INVALID_ARG, "need a > 0 and finite b");
  if (n == 0) return IPP_OK;
  hipStream_t s = (hipStream_t)stream;
  IPP_LAUNCH(c, s, "k_asinh_fwd",
             hipLaunchKernelGGL(k_asinh_fwd, dim3(grid_for(n, 4 * kBlock,
                                                           8192)),
                                dim3(kBlock), 0, s, v, y, n,
                                (float)(1.0 / a), (float)b,
                                (const double*)nullptr));
  return IPP_OK;
}

ipp_status ipp_asinh_backward(void* ctx, const float* v, const float* dy,
                              float* dv, double* dL_dab, int64_t n, double a,
                              double b, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (n < 0 || (n > 0 && (!v || !dy)))
    return fail(c, IPP_E_INVALID_ARG, "v and dy are required, n >= 0");
  if (!std::isfinite(a) || a <= 0 || !std::isfinite(b))
    return fail(c, IPP_E_INVALID_ARG, "need a > 0 and finite b");
  const int grid = grid_for(n, 4 * kBlock, kAsinhMaxBlocks);
  if (dL_dab && c->ws_bytes < (size_t)grid * 16)
    return fail(c, IPP_E_WORKSPACE, "workspace too small for the partials");
  hipStream_t s = (hipStream_t)stream;
  double* part = dL_dab ? (double*)c->ws : nullptr;
  ++c->ws_gen;
  IPP_LAUNCH(c, s, "k_asinh_bwd",
             hipLaunchKernelGGL(k_asinh_bwd, dim3(grid), dim3(kBlock), 0, s,
                                v, dy, dv, n, a, b, (const double*)nullptr,
                                part));
  if (dL_dab)
    IPP_LAUNCH(c, s, "k_asinh_bwd_final",
               hipLaunchKernelGGL(k_asinh_bwd_final, dim3(1), dim3(kBlock), 0,
                                  s, part, grid, dL_dab));
  return IPP_OK;
}

ipp_status ipp_asinh_backward_noalloc(void* ctx, const float* v,
                                      const float* dy, float* dv,
                                      double* dL_dab, int64_t n, double a,
                                      double b, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (n < 0 || (n > 0 && (!v || !dy)))
    return fail(c, IPP_E_INVALID_ARG, "v and dy are required, n >= 0");
  if (!std::isfinite(a) || a <= 0 || !std::isfinite(b))
    return fail(c, IPP_E_INVALID_ARG, "need a > 0 and finite b");
  // grid-stride workgroups, at most kAsinhMaxBlocks of them: their
  // partials always fit the static scratch, whatever n is
  const int grid = grid_for(n, 4 * kBlock, kAsinhMaxBlocks);
  if (grid > kAsinhMaxBlocks)
    return fail(c, IPP_E_CAPACITY,
                "more block partials than the static scratch holds (" +
                    std::to_string(2 * kAsinhMaxBlocks) + " doubles)");
  double* part = nullptr;
  if (dL_dab) {
    const hipError_t e = asinh_scratch(c->device, &part);
    if (e != hipSuccess)
      return fail(c, IPP_E_DEVICE, std::string("scratch lookup: ") +
                                       hipGetErrorString(e));
  }
  hipStream_t s = (hipStream_t)stream;
  IPP_LAUNCH(c, s, "k_asinh_bwd",
             hipLaunchKernelGGL(k_asinh_bwd, dim3(grid), dim3(kBlock), 0, s,
                                v, dy, dv, n, a, b, (const double*)nullptr,
                                part));
  if (dL_dab)
    IPP_LAUNCH(c, s, "k_asinh_bwd_final",
               hipLaunchKernelGGL(k_asinh_bwd_final, dim3(1), dim3(kBlock), 0,
                                  s, part, grid, dL_dab));
  return IPP_OK;
}

ipp_status ipp_asinh_dev(void* ctx, const float* v, float* y, int64_t n,
                         const double* ab, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (n < 0 || (n > 0 && (!v || !y)))
    return fail(c, IPP_E_INVALID_ARG, "v and y are required, n >= 0");
  if (!ab) return fail(c, IPP_E_INVALID_ARG, "ab is NULL");
  if (n == 0) return IPP_OK;
  hipStream_t s = (hipStream_t)stream;
  IPP_LAUNCH(c, s, "k_asinh_fwd",
             hipLaunchKernelGGL(k_asinh_fwd, dim3(grid_for(n, 4 * kBlock,
                                                           8192)),
                                dim3(kBlock), 0, s, v, y, n, 0.0f, 0.0f,
                                ab));
  return IPP_OK;
}

ipp_status ipp_asinh_backward_dev(void* ctx, const float* v, const float* dy,
                                  float* dv, double* dL_dab, int64_t n,
                                  const double* ab, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (n < 0 || (n > 0 && (!v || !dy)))
    return fail(c, IPP_E_INVALID_ARG, "v and dy are required, n >= 0");
  if (!ab) return fail(c, IPP_E_INVALID_ARG, "ab is NULL");
  const int grid = grid_for(n, 4 * kBlock, kAsinhMaxBlocks);
  if (dL_dab && c->ws_bytes < (size_t)grid * 16)
    return fail(c, IPP_E_WORKSPACE, "workspace too small for the partials");
  hipStream_t s = (hipStream_t)stream;
  double* part = dL_dab ? (double*)c->ws : nullptr;
  ++c->ws_gen;
  IPP_LAUNCH(c, s, "k_asinh_bwd",
             hipLaunchKernelGGL(k_asinh_bwd, dim3(grid), dim3(kBlock), 0, s,
                                v, dy, dv, n, 0.0, 0.0, ab, part));
  if (dL_dab)
    IPP_LAUNCH(c, s, "k_asinh_bwd_final",
               hipLaunchKernelGGL(k_asinh_bwd_final, dim3(1), dim3(kBlock), 0,
                                  s, part, grid, dL_dab));
  return IPP_OK;
}

size_t ipp_gray_workspace_bytes(int32_t n, int32_t nbins) {
  if (n < 1 || n > 65536 || nbins < 0 || nbins == 1 || nbins > kMaxBins)
    return 0;
  GrayPlan G;
  return gray_layout(n, nbins, &G);
}

ipp_status ipp_zscale(void* ctx, const ipp_frame* frames, int32_t n,
                      int32_t nsamples, double contrast, double* z1z2,
                      double* info, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (nsamples < 1 || nsamples > IPP_ZSCALE_MAX_SAMPLES)
    return fail(c, IPP_E_INVALID_ARG, "nsamples must be in [1, 1000]");
  if (!std::isfinite(contrast) || contrast < 0)
    return fail(c, IPP_E_INVALID_ARG, "contrast must be finite and >= 0");
  if (!z1z2) return fail(c, IPP_E_INVALID_ARG, "z1z2 is NULL");
  hipStream_t s = (hipStream_t)stream;
  GrayPlan G;
  ipp_status st = gray_prepare(c, frames, n, nsamples, 0, nullptr, false,
                               &G, s);
  if (st != IPP_OK) return st;
  const GrayFrame* fr = (const GrayFrame*)((char*)c->ws + G.o_frames);
  IPP_LAUNCH(c, s, "k_zscale",
             hipLaunchKernelGGL(k_zscale, dim3(n), dim3(kBlock), 0, s, fr,
                                contrast, 2.5, 5, z1z2, info));
  return IPP_OK;
}

ipp_status ipp_gray_map(void* ctx, const ipp_frame* frames, int32_t n,
                        int32_t kind, double a, const double* lohi,
                        float* const* out, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (kind < IPP_MAP_LINEAR || kind > IPP_MAP_POWER)
    return fail(c, IPP_E_INVALID_ARG, "unknown map kind");
  if (kind != IPP_MAP_LINEAR &&
      (!std::isfinite(a) || a <= 0 || (kind == IPP_MAP_EXP && a == 1.0)))
    return fail(c, IPP_E_INVALID_ARG,
                "the map needs a finite a > 0 (and a != 1 for exp)");
  if (!lohi) return fail(c, IPP_E_INVALID_ARG, "lohi is NULL");
  hipStream_t s = (hipStream_t)stream;
  GrayPlan G;
  ipp_status st = gray_prepare(c, frames, n, 0, 0, out, true, &G, s);
  if (st != IPP_OK) return st;
  float cc = 1.0f, lna = 0.0f;
  if (kind == IPP_MAP_LOG) cc = (float)(1.0 / std::log1p(a));
  if (kind == IPP_MAP_EXP) {
    cc = (float)(1.0 / (a - 1.0));
    lna = (float)std::log(a);
  }
  const GrayFrame* fr = (const GrayFrame*)((char*)c->ws + G.o_frames);
  IPP_LAUNCH(c, s, "k_gray_map",
             hipLaunchKernelGGL(k_gray_map, dim3(grid_for(G.rows, 1, 4096)),
                                dim3(kBlock), 0, s, fr, n, G.rows, kind,
                                (float)a, cc, lna, lohi));
  return IPP_OK;
}

ipp_status ipp_equalize(void* ctx, const ipp_frame* frames, int32_t n,
                        int32_t nbins, float* const* out, uint32_t* counts,
                        void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (nbins < 2 || nbins > IPP_EQ_MAX_BINS)
    return fail(c, IPP_E_INVALID_ARG, "nbins must be in [2, 4096]");
  hipStream_t s = (hipStream_t)stream;
  GrayPlan G;
  ipp_status st = gray_prepare(c, frames, n, 0, nbins, out, true, &G, s);
  if (st != IPP_OK) return st;
  char* b = (char*)c->ws;
  const GrayFrame* fr = (const GrayFrame*)(b + G.o_frames);
  uint32_t* mm = (uint32_t*)(b + G.o_mm);
  uint32_t* cnt = counts ? counts : (uint32_t*)(b + G.o_counts);
  double* cdf = (double*)(b + G.o_cdf);
  const int64_t nc = (int64_t)n * nbins;
  // fill kernels, not memsets: the call may be captured into a graph
  IPP_LAUNCH(c, s, "k_fill_i32",
             hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, s,
                                (int32_t*)mm, (int64_t)n, (int32_t)-1));
  IPP_LAUNCH(c, s, "k_fill_i32",
             hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, s,
                                (int32_t*)mm + n, (int64_t)n, 0));
  IPP_LAUNCH(c, s, "k_fill_i32",
             hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nc, kBlock, 4096)),
                                dim3(kBlock), 0, s, (int32_t*)cnt, nc, 0));
  const int gr = grid_for(G.rows, 16, 4096);
  IPP_LAUNCH(c, s, "k_eq_minmax",
             hipLaunchKernelGGL(k_eq_minmax, dim3(gr), dim3(kBlock), 0, s, fr,
                                n, G.rows, mm));
  IPP_LAUNCH(c, s, "k_eq_hist",
             hipLaunchKernelGGL(k_eq_hist, dim3(gr), dim3(kBlock), 0, s, fr,
                                n, G.rows, nbins, mm, cnt));
  IPP_LAUNCH(c, s, "k_eq_cdf",
             hipLaunchKernelGGL(k_eq_cdf, dim3(n), dim3(kBlock), 0, s, cnt,
                                nbins, cdf));
  IPP_LAUNCH(c, s, "k_eq_map",
             hipLaunchKernelGGL(k_eq_map, dim3(grid_for(G.rows, 32, 2048)),
                                dim3(kBlock), 0, s, fr, n, G.rows, nbins, mm,
                                cdf));
  return IPP_OK;
}

void ipp_deblend_params_default(ipp_deblend_params* d) {
  if (!d) return;
  d->nthresh = 32;
  d->clean = 1;
  d->mincont = 0.005;
  d->clean_param = 1.0;
}

size_t ipp_deblend_workspace_bytes(const ipp_frame* frames, int32_t n,
                                   int64_t cand_capacity,
                                   int64_t scratch_bytes) {
  if (!check_frames(frames, n).empty() || cand_capacity < 0 ||
      scratch_bytes < 0)
    return 0;
  ipp_params pd;
  ipp_params_default(&pd);
  const Plan P = make_plan(frames, n, pd, 1, kPlanFrames);
  return deblend_layout(P.total, n, cand_capacity).o_pool +
         align_up((size_t)scratch_bytes);
}

ipp_status ipp_deblend(void* ctx, const ipp_frame* frames, int32_t n,
                       const ipp_params* p, const ipp_deblend_params* dp,
                       const ipp_maps* maps, const ipp_sources* cand,
                       int32_t* const* objects, ipp_sources* obj,
                       int32_t* parent, int64_t* diag, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (!dp) return fail(c, IPP_E_INVALID_ARG, "deblend params are NULL");
  if (dp->nthresh < 2 || dp->nthresh > db::kMaxLevels ||
      (dp->nthresh & (dp->nthresh - 1)))
    return fail(c, IPP_E_INVALID_ARG,
                "nthresh must be a power of two in [2, 64]");
  if (!std::isfinite(dp->mincont) || dp->mincont < 0 ||
      !std::isfinite(dp->clean_param) || dp->clean_param < 0)
    return fail(c, IPP_E_INVALID_ARG,
                "mincont and clean_param must be finite and >= 0");
  if (!cand || cand->capacity < 0 || !cand->frame || !cand->label ||
      !cand->npix || !cand->xmin || !cand->xmax || !cand->ymin ||
      !cand->ymax || !cand->peak || !cand->peak_x || !cand->peak_y ||
      !cand->frame_offsets)
    return fail(c, IPP_E_INVALID_ARG,
                "candidates: frame, label, npix, bounding box, peak, "
                "peak_x, peak_y and frame_offsets are required");
  std::string m = check_sources(obj, true);
  if (!m.empty()) return fail(c, IPP_E_INVALID_ARG, "objects: " + m);
  if (!parent) return fail(c, IPP_E_INVALID_ARG, "parent is NULL");
  if (!objects) return fail(c, IPP_E_INVALID_ARG, "objects is NULL");
  Plan P;
  ipp_status st = prepare(c, frames, n, p, kPlanFrames, &P);
  if (st != IPP_OK) return st;
  if (!maps) return fail(c, IPP_E_INVALID_ARG, "maps is NULL");
  for (int i = 0; i < n; ++i) {
    if (!maps[i].bkg || !maps[i].rms || !maps[i].labels || !objects[i])
      return fail(c, IPP_E_INVALID_ARG,
                  "maps[f].bkg, .rms, .labels and objects[f] are required");
    P.fd[i].bkg = maps[i].bkg;
    P.fd[i].rms = maps[i].rms;
    P.fd[i].labels = maps[i].labels;
    P.fd[i].objects = objects[i];
  }
  const int64_t cap = cand->capacity;
  const DeblendWs D = deblend_layout(P.total, n, cap);
  if (D.o_pool > c->ws_bytes)
    return fail(c, IPP_E_WORKSPACE,
                "workspace too small: need at least " +
                    std::to_string(D.o_pool) + " bytes, have " +
                    std::to_string(c->ws_bytes));
  const int64_t pool_units = (int64_t)((c->ws_bytes - D.o_pool) / 256);
  hipStream_t s = (hipStream_t)stream;
  Work w = make_work(P, c->ws, n);
  ++c->ws_gen;
  if ((st = upload(c, P, w, s)) != IPP_OK) return st;
  std::vector<FrameDev> fd2(P.fd);
  for (auto& d : fd2) d.labels = d.objects;
  char* b = (char*)c->ws;
  hipError_t e = hipMemcpyAsync(b + D.o_fd2, fd2.data(),
                                sizeof(FrameDev) * fd2.size(),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess)
    return fail(c, IPP_E_DEVICE, std::string("descriptor upload failed: ") +
                                     hipGetErrorString(e));
  Work w2 = w;
  w2.frames = (FrameDev*)(b + D.o_fd2);
  int64_t* need = (int64_t*)(b + D.o_need);
  int64_t* off = (int64_t*)(b + D.o_off);
  int64_t* cnt = (int64_t*)(b + D.o_cnt);
  int64_t* ooff = (int64_t*)(b + D.o_ooff);
  int64_t* blk = (int64_t*)(b + D.o_blk);
  int64_t* tot = (int64_t*)(b + D.o_tot);
  int32_t* big = (int32_t*)(b + D.o_big);
  char* pool = b + D.o_pool;
  const int64_t rows = cap + 1;
  IPP_LAUNCH(c, s, "k_fill_i64",
             hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, s,
                                w.counters, (int64_t)4, (int64_t)0));
  // tot[2], tot[3]: the two kernels' queue counters; tot[4], tot[5]: the
  // workgroup kernel's list lengths (boxes above kDbBigBox from the front
  // of `big`, the other large boxes from its back)
  IPP_LAUNCH(c, s, "k_fill_i64",
             hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, s, tot + 2,
                                (int64_t)4, (int64_t)0));
  IPP_LAUNCH(c, s, "k_db_need",
             hipLaunchKernelGGL(k_db_need,
                                dim3(grid_for(rows, kBlock, 16384)),
                                dim3(kBlock), 0, s, *cand, need, big,
                                tot + 4));
  if ((st = scan64(c, need, blk, D.nblk, off, rows, tot, s)) != IPP_OK)
    return st;
  // persistent workgroups (as many as fit the device at once) that take
  // candidates from a counter
  IPP_LAUNCH(c, s, "k_db_small",
             hipLaunchKernelGGL(k_db_small,
                                dim3(grid_for(rows, kWaves,
                                              c->n_cu * kDbSmallPerCu)),
                                dim3(kBlock), 0, s, w, *cand, off, tot, pool,
                                pool_units, p->det_nsigma, p->connectivity,
                                dp->nthresh, dp->clean, dp->mincont,
                                dp->clean_param, cnt, tot + 2));
  IPP_LAUNCH(c, s, "k_db_large",
             hipLaunchKernelGGL(k_db_large,
                                dim3(grid_for(rows, 1,
                                              c->n_cu * kDbLargePerCu)),
                                dim3(kBlock), 0, s, w, *cand, off, tot, pool,
                                pool_units, p->det_nsigma, p->connectivity,
                                dp->nthresh, dp->clean, dp->mincont,
                                dp->clean_param, cnt, tot + 3, big,
                                tot + 4));
  if ((st = scan64(c, cnt, blk, D.nblk, ooff, rows, tot + 1, s)) != IPP_OK)
    return st;
  int64_t maxpix = 1;
  for (int i = 0; i < n; ++i)
    maxpix = std::max<int64_t>(maxpix, (int64_t)frames[i].h * frames[i].w);
  IPP_LAUNCH(c, s, "k_db_zero",
             hipLaunchKernelGGL(k_db_zero,
                                dim3(grid_for(maxpix, kBlock, 1024),
                                     std::min(n, 65535)),
                                dim3(kBlock), 0, s, w));
  IPP_LAUNCH(c, s, "k_db_write",
             hipLaunchKernelGGL(k_db_write,
                                dim3(grid_for(rows, kWaves, 16384)),
                                dim3(kBlock), 0, s, w, *cand,
                                off, tot, pool, pool_units, cnt, ooff, *obj,
                                parent));
  IPP_LAUNCH(c, s, "k_db_offsets",
             hipLaunchKernelGGL(k_db_offsets,
                                dim3(grid_for((int64_t)n + 1, kBlock, 4096)),
                                dim3(kBlock), 0, s, w, *cand, ooff, tot + 1,
                                *obj));
  IPP_LAUNCH(c, s, "k_source_stats",
             hipLaunchKernelGGL(k_source_stats,
                                dim3(grid_for(obj->capacity, 4, 4096)),
                                dim3(kBlock), 0, s, w2, *obj));
  IPP_LAUNCH(c, s, "k_db_flags",
             hipLaunchKernelGGL(k_db_flags,
                                dim3(grid_for(obj->capacity, kBlock, 4096)),
                                dim3(kBlock), 0, s, *cand, cnt, tot + 1,
                                *obj, parent));
  if (diag)
    IPP_LAUNCH(c, s, "k_db_diag",
               hipLaunchKernelGGL(k_db_diag, dim3(1), dim3(64), 0, s, tot,
                                  pool_units, w.counters, diag));
  return IPP_OK;
}

void ipp_auto_params_default(ipp_auto_params* a) {
  if (!a) return;
  a->kron_factor = 2.5;
  a->kron_min = 3.5;
  a->search = 6.0;
}

ipp_status ipp_photometry_auto(void* ctx, const ipp_frame* frames, int32_t n,
                               const ipp_maps* maps, const ipp_sources* src,
                               const double* mom, const ipp_auto_params* ap,
                               double* kron, double* flux, double* area,
                               uint32_t* flags, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (!src || src->capacity < 0 || !src->frame || !src->x || !src->y)
    return fail(c, IPP_E_INVALID_ARG, "sources: frame, x and y are required");
  if (!mom || !kron || !flux || !area || !flags)
    return fail(c, IPP_E_INVALID_ARG,
                "mom, kron, flux, area and flags are required");
  ipp_auto_params a;
  ipp_auto_params_default(&a);
  if (ap) a = *ap;
  if (!std::isfinite(a.kron_factor) || a.kron_factor <= 0 ||
      !std::isfinite(a.kron_min) || a.kron_min <= 0 ||
      !std::isfinite(a.search) || a.search <= 0 || a.search > 64)
    return fail(c, IPP_E_INVALID_ARG,
                "kron_factor and kron_min must be > 0, search in (0, 64]");
  ipp_params pd;
  ipp_params_default(&pd);
  Plan P;
  ipp_status st = prepare(c, frames, n, &pd, kPlanFrames, &P);
  if (st != IPP_OK) return st;
  if (!maps) return fail(c, IPP_E_INVALID_ARG, "maps is NULL");
  for (int i = 0; i < n; ++i) {
    if (!maps[i].bkg)
      return fail(c, IPP_E_INVALID_ARG, "maps[f].bkg is required");
    P.fd[i].bkg = maps[i].bkg;
  }
  if (src->capacity == 0) return IPP_OK;
  hipStream_t s = (hipStream_t)stream;
  Work w = make_work(P, c->ws, n);
  ++c->ws_gen;
  if ((st = upload(c, P, w, s)) != IPP_OK) return st;
  IPP_LAUNCH(c, s, "k_kron",
             hipLaunchKernelGGL(k_kron,
                                dim3(grid_for(src->capacity, kWaves, 16384)),
                                dim3(kBlock), 0, s, w, *src, mom,
                                a.kron_factor, a.kron_min, a.search, kron,
                                flux, area, flags));
  IPP_LAUNCH(c, s, "k_kron_big",
             hipLaunchKernelGGL(k_kron_big,
                                dim3(grid_for(src->capacity, kBigThreads,
                                              4 * c->n_cu)),
                                dim3(kBigThreads), 0, s, w, *src, mom,
                                a.kron_factor, a.kron_min, a.search, kron,
                                flux, area, flags));
  return IPP_OK;
}

void ipp_subtract_params_default(ipp_subtract_params* sp) {
  if (!sp) return;
  std::memset(sp, 0, sizeof(*sp));
  sp->half_width = 10;
  sp->stamp = 21;
  sp->n_gauss = 3;
  sp->spatial_order = 2;
  sp->bkg_order = 1;
  const int ord[3] = {6, 4, 2};
  const double sig[3] = {0.7, 1.5, 3.0};
  for (int g = 0; g < 3; ++g) {
    sp->order[g] = ord[g];
    sp->sigma[g] = sig[g];
  }
}

namespace {
std::string check_subtract(const ipp_subtract_params* sp) {
  if (!sp) return "subtract params are NULL";
  if (sp->half_width < 1 || sp->half_width > kSubMaxHw)
    return "half_width must be in [1, 15]";
  if (sp->stamp < 1 || sp->stamp > kSubMaxStamp)
    return "stamp must be in [1, 32]";
  if (sp->n_gauss < 1 || sp->n_gauss > kSubMaxGauss)
    return "n_gauss must be in [1, 4]";
  if (sp->spatial_order < 0 || sp->spatial_order > 4 || sp->bkg_order < 0 ||
      sp->bkg_order > 4)
    return "spatial_order and bkg_order must be in [0, 4]";
  for (int g = 0; g < sp->n_gauss; ++g) {
    if (sp->order[g] < 0 || sp->order[g] > kSubMaxOrder)
      return "orders must be in [0, 7]";
    if (!std::isfinite(sp->sigma[g]) || sp->sigma[g] <= 0)
      return "sigmas must be finite and > 0";
  }
  return "";
}
int64_t sub_nbasis(const ipp_subtract_params* sp) {
  int64_t nb = 0;
  for (int g = 0; g < sp->n_gauss; ++g)
    nb += (int64_t)(sp->order[g] + 1) * (sp->order[g] + 2) / 2;
  return nb;
}
}  // namespace

int64_t ipp_subtract_coef_count(const ipp_subtract_params* sp) {
  if (!check_subtract(sp).empty()) return 0;
  const int64_t ps = (sp->spatial_order + 1) * (sp->spatial_order + 2) / 2;
  const int64_t pb = (sp->bkg_order + 1) * (sp->bkg_order + 2) / 2;
  return sub_nbasis(sp) * ps + pb;
}

ipp_status ipp_subtract(void* ctx, const ipp_frame* sci,
                        const ipp_frame* tmpl, int32_t n,
                        const ipp_subtract_params* sp, const double* coef,
                        float* const* diff, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  std::string m = check_subtract(sp);
  if (!m.empty()) return fail(c, IPP_E_INVALID_ARG, m);
  m = check_frames(sci, n);
  if (m.empty()) m = check_frames(tmpl, n);
  if (!m.empty()) return fail(c, IPP_E_INVALID_ARG, m);
  if (!coef || !diff) return fail(c, IPP_E_INVALID_ARG,
                                  "coef and diff are required");
  const int64_t per = ipp_subtract_coef_count(sp);
  std::vector<SubFrame> fr(n);
  int64_t stamps = 0;
  for (int i = 0; i < n; ++i) {
    if (tmpl[i].h != sci[i].h || tmpl[i].w != sci[i].w)
      return fail(c, IPP_E_INVALID_ARG,
                  "template " + std::to_string(i) +
                      " differs in shape from its frame");
    if (!diff[i])
      return fail(c, IPP_E_INVALID_ARG,
                  "diff[" + std::to_string(i) + "] is NULL");
    SubFrame& d = fr[i];
    d.I = sci[i].pix;
    d.R = tmpl[i].pix;
    d.pitchI = sci[i].pitch;
    d.pitchR = tmpl[i].pitch;
    d.h = sci[i].h;
    d.w = sci[i].w;
    d.nsy = (d.h + sp->stamp - 1) / sp->stamp;
    d.nsx = (d.w + sp->stamp - 1) / sp->stamp;
    d.stamp0 = stamps;
    stamps += (int64_t)d.nsy * d.nsx;
    d.D = diff[i];
    d.coef = coef + (int64_t)i * per;
  }
  const size_t need = sizeof(SubFrame) * (size_t)n;
  if (need > c->ws_bytes)
    return fail(c, IPP_E_WORKSPACE,
                "workspace too small: need " + std::to_string(need) +
                    " bytes, have " + std::to_string(c->ws_bytes));
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSetDevice(c->device);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws, fr.data(), need, hipMemcpyHostToDevice, s);
  if (e != hipSuccess)
    return fail(c, IPP_E_DEVICE, std::string("descriptor upload failed: ") +
                                     hipGetErrorString(e));
  ++c->ws_gen;
  SubBasis bs;
  std::memset(&bs, 0, sizeof(bs));
  bs.hw = sp->half_width;
  bs.stamp = sp->stamp;
  bs.ngauss = sp->n_gauss;
  bs.spatial_order = sp->spatial_order;
  bs.bkg_order = sp->bkg_order;
  bs.nbasis = (int32_t)sub_nbasis(sp);
  for (int g = 0; g < sp->n_gauss; ++g) {
    bs.order[g] = sp->order[g];
    bs.sigma[g] = sp->sigma[g];
  }
  const dim3 g((unsigned)std::min<int64_t>(stamps, 1 << 20));
  const dim3 b(sub_threads(sp->stamp));
  const size_t lds = sub_lds_bytes(sp->stamp, sp->half_width);
  const SubFrame* fd = (const SubFrame*)c->ws;
  switch (sp->half_width) {
#define IPP_SUB_CASE(H)                                                   \
  case H:                                                                 \
    IPP_LAUNCH(c, s, "k_subtract",                                        \
               hipLaunchKernelGGL((k_subtract_t<H>), g, b, lds, s, fd, n, \
                                  bs, stamps));                           \
    break;
    IPP_SUB_CASE(1) IPP_SUB_CASE(2) IPP_SUB_CASE(3) IPP_SUB_CASE(4)
    IPP_SUB_CASE(5) IPP_SUB_CASE(6) IPP_SUB_CASE(7) IPP_SUB_CASE(8)
    IPP_SUB_CASE(9) IPP_SUB_CASE(10) IPP_SUB_CASE(11) IPP_SUB_CASE(12)
    IPP_SUB_CASE(13) IPP_SUB_CASE(14) IPP_SUB_CASE(15)
#undef IPP_SUB_CASE
    default:
      return fail(c, IPP_E_INVALID_ARG, "half_width must be in [1, 15]");
  }
  return IPP_OK;
}

ipp_status ipp_source_moments(void* ctx, const ipp_frame* frames, int32_t n,
                              const ipp_maps* maps, const ipp_sources* src,
                              double* mom, void* stream) {
  IppCtx* c = (IppCtx*)ctx;
  if (!c) return IPP_E_INVALID_ARG;
  if (!src || src->capacity < 0 || !src->frame || !src->label ||
      !src->xmin || !src->xmax || !src->ymin || !src->ymax)
    return fail(c, IPP_E_INVALID_ARG,
                "sources: frame, label and the bounding box are required");
  if (!mom) return fail(c, IPP_E_INVALID_ARG, "mom is NULL");
  ipp_params pd;
  ipp_params_default(&pd);
  Plan P;
  ipp_status st = prepare(c, frames, n, &pd, kPlanFrames, &P);
  if (st != IPP_OK) return st;
  if (!maps) return fail(c, IPP_E_INVALID_ARG, "maps is NULL");
  for (int i = 0; i < n; ++i) {
    if (!maps[i].bkg || !maps[i].labels)
      return fail(c, IPP_E_INVALID_ARG,
                  "maps[f].bkg and maps[f].labels are required");
    P.fd[i].bkg = maps[i].bkg;
    P.fd[i].labels = maps[i].labels;
  }
  if (src->capacity == 0) return IPP_OK;
  hipStream_t s = (hipStream_t)stream;
  Work w = make_work(P, c->ws, n);
  ++c->ws_gen;
  if ((st = upload(c, P, w, s)) != IPP_OK) return st;
  IPP_LAUNCH(c, s, "k_source_moments",
             hipLaunchKernelGGL(k_source_moments,
                                dim3(grid_for(src->capacity, kWaves, 16384)),
                                dim3(kBlock), 0, s, w, *src, mom));
  return IPP_OK;
}

}  // extern "C"
