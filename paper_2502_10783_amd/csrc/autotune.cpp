// Autotuner of the batched pipeline: picks the mesh size and the detection
// tile shape that run a given batch fastest on this device, and remembers
// the choice in a small JSON cache keyed by device, batch shape mix and the
// remaining parameters.  Built on the public ABI only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ipp.h"

namespace {

uint64_t fnv1a(const void* d, size_t n) {
  const uint8_t* b = (const uint8_t*)d;
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

std::string make_key(int device, const ipp_frame* f, int32_t n,
                     const ipp_params& p, uint32_t what) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, device) == hipSuccess)
    arch = prop.gcnArchName;
  for (auto& ch : arch)
    if (ch == '"' || ch == '\\' || ch == ':') ch = '_';
  std::map<std::pair<int, int>, int> shapes;
  for (int i = 0; i < n; ++i) shapes[{f[i].h, f[i].w}]++;
  ipp_params q = p;
  if (what & IPP_TUNE_MESH) q.mesh_h = q.mesh_w = 0;
  if (what & IPP_TUNE_TILE) q.tile_h = q.tile_w = 0;
  std::ostringstream k;
  k << arch << "|";
  for (auto& s : shapes)
    k << s.first.first << "x" << s.first.second << "*" << s.second << ",";
  char hx[32];
  std::snprintf(hx, sizeof(hx), "|%016llx|%u",
                (unsigned long long)fnv1a(&q, sizeof(q)), what);
  k << hx;
  return k.str();
}

// Cache file: a JSON object with one entry per line,
//   "<key>": {"mesh_h": M, "mesh_w": M, "tile_h": T, "tile_w": T, "ms": X}
bool cache_lookup(const char* path, const std::string& key, ipp_params* p,
                  double* ms) {
  std::ifstream in(path);
  if (!in) return false;
  std::string line, tag = "\"" + key + "\":";
  while (std::getline(in, line)) {
    const size_t at = line.find(tag);
    if (at == std::string::npos) continue;
    int mh, mw, th, tw;
    double t;
    const char* b = line.c_str() + at + tag.size();
    if (std::sscanf(b,
                    " {\"mesh_h\": %d, \"mesh_w\": %d, \"tile_h\": %d, "
                    "\"tile_w\": %d, \"ms\": %lf}",
                    &mh, &mw, &th, &tw, &t) == 5) {
      p->mesh_h = mh;
      p->mesh_w = mw;
      p->tile_h = th;
      p->tile_w = tw;
      if (ms) *ms = t;
      return true;
    }
  }
  return false;
}

void cache_store(const char* path, const std::string& key,
                 const ipp_params& p, double ms) {
  std::vector<std::string> keep;
  {
    std::ifstream in(path);
    std::string line, tag = "\"" + key + "\":";
    while (in && std::getline(in, line)) {
      if (line.find("\": {\"mesh_h\"") == std::string::npos) continue;
      if (line.find(tag) != std::string::npos) continue;
      while (!line.empty() && (line.back() == ',' || line.back() == ' '))
        line.pop_back();
      keep.push_back(line);
    }
  }
  char buf[512];
  std::snprintf(buf, sizeof(buf),
                "  \"%s\": {\"mesh_h\": %d, \"mesh_w\": %d, \"tile_h\": %d, "
                "\"tile_w\": %d, \"ms\": %.6f}",
                key.c_str(), p.mesh_h, p.mesh_w, p.tile_h, p.tile_w, ms);
  keep.push_back(buf);
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream out(tmp);
    out << "{\n";
    for (size_t i = 0; i < keep.size(); ++i)
      out << keep[i] << (i + 1 < keep.size() ? ",\n" : "\n");
    out << "}\n";
  }
  std::rename(tmp.c_str(), path);
}

struct Scratch {
  std::vector<void*> blocks;
  ~Scratch() {
    for (void* b : blocks) hipFree(b);
  }
  void* get(size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 8) != hipSuccess) return nullptr;
    blocks.push_back(p);
    return p;
  }
};

}  // namespace

extern "C" ipp_status ipp_autotune(void* ctx, const ipp_frame* frames,
                                   int32_t n, ipp_params* p, uint32_t what,
                                   const char* cache_path, double* best_ms,
                                   void* stream) {
  if (!ctx || !frames || n < 1 || !p) return IPP_E_INVALID_ARG;
  if (ipp_params_validate(p) != IPP_OK) return IPP_E_INVALID_ARG;
  if (ipp_workspace_bytes(frames, n, p, 0) == 0) return IPP_E_INVALID_ARG;
  int device = 0;
  hipGetDevice(&device);
  const std::string key = make_key(device, frames, n, *p, what);
  if (cache_path && cache_lookup(cache_path, key, p, best_ms))
    return IPP_OK;

  std::vector<int> meshes = {p->mesh_h};
  if (what & IPP_TUNE_MESH) meshes = {32, 64, 128};
  std::vector<std::pair<int, int>> tiles = {{p->tile_h, p->tile_w}};
  if (what & IPP_TUNE_TILE) tiles = {{64, 64}, {32, 128}, {128, 32}};

  // outputs for the trial runs
  Scratch S;
  int64_t npix = 0;
  for (int i = 0; i < n; ++i) npix += (int64_t)frames[i].h * frames[i].w;
  std::vector<ipp_maps> maps(n);
  float* bkg = (float*)S.get(sizeof(float) * npix);
  int32_t* lab = (int32_t*)S.get(sizeof(int32_t) * npix);
  if (!bkg || !lab) return IPP_E_DEVICE;
  int64_t off = 0;
  for (int i = 0; i < n; ++i) {
    maps[i].bkg = bkg + off;
    maps[i].rms = nullptr;
    maps[i].labels = lab + off;
    off += (int64_t)frames[i].h * frames[i].w;
  }
  ipp_sources src;
  std::memset(&src, 0, sizeof(src));
  src.capacity = npix / 64 + 1024;
  const size_t cap = (size_t)src.capacity;
  src.n_total = (int64_t*)S.get(8);
  src.frame_offsets = (int64_t*)S.get(8 * (n + 1));
  int32_t** i32cols[] = {&src.frame, &src.label, &src.npix, &src.xmin,
                         &src.xmax, &src.ymin, &src.ymax, &src.peak_x,
                         &src.peak_y};
  for (auto c : i32cols) *c = (int32_t*)S.get(4 * cap);
  double** f64cols[] = {&src.peak, &src.flux_iso, &src.x, &src.y,
                        &src.flux_ap, &src.sky, &src.area_ap, &src.area_ann};
  for (auto c : f64cols) *c = (double*)S.get(8 * cap);
  src.flags = (uint32_t*)S.get(4 * cap);
  for (void* b : S.blocks)
    if (!b) return IPP_E_DEVICE;

  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  double best = 1e300;
  ipp_params bestp = *p;
  ipp_status last = IPP_OK;
  for (int m : meshes) {
    for (auto t : tiles) {
      ipp_params q = *p;
      q.mesh_h = q.mesh_w = m;
      q.tile_h = t.first;
      q.tile_w = t.second;
      const size_t need = ipp_workspace_bytes(frames, n, &q, 0);
      if (need == 0) continue;
      if ((last = ipp_ctx_reserve(ctx, need)) != IPP_OK) break;
      last = ipp_process_batch(ctx, frames, n, &q, maps.data(), &src,
                               nullptr, nullptr, stream);
      if (last != IPP_OK) break;
      hipEventRecord(e0, s);
      const int reps = 3;
      for (int r = 0; r < reps; ++r)
        ipp_process_batch(ctx, frames, n, &q, maps.data(), &src, nullptr,
                          nullptr, stream);
      hipEventRecord(e1, s);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      const double per = ms / reps;
      if (per < best) {
        best = per;
        bestp = q;
      }
    }
    if (last != IPP_OK) break;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipStreamSynchronize(s);
  if (best >= 1e300) return last != IPP_OK ? last : IPP_E_UNSUPPORTED;
  *p = bestp;
  if (best_ms) *best_ms = best;
  if (cache_path) cache_store(cache_path, key, bestp, best);
  return IPP_OK;
}
