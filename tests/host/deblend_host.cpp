// Test harness: the library's per-candidate deblending routine compiled
// for the host, so its algorithm can be compared with the oracle on a
// machine without a GPU.  Not part of the library.
#include <cstdlib>
#include <vector>

#include "../../paper_2502_10783_amd/csrc/deblend_core.h"

extern "C" int db_candidate(const double* val, int bw, int bh, int x0,
                            int y0, int npix, double t0, double peak,
                            int conn, int nthresh, int clean, double mincont,
                            double kc, int* asg_out) {
  using namespace ipp::db;
  const int64_t A = (int64_t)bw * bh;
  std::vector<char> buf(scratch_bytes(A, npix) + 16);
  char* b = buf.data();
  b += (16 - ((uintptr_t)b & 15)) & 15;
  Scratch s = carve(b, A, npix);
  for (int64_t p = 0; p < A; ++p) s.val[p] = val[p];
  Cand c;
  c.bw = bw;
  c.bh = bh;
  c.x0 = x0;
  c.y0 = y0;
  c.npix = npix;
  c.t0 = t0;
  c.peak = peak;
  c.conn = conn;
  c.nthresh = nthresh;
  c.clean = clean;
  c.mincont = mincont;
  c.kc = kc;
  const int k = deblend_one(c, s);
  for (int64_t p = 0; p < A; ++p) asg_out[p] = s.asg[p];
  return k;
}
