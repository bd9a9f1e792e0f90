// Host-only driver for the sanitizer build of the Matrix Market reader
// (test infrastructure): linked with csrc/mtx.hip alone, it defines the two
// status helpers the reader reports through and a graph builder that is
// never reached, then reads every file named on the command line twice (the
// count-only call, then the call that fills arrays of exactly that size) and
// prints "status n m checksum" per file.
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "gm_internal.h"

namespace gm {
gm_status fail(gm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return st;
}
gm_status ok() { return GM_OK; }
}  // namespace gm

extern "C" gm_status gm_graph_from_coo(int64_t, int64_t, const int32_t*, const int32_t*,
                                       const void*, int32_t, uint32_t, uint32_t, void*,
                                       gm_graph*) {
  return GM_EINVAL;
}

int main(int argc, char** argv) {
  for (int a = 1; a < argc; ++a) {
    int64_t n = 0, m = 0;
    int32_t wt = 0;
    gm_status st = gm_mtx_read(argv[a], &n, &m, nullptr, nullptr, nullptr, &wt);
    unsigned long long sum = 0;
    if (st == GM_OK) {
      std::vector<int32_t> src((size_t)m), dst((size_t)m);
      std::vector<uint32_t> w((size_t)m);
      st = gm_mtx_read(argv[a], &n, &m, src.data(), dst.data(), w.data(), &wt);
      for (int64_t e = 0; e < m && st == GM_OK; ++e)
        sum = sum * 1000003ull + (unsigned long long)(uint32_t)src[e] * 31ull +
              (uint32_t)dst[e] + (wt == GM_W_NONE ? 0ull : w[e]);
    }
    std::printf("%d %lld %lld %llu\n", (int)st, (long long)n, (long long)m, sum);
  }
  return 0;
}
