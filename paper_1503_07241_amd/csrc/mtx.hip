// Matrix Market input (the graph file format the paper's API reads, App. A
// ReadMTX): a "coordinate" matrix whose entry (i, j) is an edge i -> j
// (1-based in the file, 0-based here), with its value as the edge value.
// Host code only: the file is parsed into an edge list, then built on the
// device by gm_graph_from_coo.
#include <algorithm>
#include <cctype>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "gm_internal.h"

namespace gm {
namespace {

struct MtxHeader {
  int field = 0;  // 0 pattern, 1 integer, 2 real
  bool symmetric = false;
  int64_t rows = 0, cols = 0, entries = 0;
};

std::string lower(std::string s) {
  for (char& c : s) c = (char)std::tolower((unsigned char)c);
  return s;
}

// Parses the banner and the size line; leaves f at the first entry.
gm_status read_header(FILE* f, const char* path, MtxHeader* h) {
  char line[1024];
  if (!std::fgets(line, sizeof(line), f)) return fail(GM_EINVAL, "%s: empty file", path);
  char a[64] = {}, b[64] = {}, c[64] = {}, d[64] = {}, e[64] = {};
  if (std::sscanf(line, "%63s %63s %63s %63s %63s", a, b, c, d, e) != 5 ||
      lower(a) != "%%matrixmarket" || lower(b) != "matrix" || lower(c) != "coordinate")
    return fail(GM_EINVAL, "%s: not a MatrixMarket coordinate matrix", path);
  const std::string field = lower(d), sym = lower(e);
  if (field == "pattern")
    h->field = 0;
  else if (field == "integer")
    h->field = 1;
  else if (field == "real" || field == "double")
    h->field = 2;
  else
    return fail(GM_EUNSUPPORTED, "%s: field '%s' (pattern, integer or real)", path, d);
  if (sym == "general")
    h->symmetric = false;
  else if (sym == "symmetric")
    h->symmetric = true;
  else
    return fail(GM_EUNSUPPORTED, "%s: symmetry '%s' (general or symmetric)", path, e);
  while (std::fgets(line, sizeof(line), f)) {
    const char* p = line;
    while (*p == ' ' || *p == '\t') ++p;
    if (*p == '%' || *p == '\n' || *p == '\r' || *p == '\0') continue;
    long long r = 0, cc = 0, nz = 0;
    if (std::sscanf(p, "%lld %lld %lld", &r, &cc, &nz) != 3 || r < 0 || cc < 0 || nz < 0)
      return fail(GM_EINVAL, "%s: bad size line", path);
    h->rows = r;
    h->cols = cc;
    h->entries = nz;
    return GM_OK;
  }
  return fail(GM_EINVAL, "%s: no size line", path);
}

// Reads every entry into (src, dst, value) vectors, symmetric entries (i != j)
// twice, checking ids and values.
gm_status read_entries(FILE* f, const char* path, const MtxHeader& h, std::vector<int32_t>* src,
                       std::vector<int32_t>* dst, std::vector<double>* val) {
  char line[1024];
  int64_t got = 0;
  while (got < h.entries && std::fgets(line, sizeof(line), f)) {
    const char* p = line;
    while (*p == ' ' || *p == '\t') ++p;
    if (*p == '%' || *p == '\n' || *p == '\r' || *p == '\0') continue;
    char* q = nullptr;
    errno = 0;
    const long long i = std::strtoll(p, &q, 10);
    if (q == p) return fail(GM_EINVAL, "%s: entry %lld: no row", path, (long long)got + 1);
    p = q;
    const long long j = std::strtoll(p, &q, 10);
    if (q == p) return fail(GM_EINVAL, "%s: entry %lld: no column", path, (long long)got + 1);
    p = q;
    double v = 1.0;
    if (h.field != 0) {
      v = std::strtod(p, &q);
      if (q == p) return fail(GM_EINVAL, "%s: entry %lld: no value", path, (long long)got + 1);
    }
    if (i < 1 || i > h.rows || j < 1 || j > h.cols)
      return fail(GM_EINVAL, "%s: entry %lld (%lld, %lld) outside the %lld x %lld matrix", path,
                  (long long)got + 1, i, j, (long long)h.rows, (long long)h.cols);
    if (h.field == 1 && !(v >= 0 && v <= 4294967295.0 && v == std::floor(v)))  // NaN fails
      return fail(GM_EUNSUPPORTED, "%s: entry %lld: integer value %g is not a uint32", path,
                  (long long)got + 1, v);
    src->push_back((int32_t)(i - 1));
    dst->push_back((int32_t)(j - 1));
    val->push_back(v);
    if (h.symmetric && i != j) {
      src->push_back((int32_t)(j - 1));
      dst->push_back((int32_t)(i - 1));
      val->push_back(v);
    }
    ++got;
  }
  if (got < h.entries)
    return fail(GM_EINVAL, "%s: %lld entries announced, %lld found", path, (long long)h.entries,
                (long long)got);
  return GM_OK;
}

// The whole file as an edge list: n = max(rows, cols), values as the
// field's edge type.
gm_status read_mtx(const char* path, int64_t* n, std::vector<int32_t>* src,
                   std::vector<int32_t>* dst, std::vector<double>* val, int32_t* wtype) {
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(GM_EINVAL, "%s: cannot open (%s)", path, std::strerror(errno));
  MtxHeader h;
  gm_status st = read_header(f, path, &h);
  if (st == GM_OK && (h.rows > INT32_MAX || h.cols > INT32_MAX || h.rows + h.cols == 0))
    st = fail(GM_EINVAL, "%s: %lld x %lld matrix (1 .. 2^31 - 1 rows and columns)", path,
              (long long)h.rows, (long long)h.cols);
  if (st == GM_OK) st = read_entries(f, path, h, src, dst, val);
  std::fclose(f);
  if (st != GM_OK) return st;
  *n = std::max(h.rows, h.cols);
  *wtype = h.field == 0 ? GM_W_NONE : h.field == 1 ? GM_W_U32 : GM_W_F32;
  return GM_OK;
}

}  // namespace
}  // namespace gm

using namespace gm;

extern "C" {

gm_status gm_mtx_read(const char* path, int64_t* n, int64_t* m, int32_t* src, int32_t* dst,
                      void* w, int32_t* wtype) {
  if (!path || !n || !m || !wtype) return fail(GM_EINVAL, "path/n/m/wtype is NULL");
  return guarded([&]() -> gm_status {
    int64_t nn = 0;
    int32_t wt = GM_W_NONE;
    std::vector<int32_t> s, d;
    std::vector<double> v;
    if (const gm_status st = read_mtx(path, &nn, &s, &d, &v, &wt)) return st;
    const bool fill = src || dst || w;
    if (fill && (int64_t)s.size() > *m)
      return fail(GM_EINVAL, "%s: %zu edges do not fit arrays of %lld", path, s.size(),
                  (long long)*m);
    *n = nn;
    *m = (int64_t)s.size();
    *wtype = wt;
    if (src) std::memcpy(src, s.data(), s.size() * 4);
    if (dst) std::memcpy(dst, d.data(), d.size() * 4);
    if (w && wt == GM_W_U32)
      for (size_t e = 0; e < v.size(); ++e) static_cast<uint32_t*>(w)[e] = (uint32_t)v[e];
    if (w && wt == GM_W_F32)
      for (size_t e = 0; e < v.size(); ++e) static_cast<float*>(w)[e] = (float)v[e];
    return ok();
  });
}

gm_status gm_graph_from_mtx(const char* path, uint32_t prep, uint32_t layouts, void* stream,
                            gm_graph* out) {
  if (!out) return fail(GM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!path) return fail(GM_EINVAL, "path is NULL");
  int64_t n = 0;
  int32_t wt = GM_W_NONE;
  std::vector<int32_t> s, d;
  std::vector<double> v;
  gm_status st = guarded([&]() -> gm_status { return read_mtx(path, &n, &s, &d, &v, &wt); });
  if (st != GM_OK) return st;
  std::vector<uint32_t> wu;
  std::vector<float> wf;
  const void* w = nullptr;
  st = guarded([&]() -> gm_status {
    if (wt == GM_W_U32) {
      wu.resize(v.size());
      for (size_t e = 0; e < v.size(); ++e) wu[e] = (uint32_t)v[e];
      w = wu.data();
    } else if (wt == GM_W_F32) {
      wf.resize(v.size());
      for (size_t e = 0; e < v.size(); ++e) wf[e] = (float)v[e];
      w = wf.data();
    }
    return GM_OK;
  });
  if (st != GM_OK) return st;
  return gm_graph_from_coo(n, (int64_t)s.size(), s.data(), d.data(), s.empty() ? nullptr : w,
                           s.empty() ? GM_W_NONE : wt, prep, layouts, stream, out);
}

}  // extern "C"
