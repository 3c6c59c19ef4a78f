// On-disk cache of the host-built tables of a grid.  Building the exact ghost
// map is the slow part of hope_grid_create (seconds at C360); a cache file
// holds every table the device path needs, keyed by the parameters the tables
// depend on and by the build of the table code, so a later create with the
// same parameters only reads and checks the file.
//
// File: "HOPETAB1", the build stamp of the table code, the key, the scalars,
// then each table as (element count, raw little-endian elements), and an
// FNV-1a 64 checksum of everything before it.  A file that is missing,
// truncated, from another build, for other parameters, with a bad checksum
// or with an index outside its range is ignored and replaced.  The ghost
// map's per-entry values in uncompressed form (HostTables::g_val) are not
// stored; the device path reads the compressed records.
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unistd.h>

#include "hope.h"
#include "hope_internal.hpp"

namespace hope {
namespace {

const char kMagic[8] = {'H', 'O', 'P', 'E', 'T', 'A', 'B', '1'};

struct Key {
  int32_t n, k, weno, ghost_iters;
  double radius, eps, theta;
};

uint64_t fnv1a(uint64_t h, const void* p, size_t len) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < len; ++i) {
    h ^= b[i];
    h *= 1099511628211ULL;
  }
  return h;
}

std::string cache_path(const char* dir, const Key& key) {
  uint64_t h = fnv1a(14695981039346656037ULL, &key.n, 4 * sizeof(int32_t));
  h = fnv1a(h, &key.radius, 3 * sizeof(double));
  h = fnv1a(h, tables_build_stamp(), std::strlen(tables_build_stamp()));
  char name[64];
  std::snprintf(name, sizeof(name), "/hope_grid_%016" PRIx64 ".bin", h);
  return std::string(dir) + name;
}

// Sequential writer / reader with the running checksum.
struct Out {
  FILE* f;
  uint64_t h = 14695981039346656037ULL;
  bool ok = true;
  void raw(const void* p, size_t len) {
    if (!ok || len == 0) return;
    h = fnv1a(h, p, len);
    ok = std::fwrite(p, 1, len, f) == len;
  }
  template <typename T> void vec(const std::vector<T>& v) {
    const uint64_t c = v.size();
    raw(&c, sizeof(c));
    raw(v.data(), v.size() * sizeof(T));
  }
};

struct In {
  FILE* f;
  uint64_t h = 14695981039346656037ULL;
  bool ok = true;
  long remaining;
  void raw(void* p, size_t len) {
    if (!ok || len == 0) return;
    if ((long)len > remaining) { ok = false; return; }
    ok = std::fread(p, 1, len, f) == len;
    if (ok) { h = fnv1a(h, p, len); remaining -= (long)len; }
  }
  template <typename T> void vec(std::vector<T>& v) {
    uint64_t c = 0;
    raw(&c, sizeof(c));
    if (!ok || c > (uint64_t)remaining / sizeof(T)) { ok = false; return; }
    v.resize(c);
    raw(v.data(), c * sizeof(T));
  }
};

// The scalars and tables in file order; the same function writes and reads.
template <typename S> void scalars(S& s, HostTables& t) {
  int32_t iv[9] = {t.n, t.k, t.r, t.m, t.P, t.weno, t.l, t.s, t.ghost_sweeps};
  double dv[4] = {t.radius, t.eps, t.theta, t.delta};
  s.raw(iv, sizeof(iv));
  s.raw(dv, sizeof(dv));
  t.n = iv[0]; t.k = iv[1]; t.r = iv[2]; t.m = iv[3]; t.P = iv[4]; t.weno = iv[5]; t.l = iv[6]; t.s = iv[7];
  t.ghost_sweeps = iv[8];
  t.radius = dv[0]; t.eps = dv[1]; t.theta = dv[2]; t.delta = dv[3];
}

template <typename S> void tables(S& s, HostTables& t) {
  s.vec(t.gnode); s.vec(t.gw); s.vec(t.wc); s.vec(t.wsub);
  s.vec(t.gp); s.vec(t.gm); s.vec(t.sp); s.vec(t.sm); s.vec(t.d1); s.vec(t.V); s.vec(t.lam);
  s.vec(t.Xe); s.vec(t.Xg); s.vec(t.sqe); s.vec(t.sqg);
  s.vec(t.g_dst); s.vec(t.g_ptr); s.vec(t.g_col);
  s.vec(t.z_dst); s.vec(t.z_info); s.vec(t.z_ptr); s.vec(t.z_ent); s.vec(t.z_cval);
  s.vec(t.bt_cell); s.vec(t.bt_side); s.vec(t.bt_rev); s.vec(t.bt_conv);
}

bool in_range(const std::vector<int32_t>& v, int64_t lo, int64_t hi) {
  for (int32_t x : v)
    if (x < lo || x >= hi) return false;
  return true;
}

bool row_pointers(const std::vector<int32_t>& ptr, size_t rows, size_t nnz) {
  if (ptr.size() != rows + 1 || ptr[0] != 0 || (size_t)ptr[rows] != nnz) return false;
  for (size_t i = 0; i < rows; ++i)
    if (ptr[i + 1] < ptr[i]) return false;
  return true;
}

// Sizes and index ranges of loaded tables, so that no kernel or host loop
// can index outside them.
bool consistent(const HostTables& t, const Key& key) {
  const int n = t.n, k = t.k, m = t.m;
  if (n != key.n || k != key.k || t.weno != key.weno || t.r != (k - 1) / 2 || m != (k + 1) / 2 ||
      t.P != n + 2 * t.r)
    return false;
  const int64_t plane = 6LL * t.P * t.P;
  if (t.gnode.size() != (size_t)m || t.gw.size() != (size_t)m || t.wc.size() != (size_t)(2 + m) * k) return false;
  if (t.Xe.size() != (size_t)n + 1 || t.sqe.size() != (size_t)n + 1 || t.Xg.size() != (size_t)n * m ||
      t.sqg.size() != (size_t)n * m)
    return false;
  if (t.weno) {
    const size_t l = (size_t)(k + 1) / 2, npts = 4 * (size_t)m + (size_t)m * m;
    if ((size_t)t.l != l || (size_t)t.s != l * l || t.wsub.size() != l * (2 + m) * l ||
        t.d1.size() != (2 + m) * l || t.V.size() != l * l * l || t.lam.size() != l * l ||
        t.gp.size() != npts * l * l || t.gm.size() != npts * l * l || t.sp.size() != npts || t.sm.size() != npts)
      return false;
  } else if (!t.wsub.empty() || !t.gp.empty() || !t.gm.empty() || !t.sp.empty() || !t.sm.empty() ||
             !t.d1.empty() || !t.V.empty() || !t.lam.empty()) {
    return false;
  }
  // ghost map, plain rows (the adjoint's transpose is built from them)
  const size_t rows = t.g_dst.size();
  if (!row_pointers(t.g_ptr, rows, t.g_col.size()) || !in_range(t.g_dst, 0, plane) ||
      !in_range(t.g_col, 0, plane))
    return false;
  // compressed rows
  const size_t zrows = t.z_dst.size();
  if (zrows != rows || t.z_info.size() != zrows || t.z_ent.size() != 2 * t.g_col.size() ||
      !row_pointers(t.z_ptr, zrows, t.z_ent.size() / 2) || !in_range(t.z_dst, 0, plane) || t.z_cval.size() % 6)
    return false;
  const int64_t records = (int64_t)(t.z_cval.size() / 6);
  for (size_t zr = 0; zr < zrows; ++zr) {
    const int64_t base = t.z_info[zr] & 0x0fffffff;
    for (int32_t e = t.z_ptr[zr]; e < t.z_ptr[zr + 1]; ++e) {
      const int32_t col = t.z_ent[2 * (size_t)e], ce = t.z_ent[2 * (size_t)e + 1];
      if (col < 0 || col >= plane || ce < 0 || base + (ce & 0x1fff) >= records) return false;
    }
  }
  // panel-edge maps
  const size_t sides = 24 * (size_t)n;
  if (t.bt_cell.size() != sides || t.bt_side.size() != sides || t.bt_rev.size() != sides ||
      t.bt_conv.size() != sides * m * 5 || !in_range(t.bt_cell, 0, plane) || !in_range(t.bt_side, 0, 4) ||
      !in_range(t.bt_rev, 0, 2))
    return false;
  return true;
}

bool load(const std::string& path, const Key& key, HostTables& t) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return false;
  std::fseek(f, 0, SEEK_END);
  const long size = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  In in{f};
  in.remaining = size - (long)sizeof(uint64_t);
  char magic[8] = {};
  in.raw(magic, sizeof(magic));
  char stamp[64] = {};
  in.raw(stamp, sizeof(stamp));
  Key fk{};
  in.raw(&fk, sizeof(fk));
  bool ok = in.ok && std::memcmp(magic, kMagic, 8) == 0 &&
            std::strncmp(stamp, tables_build_stamp(), sizeof(stamp) - 1) == 0 && std::memcmp(&fk, &key, sizeof(key)) == 0;
  if (ok) {
    scalars(in, t);
    tables(in, t);
    uint64_t sum = 0;
    const uint64_t h = in.h;
    ok = in.ok && in.remaining == 0 && std::fread(&sum, sizeof(sum), 1, f) == 1 && sum == h;
  }
  std::fclose(f);
  return ok && consistent(t, key);
}

void store(const std::string& path, const Key& key, HostTables& t) {
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return;
  Out out{f};
  out.raw(kMagic, sizeof(kMagic));
  char stamp[64] = {};
  std::strncpy(stamp, tables_build_stamp(), sizeof(stamp) - 1);
  out.raw(stamp, sizeof(stamp));
  out.raw(&key, sizeof(key));
  scalars(out, t);
  tables(out, t);
  const uint64_t sum = out.h;
  bool ok = out.ok && std::fwrite(&sum, sizeof(sum), 1, f) == 1;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

}  // namespace

int build_tables_cached(HostTables& t, const char* dir, bool* loaded, int n, int k, int weno, double radius,
                        double omega, double tilt, double eps, double theta, int ghost_iters) {
  *loaded = false;
  if (!dir || !*dir) return build_tables(t, n, k, weno, radius, omega, tilt, eps, theta, ghost_iters);
  Key key{};
  key.n = n; key.k = k; key.weno = weno; key.ghost_iters = ghost_iters;
  key.radius = radius; key.eps = eps; key.theta = theta;
  const std::string path = cache_path(dir, key);
  if (load(path, key, t)) {
    // the rotation of the axis enters only the Coriolis coefficients
    t.omega = omega;
    t.tilt = tilt;
    t.fcoef.assign(18, 0.0);
    coriolis_coefs(tilt, t.fcoef.data());
    *loaded = true;
    return 0;
  }
  t = HostTables();
  const int st = build_tables(t, n, k, weno, radius, omega, tilt, eps, theta, ghost_iters);
  if (st == 0) store(path, key, t);
  return st;
}

}  // namespace hope
