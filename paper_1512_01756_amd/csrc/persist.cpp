// Saving and loading the host tables of a handle (every System), so a later
// process can skip the setup: a little-endian binary file of a fixed header
// followed by each system's scalars and arrays in declaration order.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "host.hpp"
#include "persist.hpp"

namespace smpm {
namespace {

constexpr char kMagic[8] = {'S', 'M', 'P', 'M', 'T', 'A', 'B', '1'};

struct File {
  std::FILE *f = nullptr;
  explicit File(const char *path, const char *mode) : f(std::fopen(path, mode)) {
    if (!f) throw std::runtime_error(std::string("cannot open ") + path);
  }
  ~File() {
    if (f) std::fclose(f);
  }
};

struct Writer {
  std::FILE *f;
  void raw(const void *p, size_t n) {
    if (n && std::fwrite(p, 1, n, f) != n) throw std::runtime_error("write failed");
  }
  template <typename T> void pod(const T &v) { raw(&v, sizeof(T)); }
  template <typename T> void vec(const std::vector<T> &v) {
    const uint64_t n = v.size();
    pod(n);
    raw(v.data(), n * sizeof(T));
  }
};

struct Reader {
  std::FILE *f;
  void raw(void *p, size_t n) {
    if (n && std::fread(p, 1, n, f) != n) throw std::runtime_error("truncated or unreadable table file");
  }
  template <typename T> void pod(T &v) { raw(&v, sizeof(T)); }
  template <typename T> void vec(std::vector<T> &v) {
    uint64_t n = 0;
    pod(n);
    if (n > (uint64_t(1) << 40) / sizeof(T)) throw std::runtime_error("corrupt table file (array size)");
    v.resize(n);
    raw(v.data(), n * sizeof(T));
  }
};

// One function visits every field for both directions.
template <typename IO> void visit(IO &io, StripClass &c) {
  io.pod(c.hx);
  io.pod(c.west_if);
  io.pod(c.east_if);
  io.vec(c.G);
  io.vec(c.Dinv);
  io.vec(c.Kinv);
  io.vec(c.betaW);
  io.vec(c.betaE);
  for (auto &row : c.Wq)
    for (auto &q : row) io.vec(q);
}

template <typename IO> void visit(IO &io, System &s) {
  io.pod(s.n); io.pod(s.mx); io.pod(s.mz); io.pod(s.n2); io.pod(s.N); io.pod(s.nh); io.pod(s.d); io.pod(s.zm);
  io.pod(s.r); io.pod(s.kS); io.pod(s.kwave); io.pod(s.tau); io.pod(s.singular);
  io.vec(s.xb); io.vec(s.zb); io.vec(s.lo); io.vec(s.up); io.vec(s.strip_class);
  uint64_t nc = s.classes.size();
  io.pod(nc);
  s.classes.resize(nc);
  for (auto &c : s.classes) visit(io, c);
  io.vec(s.w_id); io.vec(s.w_win); io.vec(s.Wblk); io.pod(s.nW);
  io.vec(s.m_id); io.vec(s.m_win); io.vec(s.m_K); io.vec(s.Mblk); io.pod(s.nM); io.pod(s.nMblocks);
  io.vec(s.f_id); io.vec(s.f_win); io.vec(s.f_K); io.vec(s.Fblk); io.pod(s.nF);
  io.vec(s.sz_col); io.vec(s.SZh); io.vec(s.C); io.vec(s.Gc);
  io.vec(s.uS); io.vec(s.uL); io.vec(s.uC);
}

}  // namespace

void save_tables(const char *path, const TableHeader &h, const std::vector<System> &sys) {
  File f(path, "wb");
  Writer w{f.f};
  w.raw(kMagic, sizeof(kMagic));
  TableHeader hh = h;
  hh.nsys = (int32_t)sys.size();
  w.pod(hh);
  for (const System &s : sys) visit(w, const_cast<System &>(s));
  if (std::fflush(f.f) != 0) throw std::runtime_error("write failed");
}

void load_tables(const char *path, TableHeader &h, std::vector<System> &sys) {
  File f(path, "rb");
  Reader r{f.f};
  char magic[sizeof(kMagic)];
  r.raw(magic, sizeof(magic));
  if (std::memcmp(magic, kMagic, sizeof(kMagic)) != 0) throw std::invalid_argument("not a saved SMPM table file");
  r.pod(h);
  if (h.nsys < 1 || h.nsys > (1 << 20)) throw std::invalid_argument("corrupt table file (system count)");
  sys.assign(h.nsys, System{});
  for (System &s : sys) visit(r, s);
}

}  // namespace smpm
