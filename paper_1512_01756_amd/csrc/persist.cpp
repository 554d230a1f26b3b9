// Saving and loading the host tables of a handle (every System), so a later
// process can skip the setup: a little-endian binary file of a magic, a layout
// version and a fixed header, followed by each system's scalars and arrays in
// declaration order.  A loaded file is checked field by field before any of
// it is used.
#include <algorithm>
#include <cmath>
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

constexpr char kMagic[8] = {'S', 'M', 'P', 'M', 'T', 'A', 'B', 'L'};
// Layout version of the tables that follow the header: bumped whenever a
// field of System or StripClass, or the meaning of one, changes.
constexpr int32_t kLayoutVersion = 2;
// Limits of the device path (the same as the setup's argument checks).
constexpr int kMaxPoints = 22, kMaxHalf = 544, kMaxInterfaces = 1024, kMaxCoarse = 4096;

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

void check(bool ok, const char *what) {
  if (!ok) throw std::invalid_argument(std::string("corrupt table file (") + what + ")");
}

template <typename T> void check_size(const std::vector<T> &v, uint64_t n, const char *what) {
  check(v.size() == n, what);
}

// Every index, window and size the device tables are built from, checked
// against the grid scalars, which are checked against the setup's limits:
// a file that passes cannot make the upload or a kernel reach outside its
// arrays.  Derived quantities must equal what the setup computes.
void validate(const TableHeader &h, const std::vector<System> &sys) {
  check(h.zlabel == 0 || h.zlabel == 1, "deflation space");
  check(h.my >= 0, "m_y");
  if (h.my > 0) {
    check(h.my >= 2 && std::isfinite(h.ly) && h.ly > 0.0, "Fourier period");
    check((int64_t)sys.size() == h.my / 2 + 1, "Fourier system count");
    // one grid, one mode per system: k_m = 2 pi m / l_y
    for (size_t m = 0; m < sys.size(); ++m) {
      const System &s = sys[m], &s0 = sys[0];
      check(s.mx == s0.mx && s.mz == s0.mz && s.n == s0.n && s.xb == s0.xb && s.zb == s0.zb, "Fourier grid");
      const double km = 2.0 * M_PI * (double)m / h.ly;
      check(std::fabs(s.kwave - km) <= 1e-12 * std::max(1.0, km), "Fourier wavenumber");
    }
  }
  for (const System &s : sys) {
    check(s.n >= 2 && s.n <= kMaxPoints && s.mx >= 2 && s.mz >= 1, "grid size");
    check((int64_t)s.n * s.mz <= kMaxHalf && s.mx - 1 <= kMaxInterfaces, "grid limits");
    const int n = s.n, mx = s.mx, mz = s.mz, n2 = n * n, N = n * mz, nh = 2 * (mx - 1);
    check(s.n2 == n2 && s.N == N && s.nh == nh, "derived sizes");
    check(s.zm == (h.zlabel ? mz : 1), "coarse columns per interface");
    check(s.d == (mx - 1) * s.zm && s.d <= kMaxCoarse, "coarse size");
    check(s.r == (int64_t)n2 * mx * mz && s.kS == (int64_t)N * nh, "vector lengths");
    check(std::isfinite(s.kwave) && s.kwave >= 0.0 && std::isfinite(s.tau) && s.tau != 0.0, "k or tau");
    check(s.singular == (s.kwave == 0.0), "singular flag");
    check_size(s.xb, mx + 1, "x breakpoints");
    check_size(s.zb, mz + 1, "z breakpoints");
    for (int j = 0; j < mx; ++j) check(std::isfinite(s.xb[j + 1] - s.xb[j]) && s.xb[j + 1] > s.xb[j], "x breakpoints");
    for (int e = 0; e < mz; ++e) check(std::isfinite(s.zb[e + 1] - s.zb[e]) && s.zb[e + 1] > s.zb[e], "z breakpoints");
    check_size(s.lo, (uint64_t)mz * n, "z couplings");
    check_size(s.up, (uint64_t)mz * n, "z couplings");
    const int ncl = (int)s.classes.size();
    check(ncl >= 1 && ncl <= mx, "strip class count");
    check_size(s.strip_class, mx, "strip classes");
    for (int c : s.strip_class) check(c >= 0 && c < ncl, "strip class id");
    const uint64_t nq = 2 * (uint64_t)n * (mz - 1);
    for (const StripClass &c : s.classes) {
      check_size(c.G, (uint64_t)mz * n2 * n2, "element factors");
      check_size(c.Dinv, (uint64_t)mz * n2 * n2, "element inverses");
      check_size(c.Kinv, nq * nq, "capacitance inverse");
      check_size(c.betaW, n, "B-row functionals");
      check_size(c.betaE, n, "B-row functionals");
      for (const auto &row : c.Wq)
        for (const auto &q : row) check(q.empty() || q.size() == (uint64_t)N * N, "Schur quarter blocks");
    }
    check(s.nW >= 1 && s.nW <= nh, "Schur block count");
    check_size(s.w_id, nh, "Schur block ids");
    check_size(s.w_win, nh, "Schur windows");
    check_size(s.Wblk, (uint64_t)s.nW * N * 2 * N, "Schur blocks");
    for (int hh = 0; hh < nh; ++hh) {
      check(s.w_id[hh] >= 0 && s.w_id[hh] < s.nW, "Schur block id");
      check(s.w_win[hh] == (hh % 2 == 0 ? hh + 1 : hh - 2), "Schur window");
    }
    check(s.nMblocks == mx / 2 && s.nM % 4 == 0 && s.nM >= 4 && s.nM <= 4 * s.nMblocks, "block-Jacobi count");
    check_size(s.m_id, nh, "block-Jacobi ids");
    check_size(s.m_win, nh, "block-Jacobi windows");
    check_size(s.m_K, nh, "block-Jacobi widths");
    check_size(s.Mblk, (uint64_t)s.nM * N * 4 * N, "block-Jacobi blocks");
    for (int hh = 0; hh < nh; ++hh) {
      const int h0 = 4 * (hh / 4);
      check(s.m_id[hh] >= 0 && s.m_id[hh] < s.nM && s.m_id[hh] % 4 == hh - h0, "block-Jacobi id");
      check(s.m_win[hh] == h0 && s.m_K[hh] == std::min(4, nh - h0) * N, "block-Jacobi window");
    }
    check(s.nF >= 0 && s.nF <= nh, "fused block count");
    check_size(s.f_id, nh, "fused ids");
    check_size(s.f_win, nh, "fused windows");
    check_size(s.f_K, nh, "fused widths");
    check_size(s.Fblk, (uint64_t)s.nF * N * 8 * N, "fused blocks");
    for (int hh = 0; hh < nh; ++hh) {
      if (s.nF == 0) {
        check(s.f_id[hh] == -1, "fused id");
        continue;
      }
      check(s.f_id[hh] >= 0 && s.f_id[hh] < s.nF, "fused id");
      check(s.f_win[hh] >= 0 && s.f_win[hh] % 4 == 0 && s.f_K[hh] > 0 && s.f_K[hh] % N == 0 &&
                s.f_K[hh] <= 8 * N && (int64_t)s.f_win[hh] * N + s.f_K[hh] <= s.kS,
            "fused window");
    }
    const uint64_t ncol = (uint64_t)nh * 2 * s.zm;
    check_size(s.sz_col, ncol, "coarse column ids");
    for (int c : s.sz_col) check(c >= -1 && c < s.d, "coarse column id");
    check_size(s.SZh, ncol * N, "S Z blocks");
    check_size(s.C, (uint64_t)s.d * s.d, "coarse matrix");
    check_size(s.Gc, (uint64_t)s.d * s.d, "coarse operator");
    const bool nv = s.singular;
    check_size(s.uS, nv ? s.kS : 0, "u_S");
    check_size(s.uL, nv ? s.r : 0, "u_L");
    check_size(s.uC, nv ? (uint64_t)s.d : 0, "u_C");
  }
}

}  // namespace

void save_tables(const char *path, const TableHeader &h, const std::vector<System> &sys) {
  File f(path, "wb");
  Writer w{f.f};
  w.raw(kMagic, sizeof(kMagic));
  w.pod(kLayoutVersion);
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
  int32_t version = 0;
  r.pod(version);
  if (version != kLayoutVersion)
    throw std::invalid_argument("table file of layout version " + std::to_string(version) + ", this library reads " +
                                std::to_string(kLayoutVersion));
  r.pod(h);
  if (h.nsys < 1 || h.nsys > (1 << 20)) throw std::invalid_argument("corrupt table file (system count)");
  sys.assign(h.nsys, System{});
  for (System &s : sys) visit(r, s);
  validate(h, sys);
}

}  // namespace smpm
