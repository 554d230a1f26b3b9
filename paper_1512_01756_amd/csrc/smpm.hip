// C ABI of the SMPM Schur solver: setup (host FP64 tables -> device), the
// batched Algorithm 2 solve, FP64 iterative refinement around an FP32 inner
// solve, single-operator applies and table export.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <future>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/smpm_schur.h"
#include "device.hpp"
#include "host.hpp"
#include "setup_dev.hpp"
#include "persist.hpp"
#include "kernels.hip"

using namespace smpm;

namespace {

thread_local std::string g_err;

smpm_status fail(smpm_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define HIPCHECK(expr)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw HipError(std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

template <typename T>
T *dalloc(std::vector<void *> &owned, size_t count) {
  if (count == 0) count = 1;
  void *p = nullptr;
  if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) throw std::bad_alloc();
  owned.push_back(p);
  return static_cast<T *>(p);
}

// Device copy, column-major with the rows padded to ld, of nb row-major
// rows x cols blocks given as `parts` (consecutive runs of whole blocks, e.g.
// one per strip class): the host memory goes up as it is and the device
// transposes it, so the host neither copies nor transposes the tables.
double *dupload_cm(std::vector<void *> &owned, const std::vector<std::pair<const double *, size_t>> &parts, int nb,
                   int rows, int cols, int ld, hipStream_t st) {
  double *out = dalloc<double>(owned, (size_t)nb * ld * cols);
  if (nb == 0) return out;
  double *raw = nullptr;
  if (hipMalloc((void **)&raw, sizeof(double) * (size_t)nb * rows * cols) != hipSuccess) throw std::bad_alloc();
  try {
    size_t off = 0;
    for (const auto &pr : parts) {
      if (pr.second)
        HIPCHECK(hipMemcpyAsync(raw + off, pr.first, sizeof(double) * pr.second, hipMemcpyHostToDevice, st));
      off += pr.second;
    }
    if (off != (size_t)nb * rows * cols) throw std::runtime_error("table upload: sizes do not add up");
    const dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((ld + 31) / 32), (unsigned)std::min(nb, 65535));
    hipLaunchKernelGGL(k_colmajor_pad, grid, dim3(32, 8), 0, st, (const double *)raw, out, nb, rows, cols, ld);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(st));
  } catch (...) {
    (void)hipFree(raw);
    throw;
  }
  HIPCHECK(hipFree(raw));
  return out;
}

double *dupload_cm(std::vector<void *> &owned, const std::vector<double> &a, int nb, int rows, int cols, int ld,
                   hipStream_t st) {
  return dupload_cm(owned, {{a.data(), a.size()}}, nb, rows, cols, ld, st);
}

template <typename T>
T *dupload(std::vector<void *> &owned, const std::vector<T> &v, hipStream_t st) {
  T *p = dalloc<T>(owned, v.size());
  if (!v.empty()) HIPCHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return p;
}

// Columns [c0, c1) of one row-major rows x cols block into column-major
// storage with leading dimension ld, in 32 x 32 tiles.
template <typename T>
void colmajor_cols(const double *ab, int rows, int cols, int ld, int c0, int c1, T *ob) {
  constexpr int TB = 32;
  for (int r0 = 0; r0 < rows; r0 += TB) {
    const int r1 = std::min(rows, r0 + TB);
    for (int c = c0; c < c1; ++c)
      for (int r = r0; r < r1; ++r) ob[(size_t)c * ld + r] = (T)ab[(size_t)r * cols + c];
  }
}

// Column-major copy with the row count padded to ld (zero rows) of nb
// row-major blocks of rows x cols, on the host threads over (block, 32-column
// slice): the tables reach a GB on distinct-strip grids.
template <typename T>
std::vector<T> to_colmajor_padded(const std::vector<double> &a, int nb, int rows, int cols, int ld) {
  std::vector<T> out((size_t)nb * ld * cols, (T)0);
  const int ct = (cols + 31) / 32;
  parallel_for(nb * ct, 0, [&](int q) {
    const int b = q / ct, c0 = (q % ct) * 32;
    colmajor_cols(a.data() + (size_t)b * rows * cols, rows, cols, ld, c0, std::min(cols, c0 + 32),
                  out.data() + (size_t)b * ld * cols);
  });
  return out;
}

// Column-major copy of row-major blocks: nb blocks of rows x cols.
template <typename T>
std::vector<T> to_colmajor(const std::vector<double> &a, int nb, int rows, int cols) {
  return to_colmajor_padded<T>(a, nb, rows, cols, rows);
}

// FP32 copy on the device of an uploaded FP64 table (the same layout).
float *dconvert32(std::vector<void *> &owned, const double *src, size_t n, hipStream_t st) {
  float *p = dalloc<float>(owned, n);
  if (n > 0)
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, src, p, (int64_t)n);
  return p;
}

// FP16 copy of nb row-major rows x cols blocks, column-major with leading
// dimension ld: every segment of `seg` rows (one element's nodes) is divided by
// its largest magnitude, which goes to scale[b][row / seg].
std::vector<_Float16> to_half_scaled(const std::vector<double> &a, int nb, int rows, int cols, int ld, int seg,
                                     std::vector<float> &scale) {
  const int nseg = rows / seg;
  std::vector<_Float16> out((size_t)nb * ld * cols, (_Float16)0.0f);
  scale.assign((size_t)nb * nseg, 1.0f);
  parallel_for(nb, 0, [&](int b) {
    for (int e = 0; e < nseg; ++e) {
      double mx = 0.0;
      for (int r = e * seg; r < (e + 1) * seg; ++r)
        for (int c = 0; c < cols; ++c) mx = std::max(mx, std::fabs(a[(size_t)b * rows * cols + (size_t)r * cols + c]));
      const double sc = mx > 0.0 ? mx : 1.0;
      scale[(size_t)b * nseg + e] = (float)sc;
      for (int r = e * seg; r < (e + 1) * seg; ++r)
        for (int c = 0; c < cols; ++c)
          out[(size_t)b * ld * cols + (size_t)c * ld + r] =
              (_Float16)(float)(a[(size_t)b * rows * cols + (size_t)r * cols + c] / sc);
    }
  });
  return out;
}

constexpr int kIterChunk = 4;
// Handles with at most this many vector workgroups (kChunk elements each)
// run the GMRES vector kernels with the short basis in registers: c2 (68)
// and c3 (208) gain 1-3%, the 3380 of c4's 130 instances lose 6% to the
// halved occupancy.
constexpr int kRegBasisChunks = 1024;
// A refinement sweep's inner solve stops once its residual is below
// kSweepSafety * tol * ||b~|| (or inner_tol times its own right-hand side).
constexpr double kSweepSafety = 0.5;
// Refinement stops with ENOTCONV when a sweep leaves the worst relative
// residual above this fraction of the previous sweep's.
constexpr double kStagnation = 0.9;
constexpr int kWaves = 16;   // waves per workgroup of the GEMV-shaped kernels

}  // namespace

// One batched shared-block GEMM item list: the items, the most windows in
// one item, and two XCD-ordered unit lists over it ((item, 64-row tile), and
// 128-row tiles costliest first).
struct GList {
  const GWork *w = nullptr;
  int n = 0, maxv = 0;
  const int2 *u = nullptr, *u128 = nullptr;
  int nu = 0, nu128 = 0;
};

struct smpm_handle {
  smpm_opts opts{};
  int nrhs = 1, maxit = 300, precision = SMPM_FP64, method = SMPM_METHOD_DBJ, max_sweeps = 12;
  double tol = 1e-10, inner_tol = 1e-4;
  bool host_only = false, no_tune = false;
  std::vector<System> sys;

  std::vector<void *> owned;
  std::vector<SysDev> h_sys;
  std::vector<InstDev> h_ins;
  SysDev *d_sys = nullptr;
  InstDev *d_ins = nullptr;
  int ninst = 0, Nmax = 0, group = 1, nq_max = 0, n2_max = 0;
  // Work lists: grouped halves for S and M^-1, plain halves, element items,
  // interface and node vector chunks.  Per instance [start, start + count).
  // Systems whose strips share blocks use the MFMA GEMM: items over windows
  // grouped by block id across all instances of a system (batched launches),
  // and within one instance (single-system applies).
  // Per operator: 0 S, 1 M^-1, 2 S M^-1 (fused, grids whose strips share blocks).
  // gl[op][0]: items of up to kGemmVecs windows (16 for S M^-1); gl[op][1]:
  // the S and M^-1 lists again in items of up to 16 windows, for the narrow
  // schedules (empty when list 0 has no wider item).  g_list: the list the
  // tuner picked per [op][precision].
  GList gl[3][2] = {};
  int g_list[3][3] = {};
  GWork *g_one[3] = {};
  GVec *g_vec = nullptr;
  bool fused = false;    // every system has S M^-1 blocks
  bool use_fused[3] = {}; // per precision: one S M^-1 GEMM per iteration beat M^-1 then S at setup
  // GEMM schedule of each batched list, picked at setup by timing every
  // candidate: [op][precision] for the matvec lists, [kind][width] for the
  // element-interior lists.
  int sched[3][3] = {};   // [op][FP64, FP32, FP16 storage]
  int cg_sched[3][2] = {};
  // B A^-1 per strip class (the Schur right-hand side as one GEMM), for
  // handles whose systems all share strip classes
  bool use_ba = false;
  // the Schur right-hand side GEMM over the strips, in items of up to
  // kGemmVecs windows (list 0) and of up to 16 (list 1, for the narrow
  // schedules; empty when list 0 has no wider item); the tuner picks the
  // list and the schedule
  const GWork *g_bal[2] = {nullptr, nullptr};
  int n_bal[2] = {0, 0}, bal_maxv[2] = {0, 0};
  int ba_list = 0, ba_sched = 0;
  std::vector<int> g_start[3], g_cnt[3];
  HWork *w_S1 = nullptr, *w_M1 = nullptr;   // single items (streamed blocks)
  int n_S1 = 0, n_M1 = 0;
  std::vector<int> S1_start, S1_cnt, M1_start, M1_cnt;
  int2 *w_h = nullptr, *w_x = nullptr, *w_r = nullptr, *w_s = nullptr;
  // Element-interior GEMM items, kind 0: w = D^-1 v, 1: q = K^-1 lambda,
  // 2: v -= D^-1 P q; batched over all instances, and per instance.
  // Index [kind][w]: w = 0 items of at most 16 columns, w = 1 of up to 64.
  CGItem *cg_all[3][2] = {}, *cg_one[3][2] = {};
  CGCol *cg_cols = nullptr;
  int n_cg_all[3][2] = {};
  int2 *cg_units[3][2] = {};   // XCD-ordered (item, 64-row tile) lists of cg_all
  int n_cg_units[3][2] = {};
  // Each product again in items of at most 16 columns, as one launch of the
  // 16-column kernel (products with a wide item only); used instead of the
  // two width lists where the tuner found it faster.
  CGItem *cg_alt[3] = {};
  int n_cg_alt[3] = {};
  int2 *cg_alt_units[3] = {};
  int n_cg_alt_units[3] = {};
  int cg_alt_sched[3] = {-1, -1, -1};   // -1: the two width lists
  std::vector<int> cg_start[3][2], cg_cnt[3][2];
  int n_h = 0, n_x = 0, n_r = 0, n_s = 0;
  std::vector<int> h_start, x_start, r_start, s_start;
  int64_t tot_r = 0, tot_x = 0, tot_g = 0;

  double *F = nullptr, *v = nullptr, *Rr = nullptr, *bS = nullptr, *xS = nullptr, *rb = nullptr;
  double *z64 = nullptr, *y64 = nullptr, *t64 = nullptr;
  float *z32 = nullptr, *y32 = nullptr, *t32 = nullptr;
  double *V64 = nullptr;
  float *V32 = nullptr;
  double *part1 = nullptr, *part2 = nullptr, *partn = nullptr, *pr = nullptr, *hs = nullptr;
  int *arrive = nullptr;   // per instance: workgroups of the second CGS pass that have finished
  double *cv = nullptr, *tb = nullptr, *scale = nullptr, *Rm = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr;
  double *ycoef = nullptr, *defect = nullptr, *pairs = nullptr, *lam = nullptr, *qb = nullptr;
  double *nb2 = nullptr;   // ||b~||^2 and u_S . b~ per instance, kept from the staging step
  bool one_krylov = false; // one GMRES over every instance (SMPM_FLAG_ONE_KRYLOV)
  int zlabel = 0;          // deflation space: 0 per interface, 1 per element segment
  bool op16 = false;       // FP16 operator copies for the refinement's inner solve
  int dmax = 1;            // largest coarse dimension d over the systems
  double *sr1 = nullptr, *sr2 = nullptr, *srn = nullptr;   // segment sums (st_off layout)
  GState *gs = nullptr;
  GState *h_gs = nullptr;      // pinned
  double *h_pairs = nullptr;   // pinned
  double *h_defect = nullptr;  // pinned
  // The solve runs on an internal stream (default priority) ordered against
  // the caller's stream with events; the GMRES iteration is replayed from a
  // captured graph of kIterChunk iterations per precision.
  hipStream_t ws = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // Captured graphs, index [0] FP64 inner solve, [1] FP32 inner solve:
  // before the Krylov loop, kIterChunk iterations (g_rem: 1 .. kIterChunk - 1
  // iterations), after the loop.  The staging graph is keyed by the caller's
  // f and g, the recovery graph by u; the FP64 solve runs as a head graph
  // (staging and the loop set-up, keyed by f and g) and a tail graph (the
  // loop's end, the residual check and the recovery, keyed by u).
  hipGraphExec_t g_pre[2] = {}, g_loop[2] = {}, g_post[2] = {};
  hipGraphExec_t g_rem[2][kIterChunk] = {};
  hipGraphExec_t g_resid = nullptr, g_stage = nullptr, g_finish = nullptr;
  hipGraphExec_t g_head = nullptr, g_tail = nullptr;
  // Iterations launched before the first convergence check: the previous
  // solve's count (-1: none yet, one chunk).
  int pred_iters[2] = {-1, -1};
  // The refinement's inner solves, per sweep index (later sweeps need fewer
  // iterations): the previous solve's count of that sweep, -1 if none; and
  // the previous solve's number of sweeps (0: none yet).
  std::vector<int> pred_sweep;
  int pred_nsweeps = 0;
  // Iterations added to each prediction once a solve of this handle had to
  // go past one (a resumed FP64 loop, a cut-short inner solve or a checked
  // sweep after the unchecked ones): 0 until then, so a handle whose counts
  // never change runs exactly its previous count.
  int pred_margin[2] = {0, 0};
  // Vector kernels with the short Krylov basis in registers: for handles
  // whose vector launches are at most kRegBasisChunks workgroups.
  bool reg_basis = false;
  // The FP64 solve's report, read back with one copy: GMRES states, then
  // (||r||^2, u_S . r), the compatibility defects and (||b~||^2, u_S . b~)
  // per instance (gs, pairs, defect and nb2 point into it).
  size_t rep_bytes = 0;
  char *h_rep = nullptr;       // pinned
  // 3-D problems (smpm_setup_fourier): m_y planes, the forward and inverse
  // real DFT matrices ([2 nk][m_y] and [m_y][2 nk], row-major), and the
  // coefficient buffers of f, g, u in the batched layouts.
  int my = 0;
  double ly = 0.0;
  double *dft_f = nullptr, *dft_i = nullptr, *fhat = nullptr, *ghat = nullptr, *uhat = nullptr;
  double2 *fft_tw = nullptr;   // exp(-2 pi i k / m_y), k < m_y / 2 (m_y a power of two)
  GState *h_gs_hist = nullptr;   // pinned, [sweep][instance]
  double *h_nb = nullptr;        // pinned, ||b~||^2 and u_S . b~ per instance

  ~smpm_handle() {
    for (hipGraphExec_t *e : {&g_pre[0], &g_pre[1], &g_loop[0], &g_loop[1], &g_post[0], &g_post[1], &g_resid,
                              &g_stage, &g_finish, &g_head, &g_tail})
      if (*e) (void)hipGraphExecDestroy(*e);
    for (auto &r : g_rem)
      for (hipGraphExec_t e : r)
        if (e) (void)hipGraphExecDestroy(e);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (ws) (void)hipStreamDestroy(ws);
    for (void *p : owned) (void)hipFree(p);
    if (h_gs) (void)hipHostFree(h_gs);
    if (h_pairs) (void)hipHostFree(h_pairs);
    if (h_defect) (void)hipHostFree(h_defect);
    if (h_gs_hist) (void)hipHostFree(h_gs_hist);
    if (h_nb) (void)hipHostFree(h_nb);
    if (h_rep) (void)hipHostFree(h_rep);
  }
};

namespace {

// XCD-aware launch order for the throughput GEMMs: workgroup L of a 1-D grid
// runs on XCD L mod kXcds.  Tiles are bucketed by the block they read (key),
// blocks are assigned to buckets largest first onto the least loaded bucket,
// and bucket b fills grid positions b, b + kXcds, ...; short buckets are
// padded with (-1, 0) entries, which exit at once.
constexpr int kXcds = 8;
std::vector<int2> xcd_units(const std::vector<uintptr_t> &key, const std::vector<int> &tiles,
                            const std::vector<std::vector<int64_t>> *cost = nullptr) {
  // cost of (item, tile): given, or one per tile
  auto c = [&](int i, int r) -> int64_t { return cost ? (*cost)[i][r] : 1; };
  std::map<uintptr_t, std::vector<int>> by;
  for (int i = 0; i < (int)key.size(); ++i) by[key[i]].push_back(i);
  std::vector<std::pair<int64_t, uintptr_t>> order;
  for (auto &kv : by) {
    int64_t t = 0;
    for (int i : kv.second)
      for (int r = 0; r < tiles[i]; ++r) t += c(i, r);
    order.push_back({t, kv.first});
  }
  std::stable_sort(order.begin(), order.end(), [](auto &a, auto &b) { return a.first > b.first; });
  std::vector<std::vector<int2>> bucket(kXcds);
  std::vector<int64_t> load(kXcds, 0);
  for (auto &o : order) {
    const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    for (int i : by[o.second])
      for (int r = 0; r < tiles[i]; ++r) bucket[b].push_back(make_int2(i, r));
    load[b] += o.first;
  }
  // with costs, each XCD takes its tiles costliest first (the dispatcher
  // hands them out in order as slots free up: longest-first list scheduling)
  if (cost)
    for (auto &bk : bucket)
      std::stable_sort(bk.begin(), bk.end(), [&](const int2 &a, const int2 &b) { return c(a.x, a.y) > c(b.x, b.y); });
  size_t depth = 0;
  for (auto &bk : bucket) depth = std::max(depth, bk.size());
  std::vector<int2> u(depth * kXcds, make_int2(-1, 0));
  for (int b = 0; b < kXcds; ++b)
    for (size_t k = 0; k < bucket[b].size(); ++k) u[k * kXcds + b] = bucket[b][k];
  return u;
}

// True if some block id serves more than one half.
bool shares_blocks(const std::vector<int> &ids) {
  std::map<int, int> c;
  for (int id : ids)
    if (++c[id] > 1) return true;
  return false;
}

// Group the halves of one instance that share a block id (up to `group`).
void group_halves(int inst, const std::vector<int> &ids, int group, std::vector<HWork> &out) {
  std::map<int, std::vector<int>> by;
  for (int h = 0; h < (int)ids.size(); ++h) by[ids[h]].push_back(h);
  for (auto &kv : by) {
    const std::vector<int> &hs = kv.second;
    for (size_t a = 0; a < hs.size(); a += group) {
      HWork w{};
      w.inst = inst;
      w.cnt = (int)std::min<size_t>(group, hs.size() - a);
      for (int q = 0; q < kGroup; ++q) w.h[q] = q < w.cnt ? hs[a + q] : hs[a];
      out.push_back(w);
    }
  }
}

void upload(smpm_handle *H, hipStream_t st) {
  auto &own = H->owned;
  const int maxit = H->maxit;
  for (System &s : H->sys) {
    H->Nmax = std::max(H->Nmax, s.N);
    H->nq_max = std::max(H->nq_max, 2 * s.n * (s.mz - 1));
    H->n2_max = std::max(H->n2_max, s.n2);
  }
  // Group size bounded by the GEMV's LDS budget (windows + wave partials).
  for (System &s : H->sys) {
    SysDev d{};
    d.n = s.n; d.mx = s.mx; d.mz = s.mz; d.n2 = s.n2; d.N = s.N; d.nh = s.nh; d.d = s.d; d.zm = s.zm;
    H->dmax = std::max(H->dmax, s.d);
    d.singular = s.singular ? 1 : 0; d.kS = s.kS; d.r = s.r; d.tau = s.tau;
    d.nq = 2 * s.n * (s.mz - 1);
    d.Np = (s.N + 7) / 8 * 8;   // 16-byte columns in FP64, FP32 and FP16
    d.W64 = dupload_cm(own, s.Wblk, s.nW, s.N, 2 * s.N, d.Np, st);
    d.W32 = dconvert32(own, d.W64, (size_t)s.nW * 2 * s.N * d.Np, st);
    if (s.nF > 0) {
      d.F64 = dupload_cm(own, s.Fblk, s.nF, s.N, 8 * s.N, d.Np, st);
      d.F32 = dconvert32(own, d.F64, (size_t)s.nF * 8 * s.N * d.Np, st);
    }
    if (H->op16) {
      std::vector<float> sc;
      if (s.nF > 0) {
        d.F16 = dupload(own, to_half_scaled(s.Fblk, s.nF, s.N, 8 * s.N, d.Np, s.n, sc), st);
        d.F16s = dupload(own, sc, st);
      }
      d.W16 = dupload(own, to_half_scaled(s.Wblk, s.nW, s.N, 2 * s.N, d.Np, s.n, sc), st);
      d.W16s = dupload(own, sc, st);
      d.M16 = dupload(own, to_half_scaled(s.Mblk, s.nM, s.N, 4 * s.N, d.Np, s.n, sc), st);
      d.M16s = dupload(own, sc, st);
    }
    d.w_id = dupload(own, s.w_id, st);
    d.w_win = dupload(own, s.w_win, st);
    d.M64 = dupload_cm(own, s.Mblk, s.nM, s.N, 4 * s.N, d.Np, st);
    d.M32 = dconvert32(own, d.M64, (size_t)s.nM * 4 * s.N * d.Np, st);
    d.m_id = dupload(own, s.m_id, st);
    d.m_win = dupload(own, s.m_win, st);
    d.m_K = dupload(own, s.m_K, st);
    d.sz_col = dupload(own, s.sz_col, st);
    d.SZh = dupload(own, s.SZh, st);
    d.Gc = dupload(own, to_colmajor<double>(s.Gc, 1, s.d, s.d), st);
    d.GcR = s.zm == 1 ? dupload(own, s.Gc, st) : nullptr;
    d.uS = s.singular ? dupload(own, s.uS, st) : nullptr;
    d.uL = s.singular ? dupload(own, s.uL, st) : nullptr;
    // element inverses (class, element) and capacitance inverses (class),
    // column-major: each class's row-major tables go up as they are and the
    // device transposes them
    const int ncl = (int)s.classes.size(), n2 = s.n2, nq = 2 * s.n * (s.mz - 1);
    std::vector<std::pair<const double *, size_t>> dparts, kparts;
    std::vector<double> beta;
    for (const StripClass &c : s.classes) {
      dparts.emplace_back(c.Dinv.data(), (size_t)s.mz * n2 * n2);
      if (nq > 0) kparts.emplace_back(c.Kinv.data(), (size_t)nq * nq);
      beta.insert(beta.end(), c.betaW.begin(), c.betaW.end());
      beta.insert(beta.end(), c.betaE.begin(), c.betaE.end());
    }
    d.Dinv = dupload_cm(own, dparts, ncl * s.mz, n2, n2, n2, st);
    d.Kinv = nq > 0 ? dupload_cm(own, kparts, ncl, nq, nq, nq, st) : dalloc<double>(own, 1);
    d.beta = dupload(own, beta, st);
    d.lo = dupload(own, s.lo, st);
    d.up = dupload(own, s.up, st);
    d.strip_class = dupload(own, s.strip_class, st);
    H->h_sys.push_back(d);
  }
  H->d_sys = dupload(own, H->h_sys, st);
  std::vector<HWork> wS1, wM1;
  std::vector<int2> wh, wx, wr, ws;
  int64_t f_off = 0, g_off = 0, x_off = 0, v_off = 0, part_off = 0, pr_off = 0, hs_off = 0, c_off = 0,
          st_off = 0, rr_off = 0, lam_off = 0;
  for (int si = 0; si < (int)H->sys.size(); ++si) {
    const System &s = H->sys[si];
    const int nq = 2 * s.n * (s.mz - 1);
    for (int q = 0; q < H->nrhs; ++q) {
      InstDev I{};
      const int inst = (int)H->h_ins.size();
      I.sys = si; I.rhs = q;
      I.nchunk_x = (int)((s.kS + kChunk - 1) / kChunk);
      I.nchunk_r = (int)((s.r + kChunk - 1) / kChunk);
      I.f_off = f_off; I.g_off = g_off; I.x_off = x_off; I.v_off = v_off;
      I.part_off = part_off; I.pr_off = pr_off; I.hs_off = hs_off; I.c_off = c_off;
      I.st_off = st_off; I.rr_off = rr_off; I.lam_off = lam_off;
      I.seg_first = inst; I.seg_count = 1;
      if (H->one_krylov) {   // the leader's GMRES scalars serve every instance
        I.seg_first = 0;
        I.st_off = 0;
        I.rr_off = 0;
      }
      f_off += s.r; g_off += 2LL * s.n * (s.mx + s.mz); x_off += s.kS; v_off += (int64_t)(maxit + 1) * s.kS;
      part_off += (int64_t)(maxit + 1) * I.nchunk_x + 2; pr_off += 2LL * I.nchunk_r;
      hs_off += (int64_t)s.nh * (s.zm > 1 ? s.zm : (s.N + 15) / 16); c_off += s.d;
      st_off += maxit + 1; rr_off += (int64_t)maxit * maxit; lam_off += (int64_t)s.mx * nq;
      // Halves of a system whose strips share blocks go through the MFMA GEMM
      // (items built below); a system with no sharing streams every half.
      {
        std::vector<HWork> tmp;
        if (!shares_blocks(s.w_id)) group_halves(inst, s.w_id, 1, tmp);
        H->S1_start.push_back((int)wS1.size());
        wS1.insert(wS1.end(), tmp.begin(), tmp.end());
        H->S1_cnt.push_back((int)wS1.size() - H->S1_start.back());
        tmp.clear();
        if (!shares_blocks(s.m_id)) group_halves(inst, s.m_id, 1, tmp);
        H->M1_start.push_back((int)wM1.size());
        wM1.insert(wM1.end(), tmp.begin(), tmp.end());
        H->M1_cnt.push_back((int)wM1.size() - H->M1_start.back());
      }
      H->h_start.push_back((int)wh.size());
      for (int h = 0; h < s.nh; ++h) wh.push_back(make_int2(inst, h));
      H->s_start.push_back((int)ws.size());
      for (int j = 0; j < s.mx; ++j) ws.push_back(make_int2(inst, j));
      H->x_start.push_back((int)wx.size());
      for (int c = 0; c < I.nchunk_x; ++c) wx.push_back(make_int2(inst, c));
      H->r_start.push_back((int)wr.size());
      for (int c = 0; c < I.nchunk_r; ++c) wr.push_back(make_int2(inst, c));
      H->h_ins.push_back(I);
    }
  }
  H->ninst = (int)H->h_ins.size();
  H->tot_r = f_off; H->tot_x = x_off; H->tot_g = g_off;
  if (H->one_krylov)
    for (InstDev &I : H->h_ins) I.seg_count = H->ninst;
  // Element-interior GEMM items: per (system, strip class, distinct element
  // inverse) for the element inverses, per (system, strip class) for the
  // capacitance inverse; the columns are the (instance, strip, element)
  // vectors that the block multiplies.
  {
    std::vector<CGItem> all[3][2], one[3][2];
    std::vector<CGCol> cols;
    // chunks of 64 columns; a class (or remainder) of at most 16 columns
    // goes to the narrow list
    auto emit = [&](const double *A, int R, int K, int lda, int ksplit, int agap, const std::vector<CGCol> &cv,
                    std::vector<CGItem> *out, bool narrow) {
      for (size_t a = 0; a < cv.size();) {
        const size_t left = cv.size() - a;
        const int w = left <= 16 || narrow ? 0 : 1;
        CGItem it{};
        it.A = A; it.R = R; it.K = K; it.lda = lda; it.ksplit = ksplit; it.agap = agap;
        it.cstart = (int)cols.size();
        it.ccount = (int)std::min<size_t>(w ? kColVecs : 16, left);
        cols.insert(cols.end(), cv.begin() + a, cv.begin() + a + it.ccount);
        out[w].push_back(it);
        a += it.ccount;
      }
    };
    // items of system si over the instances [i0, i1)
    // (narrow: every item of at most 16 columns, into out[kind][0])
    auto items = [&](int si, int i0, int i1, std::vector<CGItem> (*out)[2], bool narrow = false) {
      const System &s = H->sys[si];
      const SysDev &d = H->h_sys[si];
      const int n = s.n, n2 = s.n2, mz = s.mz, nq = 2 * s.n * (s.mz - 1);
      for (int c = 0; c < (int)s.classes.size(); ++c) {
        std::vector<int> strips;
        for (int j = 0; j < s.mx; ++j)
          if (s.strip_class[j] == c) strips.push_back(j);
        // Elements of the class with bitwise equal inverses (on a uniform
        // z-grid every element between the two physical edges) share one
        // item list: one stored block multiplies the columns of all of them.
        const double *Dh = s.classes[c].Dinv.data();
        const size_t bsz = (size_t)n2 * n2;
        std::vector<int> rep(mz);
        for (int e = 0; e < mz; ++e) {
          rep[e] = e;
          for (int f = 0; f < e; ++f)
            if (rep[f] == f && !std::memcmp(Dh + f * bsz, Dh + e * bsz, sizeof(double) * bsz)) {
              rep[e] = f;
              break;
            }
        }
        for (int e0 = 0; e0 < mz; ++e0) {
          if (rep[e0] != e0) continue;
          const double *A = d.Dinv + ((size_t)c * mz + e0) * bsz;
          std::vector<CGCol> cs, cc;
          for (int i = i0; i < i1; ++i) {
            const InstDev &I = H->h_ins[i];
            for (int e = e0; e < mz; ++e) {
              if (rep[e] != e0) continue;
              for (int j : strips) {
                const int64_t off = I.f_off + ((int64_t)j * mz + e) * n2;
                cs.push_back(CGCol{off, -1, off});
                const int64_t q0 = I.lam_off + (int64_t)j * nq;
                cc.push_back(CGCol{e >= 1 ? q0 + (int64_t)(2 * (e - 1)) * n : -1,
                                   e + 1 < mz ? q0 + (int64_t)(2 * e + 1) * n : -1, off});
              }
            }
          }
          emit(A, n2, n2, n2, n2, 0, cs, out[0], narrow);
          if (nq > 0) emit(A, n2, 2 * n, n2, n, n2 - 2 * n, cc, out[2], narrow);
        }
        if (nq > 0) {
          std::vector<CGCol> cq;
          for (int i = i0; i < i1; ++i)
            for (int j : strips) {
              const int64_t q0 = H->h_ins[i].lam_off + (int64_t)j * nq;
              cq.push_back(CGCol{q0, -1, q0});
            }
          emit(d.Kinv + (size_t)c * nq * nq, nq, nq, nq, nq, 0, cq, out[1], narrow);
        }
      }
    };
    for (int si = 0; si < (int)H->sys.size(); ++si) items(si, si * H->nrhs, (si + 1) * H->nrhs, all);
    std::vector<CGItem> alt[3][2];
    for (int si = 0; si < (int)H->sys.size(); ++si) items(si, si * H->nrhs, (si + 1) * H->nrhs, alt, true);
    // Where a product has wide items and only a few narrow ones (a launch of
    // fewer than 1024 row tiles, bound by latency), the 64-column kernel takes
    // the narrow ones too: one launch instead of two.  Many narrow items stay
    // apart, as 16-column tiles.
    const int64_t rt16 = (std::max(H->n2_max, H->nq_max) + 15) / 16;
    for (int k = 0; k < 3; ++k)
      if (!all[k][0].empty() && !all[k][1].empty() && (int64_t)all[k][0].size() * rt16 < 1024) {
        all[k][1].insert(all[k][1].end(), all[k][0].begin(), all[k][0].end());
        all[k][0].clear();
      }
    for (int i = 0; i < H->ninst; ++i) {
      int st0[3][2];
      for (int k = 0; k < 3; ++k)
        for (int w = 0; w < 2; ++w) st0[k][w] = (int)one[k][w].size();
      items(H->h_ins[i].sys, i, i + 1, one);
      for (int k = 0; k < 3; ++k)
        for (int w = 0; w < 2; ++w) {
          H->cg_start[k][w].push_back(st0[k][w]);
          H->cg_cnt[k][w].push_back((int)one[k][w].size() - st0[k][w]);
        }
    }
    for (int k = 0; k < 3; ++k)
      for (int w = 0; w < 2; ++w) {
        H->cg_all[k][w] = dupload(own, all[k][w], st); H->n_cg_all[k][w] = (int)all[k][w].size();
        H->cg_one[k][w] = dupload(own, one[k][w], st);
        std::vector<uintptr_t> key;
        std::vector<int> tiles;
        for (const CGItem &it : all[k][w]) {
          key.push_back((uintptr_t)it.A);
          tiles.push_back((it.R + 63) / 64);
        }
        std::vector<int2> u = xcd_units(key, tiles);
        H->cg_units[k][w] = dupload(own, u, st);
        H->n_cg_units[k][w] = (int)u.size();
      }
    for (int k = 0; k < 3; ++k) {
      if (all[k][1].empty()) continue;   // no wide item: the 16-column list is list 0
      H->cg_alt[k] = dupload(own, alt[k][0], st);
      H->n_cg_alt[k] = (int)alt[k][0].size();
      std::vector<uintptr_t> key;
      std::vector<int> tiles;
      for (const CGItem &it : alt[k][0]) {
        key.push_back((uintptr_t)it.A);
        tiles.push_back((it.R + 63) / 64);
      }
      std::vector<int2> u = xcd_units(key, tiles);
      H->cg_alt_units[k] = dupload(own, u, st);
      H->n_cg_alt_units[k] = (int)u.size();
    }
    H->cg_cols = dupload(own, cols, st);
  }
  // MFMA GEMM items for systems with shared blocks.
  {
    std::vector<GWork> ga[3], go[3], ga16[2];
    std::vector<GVec> gv;
    // items of one stored block over its windows, kGemmVecs windows each
    // (half as many for the fused S M^-1 blocks)
    auto emit = [&](int si, int op, int id, const std::vector<int2> &vecs, std::vector<GWork> &out, int cap = 0) {
      const System &s = H->sys[si];
      const SysDev &d = H->h_sys[si];
      const int N = s.N, slots = (N + 15) / 16;
      const int h0 = vecs[0].y;
      const int K = op == 0 ? 2 * N : (op == 1 ? s.m_K[h0] : s.f_K[h0]);
      const int cols = op == 0 ? 2 * N : (op == 1 ? 4 * N : 8 * N);
      const size_t boff = (size_t)id * cols * d.Np;
      for (size_t a = 0; a < vecs.size();) {
        GWork w{};
        w.blk64 = (op == 0 ? d.W64 : op == 1 ? d.M64 : d.F64) + boff;
        w.blk32 = (op == 0 ? d.W32 : op == 1 ? d.M32 : d.F32) + boff;
        if (H->op16) {
          w.blk16 = (op == 0 ? d.W16 : op == 1 ? d.M16 : d.F16) + boff;
          w.sc16 = (op == 0 ? d.W16s : op == 1 ? d.M16s : d.F16s) + (size_t)id * s.mz;
        }
        w.n = s.n;
        w.N = N; w.Np = d.Np; w.K = K; w.kS = s.kS; w.ident = op == 0 ? 1 : 0;
        w.vstart = (int)gv.size();
        // S M^-1 blocks are up to 4x wider than S blocks: items of 16
        // windows give twice the workgroups at half the columns each.
        const size_t width = cap ? cap : op == 2 ? kGemmVecs / 2 : kGemmVecs;
        w.vcount = (int)std::min<size_t>(width, vecs.size() - a);
        for (int q = 0; q < w.vcount; ++q) {
          const int inst = vecs[a + q].x, h = vecs[a + q].y;
          const InstDev &I = H->h_ins[inst];
          GVec e{};
          e.x0 = I.x_off; e.xv = I.v_off;
          e.win = (int64_t)(op == 0 ? s.w_win[h] : op == 1 ? s.m_win[h] : s.f_win[h]) * N;
          e.xh = (int64_t)h * N;
          e.y = I.x_off + (int64_t)h * N;
          e.inst = inst;
          e.hs = (int)(I.hs_off + h);
          e.hn = s.nh;
          e.st_off = (int)I.st_off;
          gv.push_back(e);
        }
        out.push_back(w);
        a += w.vcount;
      }
    };
    H->fused = true;
    for (int si = 0; si < (int)H->sys.size(); ++si) {
      const System &s = H->sys[si];
      if (s.nF == 0) H->fused = false;
      for (int op = 0; op < 3; ++op) {
        const std::vector<int> &ids = op == 0 ? s.w_id : op == 1 ? s.m_id : s.f_id;
        if (op < 2 ? !shares_blocks(ids) : s.nF == 0) continue;
        std::map<int, std::vector<int2>> all;
        std::vector<std::map<int, std::vector<int2>>> per(H->nrhs);
        for (int q = 0; q < H->nrhs; ++q)
          for (int h = 0; h < s.nh; ++h) {
            const int2 e = make_int2(si * H->nrhs + q, h);
            all[ids[h]].push_back(e);
            per[q][ids[h]].push_back(e);
          }
        for (auto &kv : all) {
          emit(si, op, kv.first, kv.second, ga[op]);
          if (op < 2) emit(si, op, kv.first, kv.second, ga16[op], 16);
        }
        for (int q = 0; q < H->nrhs; ++q) {
          const int inst = si * H->nrhs + q;
          std::vector<int> &st_v = H->g_start[op], &ct_v = H->g_cnt[op];
          if ((int)st_v.size() <= inst) { st_v.resize(inst + 1, 0); ct_v.resize(inst + 1, 0); }
          st_v[inst] = (int)go[op].size();
          for (auto &kv : per[q]) emit(si, op, kv.first, kv.second, go[op]);
          ct_v[inst] = (int)go[op].size() - st_v[inst];
        }
      }
    }
    auto make_list = [&](const std::vector<GWork> &items) {
      GList L;
      for (const GWork &w : items) L.maxv = std::max(L.maxv, w.vcount);
      L.w = dupload(own, items, st);
      L.n = (int)items.size();
      std::vector<uintptr_t> key;
      std::vector<int> tiles;
      for (const GWork &w : items) {
        key.push_back((uintptr_t)w.blk64);
        tiles.push_back((w.Np + 63) / 64);
      }
      std::vector<int2> u = xcd_units(key, tiles);
      L.u = dupload(own, u, st);
      L.nu = (int)u.size();
      // 128-row tiles, each costed by its MFMA work (K x live 16-row groups
      // x 16-window column tiles) plus one unit per K for the block's reads
      std::vector<int> t128;
      std::vector<std::vector<int64_t>> cost;
      for (const GWork &w : items) {
        const int nt = (w.Np + 127) / 128;
        t128.push_back(nt);
        std::vector<int64_t> cr(nt);
        for (int r = 0; r < nt; ++r) {
          const int lw = (std::min(w.N, 128 * (r + 1)) - 128 * r + 15) / 16;
          cr[r] = (int64_t)w.K * ((int64_t)std::max(lw, 0) * ((w.vcount + 15) / 16) + 1);
        }
        cost.push_back(cr);
      }
      std::vector<int2> u2 = xcd_units(key, t128, &cost);
      L.u128 = dupload(own, u2, st);
      L.nu128 = (int)u2.size();
      return L;
    };
    for (int op = 0; op < 3; ++op) {
      H->g_start[op].resize(H->ninst, 0); H->g_cnt[op].resize(H->ninst, 0);
      H->g_one[op] = dupload(own, go[op], st);
      H->gl[op][0] = make_list(ga[op]);
      if (op < 2 && H->gl[op][0].maxv > 16) H->gl[op][1] = make_list(ga16[op]);
    }
    // B A^-1 per strip class, for the Schur right-hand side of every
    // system in one GEMM over the strips (grids whose strips share classes:
    // then the blocks are few and small, and the GEMM replaces the element
    // solves of A^-1 and the B row functionals).
    H->use_ba = H->fused;
    if (H->use_ba) {
      std::vector<GWork> ba, ba16;
      for (int si = 0; si < (int)H->sys.size(); ++si) {
        const System &s = H->sys[si];
        const SysDev &d = H->h_sys[si];
        const int N = s.N, K = s.mz * s.n2, ncl = (int)s.classes.size();
        std::vector<std::vector<double>> blocks(ncl);
        parallel_for(ncl, 0, [&](int c) { class_rhs_blocks(s, s.classes[c], blocks[c]); });
        std::vector<std::pair<const double *, size_t>> parts;
        for (auto &b : blocks) parts.emplace_back(b.data(), b.size());
        const double *dba = dupload_cm(own, parts, 2 * ncl, N, K, d.Np, st);
        std::map<int, std::vector<int2>> byblk;   // block id -> (instance, strip * 2 + side)
        for (int q = 0; q < H->nrhs; ++q)
          for (int j = 0; j < s.mx; ++j) {
            const int inst = si * H->nrhs + q, cls = s.strip_class[j];
            if (j >= 1) byblk[2 * cls].push_back(make_int2(inst, 2 * j));           // west rows -> half 2 (j - 1)
            if (j + 1 < s.mx) byblk[2 * cls + 1].push_back(make_int2(inst, 2 * j + 1));   // east rows -> half 2 j + 1
          }
        // items of up to kGemmVecs windows, and of up to 16 (the narrow
        // schedules: one column tile, or the whole K range in flight)
        for (int cap : {kGemmVecs, 16}) {
          for (auto &kv : byblk) {
            const std::vector<int2> &vecs = kv.second;
            for (size_t a = 0; a < vecs.size();) {
              GWork w{};
              w.blk64 = dba + (size_t)kv.first * K * d.Np;
              w.n = s.n;
              w.N = N; w.Np = d.Np; w.K = K; w.kS = s.r; w.ident = 0;
              w.vstart = (int)gv.size();
              w.vcount = (int)std::min<size_t>(cap, vecs.size() - a);
              for (int qq = 0; qq < w.vcount; ++qq) {
                const int inst = vecs[a + qq].x, j = vecs[a + qq].y / 2, side = vecs[a + qq].y % 2;
                const int h = side == 0 ? 2 * (j - 1) : 2 * j + 1;
                const InstDev &I = H->h_ins[inst];
                GVec e{};
                e.x0 = I.f_off;
                e.win = (int64_t)j * K;
                e.y = I.x_off + (int64_t)h * N;
                e.inst = inst;
                e.hs = (int)(I.hs_off + h);
                e.hn = s.nh;
                e.st_off = (int)I.st_off;
                gv.push_back(e);
              }
              (cap == 16 ? ba16 : ba).push_back(w);
              a += w.vcount;
            }
          }
        }
      }
      H->g_bal[0] = dupload(own, ba, st);
      H->n_bal[0] = (int)ba.size();
      for (const GWork &w : ba) H->bal_maxv[0] = std::max(H->bal_maxv[0], w.vcount);
      if (H->bal_maxv[0] > 16) {   // else the two lists are the same
        H->g_bal[1] = dupload(own, ba16, st);
        H->n_bal[1] = (int)ba16.size();
        H->bal_maxv[1] = 16;
      }
    }
    H->g_vec = dupload(own, gv, st);
  }
  H->d_ins = dupload(own, H->h_ins, st);
  H->w_S1 = dupload(own, wS1, st); H->n_S1 = (int)wS1.size();
  H->w_M1 = dupload(own, wM1, st); H->n_M1 = (int)wM1.size();
  H->w_h = dupload(own, wh, st); H->n_h = (int)wh.size();
  H->w_x = dupload(own, wx, st); H->n_x = (int)wx.size();
  H->reg_basis = H->n_x <= kRegBasisChunks;
  H->w_r = dupload(own, wr, st); H->n_r = (int)wr.size();
  H->w_s = dupload(own, ws, st); H->n_s = (int)ws.size();
  H->F = dalloc<double>(own, f_off); H->v = dalloc<double>(own, f_off); H->Rr = dalloc<double>(own, f_off);
  H->bS = dalloc<double>(own, x_off); H->xS = dalloc<double>(own, x_off); H->rb = dalloc<double>(own, x_off);
  H->z64 = dalloc<double>(own, x_off); H->y64 = dalloc<double>(own, x_off); H->t64 = dalloc<double>(own, x_off);
  H->z32 = dalloc<float>(own, x_off); H->y32 = dalloc<float>(own, x_off); H->t32 = dalloc<float>(own, x_off);
  if (H->precision == SMPM_FP64) H->V64 = dalloc<double>(own, v_off);
  else H->V32 = dalloc<float>(own, v_off);
  H->part1 = dalloc<double>(own, part_off); H->part2 = dalloc<double>(own, part_off); H->partn = dalloc<double>(own, part_off);
  H->arrive = dalloc<int>(own, H->ninst);
  HIPCHECK(hipMemsetAsync(H->arrive, 0, sizeof(int) * H->ninst, st));
  H->pr = dalloc<double>(own, pr_off); H->hs = dalloc<double>(own, hs_off);
  H->cv = dalloc<double>(own, c_off); H->tb = dalloc<double>(own, c_off);
  H->scale = dalloc<double>(own, st_off); H->cs = dalloc<double>(own, st_off); H->sn = dalloc<double>(own, st_off);
  H->g = dalloc<double>(own, st_off); H->ycoef = dalloc<double>(own, st_off); H->Rm = dalloc<double>(own, rr_off);
  H->lam = dalloc<double>(own, lam_off); H->qb = dalloc<double>(own, lam_off);
  {
    static_assert(sizeof(GState) % sizeof(double) == 0, "GState packs into doubles");
    const size_t gs_d = sizeof(GState) / sizeof(double) * H->ninst;
    double *rep = dalloc<double>(own, gs_d + 5 * (size_t)H->ninst);
    H->gs = reinterpret_cast<GState *>(rep);
    H->pairs = rep + gs_d;
    H->defect = H->pairs + 2 * H->ninst;
    H->nb2 = H->defect + H->ninst;
    H->rep_bytes = sizeof(double) * (gs_d + 5 * (size_t)H->ninst);
    HIPCHECK(hipHostMalloc((void **)&H->h_rep, H->rep_bytes, hipHostMallocDefault));
  }
  if (H->one_krylov) {
    H->sr1 = dalloc<double>(own, st_off); H->sr2 = dalloc<double>(own, st_off); H->srn = dalloc<double>(own, st_off);
  }
  HIPCHECK(hipHostMalloc((void **)&H->h_gs, sizeof(GState) * H->ninst, hipHostMallocDefault));
  HIPCHECK(hipHostMalloc((void **)&H->h_pairs, sizeof(double) * 2 * H->ninst, hipHostMallocDefault));
  HIPCHECK(hipHostMalloc((void **)&H->h_defect, sizeof(double) * H->ninst, hipHostMallocDefault));
  HIPCHECK(hipHostMalloc((void **)&H->h_gs_hist, sizeof(GState) * H->ninst * (H->max_sweeps + 1),
                         hipHostMallocDefault));
  HIPCHECK(hipHostMalloc((void **)&H->h_nb, sizeof(double) * 2 * H->ninst, hipHostMallocDefault));
  HIPCHECK(hipStreamCreateWithFlags(&H->ws, hipStreamNonBlocking));
  HIPCHECK(hipEventCreateWithFlags(&H->ev_in, hipEventDisableTiming));
  HIPCHECK(hipEventCreateWithFlags(&H->ev_out, hipEventDisableTiming));
  HIPCHECK(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------------
// Launch helpers.  `inst` >= 0 restricts a launch to one instance's items.

// GEMM schedules of the shared-block matvec (see the kernels): split K over
// 16 or 8 waves per 16-row tile, or the LDS-staged 64-row tile in XCD-aware
// or plain order, staging 32 K-values per chunk (or 64: kThrXcd64,
// kThrPlain64, twice the work between the chunk barriers).
// kSplit8Deep / kSplit16Deep: split K over 8 or 16 waves with 24 or 18
// K-steps of loads in flight per wave, for lists whose items hold at most
// 16 windows (others run kSplit8 under these ids).  kTile128: the staged
// tile with 128 rows (8 waves), so a window is staged once for up to 128
// rows; kTile64K4 / kTile128K2: 64- or 128-row tiles whose 16 waves also
// split K four or two ways (shorter MFMA chains per wave).  The staged
// schedules hold 16 windows per item column group where the items do.
// kTile128Xcd: the 128-row tile over a cost-ordered XCD-aware unit list
// (each XCD's tiles costliest first); kTile128Xcd64 the same staging 64
// K-values per chunk.
enum GemmSched {
  kSplit16 = 0, kSplit8 = 1, kThrXcd = 2, kThrPlain = 3, kThrXcd64 = 4, kThrPlain64 = 5, kSplit8Deep = 6,
  kSplit16Deep = 7, kTile128 = 8, kTile64K4 = 9, kTile128K2 = 10, kTile128Xcd = 11, kTile128Xcd64 = 12,
  kNumSched = 13
};

// Default schedule when none was tuned (per-instance lists): by launch size.
int gemm_default(int count, int rt16) {
  if ((int64_t)count * rt16 < 512) return kSplit16;
  if ((int64_t)count * rt16 < 2048) return kSplit8;
  return kThrPlain;
}

template <typename TS, typename TO, typename TX, typename TY>
void gemm_launch(smpm_handle *H, int sched, const GWork *w, int count, const int2 *units, int nunits, const TX *x,
                 int vslot, const double *scale, TY *y, double *hsum, const GState *gs, hipStream_t st,
                 bool narrow, const int2 *units128 = nullptr, int nunits128 = 0) {
  const int rt16 = (H->Nmax + 15) / 16;
  if ((sched == kSplit8Deep || sched == kSplit16Deep) && !narrow) sched = kSplit8;
  auto tiles = [&](int rows) { return (unsigned)((H->Nmax + rows - 1) / rows); };
  if ((sched == kTile128Xcd || sched == kTile128Xcd64) && !units128) sched = kTile128;
  switch (sched) {
    case kTile128Xcd64:
      if (narrow)
        hipLaunchKernelGGL((k_half_gemm_t<TS, TO, TX, TY, 1, 64, 8, 1>), dim3(nunits128), dim3(512), 0, st, w, units128,
                           H->g_vec, x, vslot, scale, y, hsum, gs);
      else
        hipLaunchKernelGGL((k_half_gemm_t<TS, TO, TX, TY, 2, 64, 8, 1>), dim3(nunits128), dim3(512), 0, st, w, units128,
                           H->g_vec, x, vslot, scale, y, hsum, gs);
      break;
    case kTile128Xcd:
      if (narrow)
        hipLaunchKernelGGL((k_half_gemm_t<TS, TO, TX, TY, 1, 32, 8, 1>), dim3(nunits128), dim3(512), 0, st, w, units128,
                           H->g_vec, x, vslot, scale, y, hsum, gs);
      else
        hipLaunchKernelGGL((k_half_gemm_t<TS, TO, TX, TY, 2, 32, 8, 1>), dim3(nunits128), dim3(512), 0, st, w, units128,
                           H->g_vec, x, vslot, scale, y, hsum, gs);
      break;
    case kTile128:
      if (narrow)
        hipLaunchKernelGGL((k_half_gemm_t<TS, TO, TX, TY, 1, 32, 8, 1>), dim3(count, tiles(128)), dim3(512), 0, st, w,
                           (const int2 *)nullptr, H->g_vec, x, vslot, scale, y, hsum, gs);
      else
        hipLaunchKernelGGL((k_half_gemm_t<TS, TO, TX, TY, 2, 32, 8, 1>), dim3(count, tiles(128)), dim3(512), 0, st, w,
                           (const int2 *)nullptr, H->g_vec, x, vslot, scale, y, hsum, gs);
      break;
    case kTile64K4:
      if (narrow)
        hipLaunchKernelGGL((k_half_gemm_t<TS, TO, TX, TY, 1, 32, 4, 4>), dim3(count, tiles(64)), dim3(1024), 0, st, w,
                           (const int2 *)nullptr, H->g_vec, x, vslot, scale, y, hsum, gs);
      else
        hipLaunchKernelGGL((k_half_gemm_t<TS, TO, TX, TY, 2, 32, 4, 4>), dim3(count, tiles(64)), dim3(1024), 0, st, w,
                           (const int2 *)nullptr, H->g_vec, x, vslot, scale, y, hsum, gs);
      break;
    case kTile128K2:
      if (narrow)
        hipLaunchKernelGGL((k_half_gemm_t<TS, TO, TX, TY, 1, 32, 8, 2>), dim3(count, tiles(128)), dim3(1024), 0, st, w,
                           (const int2 *)nullptr, H->g_vec, x, vslot, scale, y, hsum, gs);
      else
        hipLaunchKernelGGL((k_half_gemm_t<TS, TO, TX, TY, 2, 32, 8, 2>), dim3(count, tiles(128)), dim3(1024), 0, st, w,
                           (const int2 *)nullptr, H->g_vec, x, vslot, scale, y, hsum, gs);
      break;
    case kSplit8Deep:
      hipLaunchKernelGGL((k_half_gemm<TS, TO, TX, TY, 8, 24, false>), dim3(count, rt16), dim3(512), 0, st, w, H->g_vec,
                         x, vslot, scale, y, hsum, gs);
      break;
    case kSplit16Deep:
      hipLaunchKernelGGL((k_half_gemm<TS, TO, TX, TY, 16, 18, false>), dim3(count, rt16), dim3(1024), 0, st, w,
                         H->g_vec, x, vslot, scale, y, hsum, gs);
      break;
    case kSplit16:
      hipLaunchKernelGGL((k_half_gemm<TS, TO, TX, TY, 16>), dim3(count, rt16), dim3(1024), 0, st, w, H->g_vec, x, vslot,
                         scale, y, hsum, gs);
      break;
    case kSplit8:
      hipLaunchKernelGGL((k_half_gemm<TS, TO, TX, TY, 8>), dim3(count, rt16), dim3(512), 0, st, w, H->g_vec, x, vslot,
                         scale, y, hsum, gs);
      break;
    case kThrXcd64:
      if (units) {
        hipLaunchKernelGGL((k_half_gemm_t<TS, TO, TX, TY, 2, 64>), dim3(nunits), dim3(256), 0, st, w, units, H->g_vec, x,
                           vslot, scale, y, hsum, gs);
        break;
      }
      [[fallthrough]];
    case kThrPlain64:
      hipLaunchKernelGGL((k_half_gemm_t<TS, TO, TX, TY, 2, 64>), dim3(count, (H->Nmax + 63) / 64), dim3(256), 0, st, w,
                         (const int2 *)nullptr, H->g_vec, x, vslot, scale, y, hsum, gs);
      break;
    case kThrXcd:
      if (units) {
        hipLaunchKernelGGL((k_half_gemm_t<TS, TO, TX, TY, 2, 32>), dim3(nunits), dim3(256), 0, st, w, units, H->g_vec, x,
                           vslot, scale, y, hsum, gs);
        break;
      }
      [[fallthrough]];
    default:
      hipLaunchKernelGGL((k_half_gemm_t<TS, TO, TX, TY, 2, 32>), dim3(count, (H->Nmax + 63) / 64), dim3(256), 0, st, w,
                         (const int2 *)nullptr, H->g_vec, x, vslot, scale, y, hsum, gs);
  }
}

// A batched list under schedule `sched`.
template <typename TS, typename TO, typename TX, typename TY>
void gemm_list(smpm_handle *H, int sched, const GList &L, const TX *x, int vslot, const double *scale, TY *y,
               double *hsum, const GState *gs, hipStream_t st) {
  gemm_launch<TS, TO, TX, TY>(H, sched, L.w, L.n, L.u, L.nu, x, vslot, scale, y, hsum, gs, st, L.maxv <= 16, L.u128,
                              L.nu128);
}

template <typename TS, typename TO, typename TX, typename TY>
void gemv_ts(smpm_handle *H, int op, const TX *x, int vslot, const double *scale, TY *y, double *hsum,
             const GState *gs, hipStream_t st, int inst) {
  const int Kmax = (op == 0 ? 2 : 4) * H->Nmax;
  // halves with a shared block: MFMA GEMM over the windows that share it
  {
    const int prec = sizeof(TS) == 8 ? 0 : (sizeof(TS) == 4 ? 1 : 2);
    if (inst < 0) {
      if (H->gl[op][0].n > 0)
        gemm_list<TS, TO, TX, TY>(H, H->sched[op][prec], H->gl[op][H->g_list[op][prec]], x, vslot, scale, y, hsum, gs,
                                  st);
    } else if (H->g_cnt[op][inst] > 0) {
      const int count = H->g_cnt[op][inst];
      gemm_launch<TS, TO, TX, TY>(H, gemm_default(count, (H->Nmax + 15) / 16), H->g_one[op] + H->g_start[op][inst],
                                  count, nullptr, 0, x, vslot, scale, y, hsum, gs, st, H->gl[op][0].maxv <= 16);
    }
  }
  // halves with their own block: streaming kernel (S or M^-1 only)
  if (op < 2) {
    const HWork *w = op == 0 ? H->w_S1 : H->w_M1;
    int count = op == 0 ? H->n_S1 : H->n_M1;
    if (inst >= 0) {
      w += op == 0 ? H->S1_start[inst] : H->M1_start[inst];
      count = op == 0 ? H->S1_cnt[inst] : H->M1_cnt[inst];
    }
    if (count > 0) {
      constexpr int TR = 64 * Vec16<TS>::R;
      const int tiles = (H->Nmax + TR - 1) / TR;
      const size_t shm = sizeof(double) * (Kmax + kWaves * TR);
      hipLaunchKernelGGL((k_half_gemv_stream<TS, TO, TX, TY, kWaves>), dim3(count, tiles), dim3(64 * kWaves), shm, st,
                         H->d_sys, H->d_ins, w, op, x, vslot, scale, y, hsum, gs);
    }
  }
}

// y = S x (op 0) or M^-1 x (op 1) for every instance (or one), arithmetic in
// TO; FP32 arithmetic reads the FP16 tables when h16 is set.
template <typename TO, typename TX, typename TY>
void gemv(smpm_handle *H, int op, const TX *x, int vslot, const double *scale, TY *y, double *hsum,
          const GState *gs, hipStream_t st, int inst = -1, bool h16 = false) {
  if constexpr (sizeof(TO) == 8) {
    gemv_ts<double, TO, TX, TY>(H, op, x, vslot, scale, y, hsum, gs, st, inst);
  } else {
    if (h16) gemv_ts<_Float16, TO, TX, TY>(H, op, x, vslot, scale, y, hsum, gs, st, inst);
    else gemv_ts<float, TO, TX, TY>(H, op, x, vslot, scale, y, hsum, gs, st, inst);
  }
}

// Element-interior GEMM schedules: split K (kSplit8) or the LDS-staged
// 64-row tile (kThrXcd with units, kThrPlain without), or the LDS-staged
// 32- or 16-row tile whose waves split K (kCol32, kCol16).  sched < 0: by size.
enum ColSched { kCol32 = 4, kCol16 = 5 };

template <int CT, int MODE, int RW>
void colgemm_t_launch(smpm_handle *H, const CGItem *items, int count, const int2 *units, int nunits,
                      const double *x, double *y, hipStream_t st, int rmax) {
  const dim3 grid = units ? dim3(nunits) : dim3(count, (rmax + 16 * RW - 1) / (16 * RW));
  hipLaunchKernelGGL((k_colgemm_t<CT, MODE, RW>), grid, dim3(256), 0, st, items, units, H->cg_cols, x, y);
}

template <int CT>
void colgemm_w(smpm_handle *H, const CGItem *items, int count, const int2 *units, int nunits, int mode,
               const double *x, double *y, hipStream_t st, int sched = -1) {
  if (count <= 0) return;
  const int rmax = std::max(H->n2_max, H->nq_max);
  const int rt16 = (rmax + 15) / 16;
  if (sched < 0) sched = (int64_t)count * rt16 < 1024 ? kSplit8 : kThrXcd;
  if (sched != kThrXcd) units = nullptr;
  if (sched == kSplit8 || sched == kSplit16) {     // split K for parallelism
    const dim3 grid(count, rt16);
    if (mode == 0) hipLaunchKernelGGL((k_colgemm<CT, 0>), grid, dim3(512), 0, st, items, H->cg_cols, x, y);
    else hipLaunchKernelGGL((k_colgemm<CT, 1>), grid, dim3(512), 0, st, items, H->cg_cols, x, y);
  } else if (sched == kCol16) {
    if (mode == 0) colgemm_t_launch<CT, 0, 1>(H, items, count, units, nunits, x, y, st, rmax);
    else colgemm_t_launch<CT, 1, 1>(H, items, count, units, nunits, x, y, st, rmax);
  } else if (sched == kCol32) {
    if (mode == 0) colgemm_t_launch<CT, 0, 2>(H, items, count, units, nunits, x, y, st, rmax);
    else colgemm_t_launch<CT, 1, 2>(H, items, count, units, nunits, x, y, st, rmax);
  } else {
    if (mode == 0) colgemm_t_launch<CT, 0, 4>(H, items, count, units, nunits, x, y, st, rmax);
    else colgemm_t_launch<CT, 1, 4>(H, items, count, units, nunits, x, y, st, rmax);
  }
}

// One element-interior product (kind 0, 1, 2) over all instances or one.
void colgemm(smpm_handle *H, int kind, int inst, int mode, const double *x, double *y, hipStream_t st) {
  if (inst < 0 && H->cg_alt_sched[kind] >= 0) {
    colgemm_w<1>(H, H->cg_alt[kind], H->n_cg_alt[kind], H->cg_alt_units[kind], H->n_cg_alt_units[kind], mode, x, y,
                 st, H->cg_alt_sched[kind]);
    return;
  }
  for (int w = 0; w < 2; ++w) {
    const CGItem *it = inst >= 0 ? H->cg_one[kind][w] + H->cg_start[kind][w][inst] : H->cg_all[kind][w];
    const int cnt = inst >= 0 ? H->cg_cnt[kind][w][inst] : H->n_cg_all[kind][w];
    const int2 *un = inst >= 0 ? nullptr : H->cg_units[kind][w];
    const int nun = inst >= 0 ? 0 : H->n_cg_units[kind][w];
    const int sc = inst >= 0 ? -1 : H->cg_sched[kind][w];
    if (w == 0) colgemm_w<1>(H, it, cnt, un, nun, mode, x, y, st, sc);
    else colgemm_w<kColVecs / 16>(H, it, cnt, un, nun, mode, x, y, st, sc);
  }
}

// dst = A(k)^-1 src (node space; src and dst must not overlap): element
// solves, the per-strip z-interface capacitance solve, element corrections.
void ainv(smpm_handle *H, const double *src, double *dst, hipStream_t st, int inst = -1) {
  colgemm(H, 0, inst, 0, src, dst, st);
  if (H->nq_max > 0) {
    const int2 *ws = H->w_s + (inst >= 0 ? H->s_start[inst] : 0);
    const int scount = inst >= 0 ? H->sys[H->h_ins[inst].sys].mx : H->n_s;
    hipLaunchKernelGGL(k_lambda, dim3(scount), dim3(kBlock), 0, st, H->d_sys, H->d_ins, ws, (const double *)dst, H->lam);
    colgemm(H, 1, inst, 0, H->lam, H->qb, st);
    colgemm(H, 2, inst, 1, H->qb, dst, st);
  }
}

// Setup-time autotuning of the GEMM schedules: every candidate schedule of
// every batched list is timed with HIP events on zeroed operands and the
// fastest is kept for the handle's lifetime.  The candidates are timed in
// two interleaved rounds of 1 warm-up and 6 timed launches each, and each
// keeps its best round: clock ramps and cold caches then hit every candidate
// alike, not the first one timed.  Without tuning, schedules follow the
// launch size.
// b_S = (B A^-1) F~ over the strips: item list `list` under schedule `sched`
void ba_launch(smpm_handle *H, int list, int sched, hipStream_t st) {
  gemm_launch<double, double, double, double>(H, sched, H->g_bal[list], H->n_bal[list], nullptr, 0,
                                              (const double *)H->F, 0, nullptr, H->bS, nullptr, nullptr, st,
                                              H->bal_maxv[list] <= 16);
}

template <typename F>
int fastest(hipStream_t st, hipEvent_t e0, hipEvent_t e1, int ncand, F &&fn) {
  std::vector<float> best(ncand, 1e30f);
  for (int round = 0; round < 2; ++round) {
    const float lead = *std::min_element(best.begin(), best.end());
    for (int c = 0; c < ncand; ++c) {
      // the second round re-times the first two candidates (timed while the
      // clocks ramp up) and every one within 1.3x of the first round's best
      if (round == 1 && c >= 2 && best[c] > 1.3f * lead) continue;
      fn(c);
      HIPCHECK(hipEventRecord(e0, st));
      for (int r = 0; r < 6; ++r) fn(c);
      HIPCHECK(hipEventRecord(e1, st));
      HIPCHECK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
      best[c] = std::min(best[c], ms);
    }
  }
  return (int)(std::min_element(best.begin(), best.end()) - best.begin());
}

void tune_schedules(smpm_handle *H, hipStream_t st) {
  const int rt16 = (H->Nmax + 15) / 16;
  for (int op = 0; op < 3; ++op)
    for (int pr = 0; pr < 3; ++pr) {
      H->sched[op][pr] = gemm_default(H->gl[op][0].n, rt16);
      H->g_list[op][pr] = 0;
    }
  for (int k = 0; k < 3; ++k)
    for (int w = 0; w < 2; ++w) H->cg_sched[k][w] = -1;
  for (int pr = 0; pr < 3; ++pr) H->use_fused[pr] = H->fused && (int64_t)H->gl[2][0].n * rt16 < 2048;
  H->ba_list = 0;
  H->ba_sched = gemm_default(H->n_bal[0], rt16);
  if (H->no_tune) return;
  const int rmax = std::max(H->n2_max, H->nq_max);
  for (int k = 0; k < 3; ++k)
    for (int w = 0; w < 2; ++w)
      H->cg_sched[k][w] = (int64_t)H->n_cg_all[k][w] * ((rmax + 15) / 16) < 1024 ? kSplit8 : kThrXcd;
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  try {
    HIPCHECK(hipMemsetAsync(H->t64, 0, sizeof(double) * H->tot_x, st));
    HIPCHECK(hipMemsetAsync(H->t32, 0, sizeof(float) * H->tot_x, st));
    HIPCHECK(hipMemsetAsync(H->F, 0, sizeof(double) * H->tot_r, st));
    HIPCHECK(hipMemsetAsync(H->v, 0, sizeof(double) * H->tot_r, st));
    if (H->nq_max > 0) {
      int64_t nl = 0;
      for (const InstDev &I : H->h_ins) nl = std::max<int64_t>(nl, I.lam_off + (int64_t)H->sys[I.sys].mx * H->h_sys[I.sys].nq);
      HIPCHECK(hipMemsetAsync(H->lam, 0, sizeof(double) * nl, st));
      HIPCHECK(hipMemsetAsync(H->qb, 0, sizeof(double) * nl, st));
    }
    // A batch's instances converge at different iterations, and most of a
    // solve's iterations run with a few instances left: there the workgroups
    // of converged instances exit at once and the cost is the live items'
    // latency, which ranks the schedules differently.  So on batches of 8
    // instances or more each candidate is timed twice per launch, with every
    // instance live and with the first tenth live (a GMRES state written
    // for the purpose and cleared again below).
    const bool mixed = H->ninst >= 8;
    if (mixed) {
      const int nlive = std::max(1, H->ninst / 10);
      for (int i = 0; i < H->ninst; ++i) {
        H->h_gs[i] = GState{};
        H->h_gs[i].active = i < nlive ? 1 : 0;
      }
      HIPCHECK(hipMemcpyAsync(H->gs, H->h_gs, sizeof(GState) * H->ninst, hipMemcpyHostToDevice, st));
    }
    // every schedule on each item list of the operator (the 16-window list
    // where there is one)
    for (int op = 0; op < 3; ++op) {
      if (H->gl[op][0].n == 0) continue;
      const int nl = H->gl[op][1].n ? 2 : 1;
      for (int pr = 0; pr < (H->op16 ? 3 : 2); ++pr) {
        const int c = fastest(st, e0, e1, nl * kNumSched, [&](int c) {
          const GList &L = H->gl[op][c / kNumSched];
          const int sc = c % kNumSched;
          for (int pass = 0; pass < (mixed ? 2 : 1); ++pass) {
            const GState *g = pass == 0 ? nullptr : H->gs;
            if (pr == 0)
              gemm_list<double, double, double, double>(H, sc, L, H->t64, 0, nullptr, H->y64,
                                                        op == 0 ? H->hs : nullptr, g, st);
            else if (pr == 1)
              gemm_list<float, float, float, float>(H, sc, L, H->t32, 0, nullptr, H->y32, op == 0 ? H->hs : nullptr,
                                                    g, st);
            else
              gemm_list<_Float16, float, float, float>(H, sc, L, H->t32, 0, nullptr, H->y32,
                                                       op == 0 ? H->hs : nullptr, g, st);
          }
        });
        H->g_list[op][pr] = c / kNumSched;
        H->sched[op][pr] = c % kNumSched;
      }
    }
    if (H->use_ba) {   // the Schur right-hand side GEMM (FP64 only), over either item list
      const int c = fastest(st, e0, e1, H->n_bal[1] ? 2 * kNumSched : kNumSched,
                            [&](int c) { ba_launch(H, c / kNumSched, c % kNumSched, st); });
      H->ba_list = c / kNumSched;
      H->ba_sched = c % kNumSched;
    }
    // one fused S M^-1 GEMM per iteration, or M^-1 then S: whichever is faster
    if (H->fused)
      for (int pr = 0; pr < (H->op16 ? 3 : 2); ++pr) {
        // full operator applications (shared-block GEMMs and streamed blocks)
        auto two = [&](int op, const void *x, void *y, const GState *g) {
          if (pr == 0)
            gemv<double, double, double>(H, op, (const double *)x, 0, nullptr, (double *)y, op != 1 ? H->hs : nullptr,
                                         g, st);
          else
            gemv<float, float, float>(H, op, (const float *)x, 0, nullptr, (float *)y, op != 1 ? H->hs : nullptr,
                                      g, st, -1, pr == 2);
        };
        const void *x = pr == 0 ? (const void *)H->t64 : (const void *)H->t32;
        void *z = pr == 0 ? (void *)H->z64 : (void *)H->z32;
        void *y = pr == 0 ? (void *)H->y64 : (void *)H->y32;
        H->use_fused[pr] = fastest(st, e0, e1, 2, [&](int c) {
          for (int pass = 0; pass < (mixed ? 2 : 1); ++pass) {   // all live, then the first tenth (above)
            const GState *g = pass == 0 ? nullptr : H->gs;
            if (c == 0) {
              two(2, x, y, g);
            } else {
              two(1, x, z, g);
              two(0, z, y, g);
            }
          }
        }) == 0;
      }
    if (mixed) HIPCHECK(hipMemsetAsync(H->gs, 0, sizeof(GState) * H->ninst, st));
    const int cand[5] = {kSplit8, kThrXcd, kThrPlain, kCol32, kCol16};
    for (int k = 0; k < 3; ++k)
      for (int w = 0; w < 2; ++w) {
        const int cnt = H->n_cg_all[k][w];
        if (cnt == 0) continue;
        const double *x = k == 0 ? H->F : (k == 1 ? H->lam : H->qb);
        double *y = k == 0 ? H->v : (k == 1 ? H->qb : H->v);
        H->cg_sched[k][w] = cand[fastest(st, e0, e1, 5, [&](int c) {
          const int sc = cand[c];
          if (w == 0) colgemm_w<1>(H, H->cg_all[k][w], cnt, H->cg_units[k][w], H->n_cg_units[k][w], k == 2 ? 1 : 0, x, y, st, sc);
          else colgemm_w<kColVecs / 16>(H, H->cg_all[k][w], cnt, H->cg_units[k][w], H->n_cg_units[k][w], k == 2 ? 1 : 0, x, y, st, sc);
        })];
      }
    // the whole product in 16-column items, one launch, against the two
    // width lists under their schedules
    for (int k = 0; k < 3; ++k) {
      H->cg_alt_sched[k] = -1;
      if (!H->n_cg_alt[k]) continue;
      const double *x = k == 0 ? H->F : (k == 1 ? H->lam : H->qb);
      double *y = k == 0 ? H->v : (k == 1 ? H->qb : H->v);
      const int c = fastest(st, e0, e1, 6, [&](int c) {
        if (c == 0) {
          colgemm(H, k, -1, k == 2 ? 1 : 0, x, y, st);
        } else {
          colgemm_w<1>(H, H->cg_alt[k], H->n_cg_alt[k], H->cg_alt_units[k], H->n_cg_alt_units[k], k == 2 ? 1 : 0, x,
                       y, st, cand[c - 1]);
        }
      });
      H->cg_alt_sched[k] = c > 0 ? cand[c - 1] : -1;
    }
    // the Schur right-hand side: the B A^-1 GEMM, or the element solves of
    // A^-1 and the B row functionals, whichever is faster (the GEMM's K is
    // m_z n^2, which on tall high-order strips costs more than the solves)
    if (H->use_ba)
      H->use_ba = fastest(st, e0, e1, 2, [&](int c) {
        if (c == 0) {
          ba_launch(H, H->ba_list, H->ba_sched, st);
          hipLaunchKernelGGL(k_bS, dim3(H->n_h), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_h,
                             (const double *)nullptr, H->bS, H->hs);
        } else {
          ainv(H, H->F, H->v, st);
          hipLaunchKernelGGL(k_bS, dim3(H->n_h), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_h, (const double *)H->v,
                             H->bS, H->hs);
        }
      }) == 0;
    HIPCHECK(hipGetLastError());
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// Schedules of the handle's GEMM lists, timed at setup (or by size).  The
// environment variables SMPM_GEMM_SCHED = 0..12 and SMPM_ELEM_SCHED = 1..5 then
// pin every shared-block matvec list (split K over 16 or 8 waves, LDS-staged
// XCD-ordered or plain, with 32- or 64-value chunks) or every element-interior
// list (split K, LDS-staged XCD-ordered, plain, 32-row or 16-row K-split
// tiles) to one schedule, for tests and experiments.
void tune(smpm_handle *H, hipStream_t st) {
  tune_schedules(H, st);
  if (const char *e = std::getenv("SMPM_GEMM_SCHED")) {
    const int v = std::atoi(e);
    if (v >= 0 && v < kNumSched)
      for (int op = 0; op < 3; ++op)
        for (int pr = 0; pr < 3; ++pr) {
          H->sched[op][pr] = v;
          H->g_list[op][pr] = 0;
        }
  }
  if (const char *e = std::getenv("SMPM_GEMM_LIST")) {   // 1: the 16-window lists where there are any
    const int l = std::atoi(e);
    if (l == 0 || l == 1)
      for (int op = 0; op < 2; ++op)
        for (int pr = 0; pr < 3; ++pr) H->g_list[op][pr] = H->gl[op][1].n ? l : 0;
  }
  if (const char *e = std::getenv("SMPM_RHS_GEMM")) {   // "schedule,list"
    int v = -1, l = 0;
    if (std::sscanf(e, "%d,%d", &v, &l) >= 1 && v >= 0 && v < kNumSched && (l == 0 || (l == 1 && H->n_bal[1]))) {
      H->ba_sched = v;
      H->ba_list = l;
    }
  }
  if (const char *e = std::getenv("SMPM_ELEM_SCHED")) {
    const int v = std::atoi(e);
    if (v >= kSplit8 && v <= kCol16) {
      const char *a = std::getenv("SMPM_ELEM_ALT");   // 1: the 16-column lists where there are any
      const bool alt = a && std::atoi(a) == 1;
      for (int k = 0; k < 3; ++k) {
        for (int w = 0; w < 2; ++w) H->cg_sched[k][w] = v;
        H->cg_alt_sched[k] = alt && H->n_cg_alt[k] ? v : -1;
      }
    }
  }
}

const int2 *xwork(smpm_handle *H, int inst, int &count) {
  if (inst < 0) { count = H->n_x; return H->w_x; }
  count = H->h_ins[inst].nchunk_x;
  return H->w_x + H->x_start[inst];
}

const int2 *hwork(smpm_handle *H, int inst, int &count) {
  if (inst < 0) { count = H->n_h; return H->w_h; }
  count = H->sys[H->h_ins[inst].sys].nh;
  return H->w_h + H->h_start[inst];
}

// ---------------------------------------------------------------------------
// Solve steps.

bool any_active(smpm_handle *H, hipStream_t st) {
  HIPCHECK(hipMemcpyAsync(H->h_gs, H->gs, sizeof(GState) * H->ninst, hipMemcpyDeviceToHost, st));
  HIPCHECK(hipStreamSynchronize(st));
  for (int i = 0; i < H->ninst; ++i)
    if (H->h_gs[i].active) return true;
  return false;
}

// Capture the work that body() enqueues on st into an executable graph.
template <typename F>
hipGraphExec_t capture(hipStream_t st, F &&body) {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  HIPCHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  try {
    body();
  } catch (...) {
    (void)hipStreamEndCapture(st, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  HIPCHECK(hipStreamEndCapture(st, &graph));
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) throw std::runtime_error("hipGraphInstantiate failed");
  return exec;
}

// 16-row tiles of the coarse vector: the second grid dimension of k_coarse
inline int ctiles(const smpm_handle *H) { return (H->dmax + 15) / 16; }

// Inner DBJ-GMRES (or BJ / Schur), operators and Krylov basis in precision T.
// FP64: b = b~, x_S = x.  FP32: b = the refinement residual, x_S += x.  The
// stopping test is |g| <= tol * sqrt(pairs[2 i]) (||b||^2, left by the
// preceding norm or residual step).
template <typename T>
struct Inner {
  static constexpr int P = sizeof(T) == 8 ? 0 : 1;
  static T *V(smpm_handle *H) { if constexpr (P == 0) return (T *)H->V64; else return (T *)H->V32; }
  static T *z(smpm_handle *H) { if constexpr (P == 0) return (T *)H->z64; else return (T *)H->z32; }
  static T *y(smpm_handle *H) { if constexpr (P == 0) return (T *)H->y64; else return (T *)H->y32; }
  static T *t(smpm_handle *H) { if constexpr (P == 0) return (T *)H->t64; else return (T *)H->t32; }
  static const double *b(smpm_handle *H) { return P == 0 ? H->bS : H->rb; }
  static double tol(smpm_handle *H) { return P == 0 ? H->tol : H->inner_tol; }
  static bool h16(smpm_handle *H) { return P == 1 && H->op16; }

  // coarse part c = G Z^T b (kept as t_b = Z^T b for the assembly), r0 = P b
  static void pre(smpm_handle *H, hipStream_t st) {
    const bool useP = H->method == SMPM_METHOD_DBJ;
    if (useP) {
      hipLaunchKernelGGL(k_zt<double>, dim3(H->n_h), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_h, b(H), 0,
                         (const double *)nullptr, (const GState *)nullptr, H->hs);
      hipLaunchKernelGGL(k_coarse, dim3(H->ninst, ctiles(H)), dim3(kBlock), sizeof(double) * H->dmax, st, H->d_sys, H->d_ins, (const double *)H->hs,
                         (const double *)nullptr, H->tb, H->cv, (const GState *)nullptr);
    }
    hipLaunchKernelGGL(k_init_basis<T>, dim3(H->n_x), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_x, b(H),
                       useP ? (const double *)H->cv : (const double *)nullptr, V(H), H->partn);
    // refinement sweeps stop at max(inner_tol ||r||, kSweepSafety tol ||b~||)
    const double bfrac = P == 0 ? 0.0 : kSweepSafety * H->tol / H->inner_tol;
    hipLaunchKernelGGL(k_gmres_start, dim3(H->ninst), dim3(kBlock), 0, st, H->d_ins, (const double *)H->partn,
                       (const double *)H->pairs, H->scale, H->g, H->gs, 1, (const double *)H->nb2, bfrac);
  }

  // z = (M^-1 + Z G Z^T) x for the additive two-level method (x: Krylov slot
  // `iter` when vslot, else the interface vector t).
  static void twolevel(smpm_handle *H, const T *x, int vslot, const double *scale, const GState *g, T *zb,
                       hipStream_t st) {
    gemv<T, T, T>(H, 1, x, vslot, scale, zb, nullptr, g, st, -1, h16(H));
    hipLaunchKernelGGL(k_zt<T>, dim3(H->n_h), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_h, x, vslot, scale, g,
                       H->hs);
    hipLaunchKernelGGL(k_coarse, dim3(H->ninst, ctiles(H)), dim3(kBlock), sizeof(double) * H->dmax, st, H->d_sys, H->d_ins, (const double *)H->hs,
                       (const double *)nullptr, (double *)nullptr, H->cv, g);
    hipLaunchKernelGGL(k_add_zc<T>, dim3(H->n_x), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_x, zb,
                       (const double *)H->cv, g);
  }

  static void iteration(smpm_handle *H, hipStream_t st) {
    const bool useM = H->method != SMPM_METHOD_SCHUR;
    const bool useP = H->method == SMPM_METHOD_DBJ;
    const int maxit = H->maxit;
    const size_t shm_dot = sizeof(double) * (maxit + 1);
    T *Vb = V(H), *zb = z(H), *yb = y(H);
    // Z^T y for P: from the matvec's epilogue (one column per interface) or
    // a segment-sum pass (one column per element segment)
    double *hsum = useP && H->zlabel == 0 ? H->hs : nullptr;
    if (H->method == SMPM_METHOD_2LAS) {
      twolevel(H, (const T *)Vb, 1, H->scale, H->gs, zb, st);
      gemv<T, T, T>(H, 0, (const T *)zb, 0, nullptr, yb, nullptr, H->gs, st, -1, h16(H));
    } else if (useM && H->use_fused[sizeof(T) == 8 ? 0 : (h16(H) ? 2 : 1)]) {   // y = (S M^-1) v in one GEMM
      gemv<T, T, T>(H, 2, (const T *)Vb, 1, H->scale, yb, hsum, H->gs, st, -1, h16(H));
    } else if (useM) {
      gemv<T, T, T>(H, 1, (const T *)Vb, 1, H->scale, zb, nullptr, H->gs, st, -1, h16(H));
      gemv<T, T, T>(H, 0, (const T *)zb, 0, nullptr, yb, hsum, H->gs, st, -1, h16(H));
    } else {
      gemv<T, T, T>(H, 0, (const T *)Vb, 1, H->scale, yb, hsum, H->gs, st, -1, h16(H));
    }
    // one coarse column per element segment: d up to (m_x - 1) m_z, so the
    // coarse values are formed once (G read once) instead of per workgroup
    const bool cpre = useP && H->zlabel != 0;
    if (cpre) {
      hipLaunchKernelGGL(k_zt<T>, dim3(H->n_h), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_h, (const T *)yb, 0,
                         (const double *)nullptr, (const GState *)H->gs, H->hs);
      hipLaunchKernelGGL(k_coarse, dim3(H->ninst, ctiles(H)), dim3(kBlock), sizeof(double) * H->dmax, st, H->d_sys,
                         H->d_ins, (const double *)H->hs, (const double *)nullptr, (double *)nullptr, H->cv,
                         (const GState *)H->gs);
    }
    if (H->reg_basis)
      hipLaunchKernelGGL((k_pcorr_dot<T, T, true>), dim3(H->n_x), dim3(kBlock), cpre ? 0 : sizeof(double) * H->dmax, st,
                         H->d_sys, H->d_ins, H->w_x, (const T *)yb, (const double *)H->hs, useP ? 1 : 0, Vb, H->part1,
                         (const GState *)H->gs, cpre ? (const double *)H->cv : (const double *)nullptr);
    else
      hipLaunchKernelGGL((k_pcorr_dot<T, T>), dim3(H->n_x), dim3(kBlock), cpre ? 0 : sizeof(double) * H->dmax, st,
                         H->d_sys, H->d_ins, H->w_x, (const T *)yb, (const double *)H->hs, useP ? 1 : 0, Vb, H->part1,
                         (const GState *)H->gs, cpre ? (const double *)H->cv : (const double *)nullptr);
    // One Krylov space over all instances (Sec. 5.2): every reduction spans
    // the segment, so the partials go through k_seg_reduce first.
    const bool seg = H->one_krylov;
    auto seg_reduce = [&](const double *part, double *out, int norm) {
      hipLaunchKernelGGL(k_seg_reduce, dim3(norm ? 1 : maxit + 1, H->ninst), dim3(kBlock), 0, st, H->d_ins, part, out,
                         (const GState *)H->gs, norm);
    };
    if (!seg) {
      // CGS2 in two passes; the second takes the Givens step in its last
      // workgroup (the first pass leaves |w|^2 for the Pythagorean norm)
      if (H->reg_basis) {
        hipLaunchKernelGGL((k_axpy_dot<T, true>), dim3(H->n_x), dim3(kBlock), shm_dot, st, H->d_sys, H->d_ins, H->w_x,
                           Vb, (const double *)H->part1, H->part2, H->partn, (const double *)H->scale,
                           (const GState *)H->gs, (const double *)nullptr);
        hipLaunchKernelGGL((k_axpy_givens<T, true>), dim3(H->n_x), dim3(kBlock), sizeof(double) * (5 * maxit + 4), st,
                           H->d_sys, H->d_ins, H->w_x, Vb, (const double *)H->part1, (const double *)H->part2,
                           (const double *)H->partn, H->scale, H->Rm, H->cs, H->sn, H->g, H->gs, H->arrive, maxit,
                           tol(H));
        return;
      }
      hipLaunchKernelGGL((k_axpy_dot<T>), dim3(H->n_x), dim3(kBlock), shm_dot, st, H->d_sys, H->d_ins, H->w_x, Vb,
                         (const double *)H->part1, H->part2, H->partn, (const double *)H->scale,
                         (const GState *)H->gs, (const double *)nullptr);
      hipLaunchKernelGGL((k_axpy_givens<T>), dim3(H->n_x), dim3(kBlock), sizeof(double) * (5 * maxit + 4), st,
                         H->d_sys, H->d_ins, H->w_x, Vb, (const double *)H->part1, (const double *)H->part2,
                         (const double *)H->partn, H->scale, H->Rm, H->cs, H->sn, H->g, H->gs, H->arrive, maxit,
                         tol(H));
      return;
    }
    seg_reduce(H->part1, H->sr1, 0);
    hipLaunchKernelGGL((k_axpy_dot<T>), dim3(H->n_x), dim3(kBlock), shm_dot, st, H->d_sys, H->d_ins, H->w_x, Vb,
                       (const double *)H->part1, H->part2, (double *)nullptr, (const double *)H->scale, (const GState *)H->gs,
                       seg ? (const double *)H->sr1 : nullptr);
    if (seg) seg_reduce(H->part2, H->sr2, 0);
    hipLaunchKernelGGL((k_axpy_dot<T>), dim3(H->n_x), dim3(kBlock), shm_dot, st, H->d_sys, H->d_ins, H->w_x, Vb,
                       (const double *)H->part2, (double *)nullptr, H->partn, (const double *)H->scale, (const GState *)H->gs,
                       seg ? (const double *)H->sr2 : nullptr);
    if (seg) seg_reduce(H->partn, H->srn, 1);
    hipLaunchKernelGGL(k_givens, dim3(H->ninst), dim3(kBlock), sizeof(double) * (3 * maxit + 2), st, H->d_ins,
                       (const double *)H->part1, (const double *)H->part2, (const double *)H->partn, H->scale, H->Rm,
                       H->cs, H->sn, H->g, H->gs, maxit, tol(H), seg ? (const double *)H->sr1 : nullptr,
                       seg ? (const double *)H->sr2 : nullptr, seg ? (const double *)H->srn : nullptr);
  }

  // x' = V y; x = M^-1 x' + coarse correction, into (or onto) x_S
  static void post(smpm_handle *H, hipStream_t st) {
    const bool useM = H->method != SMPM_METHOD_SCHUR;
    const bool useP = H->method == SMPM_METHOD_DBJ;
    const int maxit = H->maxit;
    T *Vb = V(H), *zb = z(H), *yb = y(H), *tb = t(H);
    hipLaunchKernelGGL(k_backsolve, dim3(H->ninst), dim3(kBlock), sizeof(double) * (maxit + 1 + kTriLds), st, H->d_ins,
                       (const double *)H->Rm, (const double *)H->g, (const double *)H->scale, H->ycoef,
                       (const GState *)H->gs, maxit);
    hipLaunchKernelGGL((k_combine<T, T>), dim3(H->n_x), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_x, (const T *)Vb,
                       (const double *)H->ycoef, tb, (const GState *)H->gs);
    const T *xfin = tb;
    if (H->method == SMPM_METHOD_2LAS) {
      twolevel(H, (const T *)tb, 0, nullptr, nullptr, zb, st);
      xfin = zb;
    } else if (useM) {
      gemv<T, T, T>(H, 1, (const T *)tb, 0, nullptr, zb, nullptr, nullptr, st, -1, h16(H));
      xfin = zb;
    }
    const double *cfin = nullptr;
    if (useP) {   // c' = G (Z^T b - Z^T S z): x = z + Z c'
      gemv<T, T, T>(H, 0, xfin, 0, nullptr, yb, H->zlabel == 0 ? H->hs : nullptr, nullptr, st, -1, h16(H));
      if (H->zlabel != 0)
        hipLaunchKernelGGL(k_zt<T>, dim3(H->n_h), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_h, (const T *)yb, 0,
                           (const double *)nullptr, (const GState *)nullptr, H->hs);
      hipLaunchKernelGGL(k_coarse, dim3(H->ninst, ctiles(H)), dim3(kBlock), sizeof(double) * H->dmax, st, H->d_sys, H->d_ins, (const double *)H->hs,
                         (const double *)H->tb, (double *)nullptr, H->cv, (const GState *)nullptr);
      cfin = H->cv;
    }
    hipLaunchKernelGGL(k_xupdate<T>, dim3(H->n_x), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_x, P == 0 ? 0 : 1,
                       xfin, cfin, H->xS, (double *)nullptr, (const double *)nullptr);
  }

  // The iteration graphs: kIterChunk iterations, and 1 .. kIterChunk - 1.
  static void capture_loops(smpm_handle *H, hipStream_t st) {
    if (!H->g_loop[P])
      H->g_loop[P] = capture(st, [&] {
        for (int c = 0; c < kIterChunk; ++c) iteration(H, st);
      });
    for (int n = 1; n < kIterChunk; ++n)
      if (!H->g_rem[P][n])
        H->g_rem[P][n] = capture(st, [&] {
          for (int c = 0; c < n; ++c) iteration(H, st);
        });
    if (P == 1) {   // the refinement's inner solves (FP64 folds these into its head and tail)
      if (!H->g_pre[P]) H->g_pre[P] = capture(st, [&] { pre(H, st); });
      if (!H->g_post[P]) H->g_post[P] = capture(st, [&] { post(H, st); });
    }
  }

  // Enqueue n GMRES iterations: whole chunks, then one graph of the rest.
  static void iterations(smpm_handle *H, int n, hipStream_t st) {
    if (!H->g_loop[P])
      H->g_loop[P] = capture(st, [&] {
        for (int c = 0; c < kIterChunk; ++c) iteration(H, st);
      });
    for (; n >= kIterChunk; n -= kIterChunk) HIPCHECK(hipGraphLaunch(H->g_loop[P], st));
    if (n > 0) {
      if (!H->g_rem[P][n])
        H->g_rem[P][n] = capture(st, [&] {
          for (int c = 0; c < n; ++c) iteration(H, st);
        });
      HIPCHECK(hipGraphLaunch(H->g_rem[P][n], st));
    }
  }

  // The predicted iterations (the previous solve's count, of the same sweep
  // for the refinement; one chunk for the first solve), capped at maxit;
  // returns how many were enqueued.
  static int predicted(smpm_handle *H, int slot, hipStream_t st) {
    int pred = H->pred_iters[P];
    if (P == 1 && slot < (int)H->pred_sweep.size() && H->pred_sweep[slot] >= 0) pred = H->pred_sweep[slot];
    pred = pred < 0 ? kIterChunk : pred + H->pred_margin[P];
    const int n = std::min(pred, H->maxit);
    iterations(H, n, st);
    return n;
  }

  // Further chunks while an instance is still iterating (one host check per
  // chunk).
  static void until_done(smpm_handle *H, int launched, hipStream_t st) {
    while (launched < H->maxit && any_active(H, st)) {
      const int n = std::min(kIterChunk, H->maxit - launched);
      iterations(H, n, st);
      launched += n;
    }
  }

  // One inner solve of exactly the predicted iterations, with no host check:
  // an instance still iterating then yields a less accurate correction,
  // which the refinement's later sweeps make up for.  States to slot `slot`.
  static void run_fixed(smpm_handle *H, int slot, hipStream_t st) {
    if (!H->g_pre[P]) H->g_pre[P] = capture(st, [&] { pre(H, st); });
    if (!H->g_post[P]) H->g_post[P] = capture(st, [&] { post(H, st); });
    HIPCHECK(hipGraphLaunch(H->g_pre[P], st));
    predicted(H, slot, st);
    HIPCHECK(hipGraphLaunch(H->g_post[P], st));
    HIPCHECK(hipMemcpyAsync(H->h_gs_hist + (size_t)slot * H->ninst, H->gs, sizeof(GState) * H->ninst,
                            hipMemcpyDeviceToHost, st));
  }

  // Enqueue one inner solve; its final GMRES states are copied to the pinned
  // history slot `slot` (read after the solve's last synchronization).
  static void run(smpm_handle *H, int slot, hipStream_t st) {
    if (!H->g_pre[P]) H->g_pre[P] = capture(st, [&] { pre(H, st); });
    if (!H->g_post[P]) H->g_post[P] = capture(st, [&] { post(H, st); });
    HIPCHECK(hipGraphLaunch(H->g_pre[P], st));
    until_done(H, predicted(H, slot, st), st);
    HIPCHECK(hipGraphLaunch(H->g_post[P], st));
    HIPCHECK(hipMemcpyAsync(H->h_gs_hist + (size_t)slot * H->ninst, H->gs, sizeof(GState) * H->ninst,
                            hipMemcpyDeviceToHost, st));
  }
};

// r = b~ - S x_S (FP64); pairs[2 i] = ||r||^2, pairs[2 i + 1] = u_S . r; then
// r <- r - u_S (u_S . r) (the refinement residual, k = 0).  after_dbj: the
// final check of an FP64 DBJ solve, right after its assembly left S z in
// y64 and the coarse correction c in cv with x_S = z + Z c: then
// S x_S = S z + (S Z) c needs no further Schur product, and r is only
// measured, not projected.
void residual64(smpm_handle *H, hipStream_t st, bool after_dbj = false) {
  if (after_dbj) {
    hipLaunchKernelGGL(k_xupdate<double>, dim3(H->n_x), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_x, 2,
                       (const double *)H->y64, (const double *)H->cv, H->rb, H->partn, (const double *)H->bS);
    hipLaunchKernelGGL(k_reduce_pairs, dim3(H->ninst), dim3(kBlock), 0, st, H->d_ins, (const double *)H->partn,
                       H->pairs, (double *)nullptr);
    return;
  }
  gemv<double, double, double>(H, 0, H->xS, 0, nullptr, H->y64, nullptr, nullptr, st);
  hipLaunchKernelGGL(k_xupdate<double>, dim3(H->n_x), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_x, 2,
                     (const double *)H->y64, (const double *)nullptr, H->rb, H->partn, (const double *)H->bS);
  hipLaunchKernelGGL(k_reduce_pairs, dim3(H->ninst), dim3(kBlock), 0, st, H->d_ins, (const double *)H->partn, H->pairs,
                     (double *)nullptr);
  hipLaunchKernelGGL(k_proj_x_scalar, dim3(H->n_x), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_x, H->rb,
                     (const double *)H->pairs);
}

// F = f + tau g into the handle's F: the one step of the solve that reads the
// caller's f and g.  It is launched on its own, ahead of the captured graphs,
// so that the graphs never hold a caller pointer and are captured once per
// handle whatever buffers the caller passes.
void read_rhs(smpm_handle *H, const double *f, const double *g, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs, dim3(H->n_r), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_r, f, g, H->F, H->pr);
}

// The rest of the Schur right-hand side of Algorithm 2, from F = f + tau g:
// F~ = F - u_L u_L^T F, v = A^-1 F~, b~ = B v - u_S u_S^T B v; then pairs =
// (||b~||^2, u_S . b~), and for the refined form r = b~, x_S = 0.
void stage_rhs(smpm_handle *H, hipStream_t st) {
  hipLaunchKernelGGL(k_proj_r, dim3(H->n_r), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_r, H->F, H->pr, H->defect);
  if (H->use_ba) {   // b_S = (B A^-1) F~ in one GEMM over the strips, then u_S . b_S per half
    ba_launch(H, H->ba_list, H->ba_sched, st);
    hipLaunchKernelGGL(k_bS, dim3(H->n_h), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_h, (const double *)nullptr,
                       H->bS, H->hs);
  } else {
    ainv(H, H->F, H->v, st);
    hipLaunchKernelGGL(k_bS, dim3(H->n_h), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_h, (const double *)H->v, H->bS,
                       H->hs);
  }
  hipLaunchKernelGGL(k_proj_x, dim3(H->n_x), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_x, H->bS, (const double *)H->hs,
                     H->partn);
  hipLaunchKernelGGL(k_reduce_pairs, dim3(H->ninst), dim3(kBlock), 0, st, H->d_ins, (const double *)H->partn, H->pairs,
                     H->nb2);
  if (H->precision != SMPM_FP64) {   // r = b~ (a copy through mode 0), x_S = 0
    hipLaunchKernelGGL(k_xupdate<double>, dim3(H->n_x), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_x, 0,
                       (const double *)H->bS, (const double *)nullptr, H->rb, (double *)nullptr,
                       (const double *)nullptr);
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((H->tot_x + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, H->xS, H->tot_x,
                       0.0);
  }
}

// Interior recovery of Algorithm 2: v = A^-1 (F~ - E x_S) into the handle's v
// (free once b~ is formed) and the partial sums of its mean.
void finish_u(smpm_handle *H, hipStream_t st) {
  hipLaunchKernelGGL(k_recover_rhs, dim3(H->n_r), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_r, (const double *)H->F,
                     (const double *)H->xS, H->Rr);
  ainv(H, H->Rr, H->v, st);
  hipLaunchKernelGGL(k_sum_r, dim3(H->n_r), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_r, (const double *)H->v, H->pr);
}

// The gauge and the output: u = v minus its nodal mean for k = 0, u = v for
// k > 0.  Like read_rhs, launched outside the captured graphs, as the one
// step that writes the caller's u.
void write_u(smpm_handle *H, double *u, hipStream_t st) {
  hipLaunchKernelGGL(k_sub_mean, dim3(H->n_r), dim3(kBlock), 0, st, H->d_sys, H->d_ins, H->w_r, (const double *)H->v, u,
                     (const double *)H->pr);
}

// Every graph a solve of this handle launches, captured once at setup (the
// graphs read and write the handle's own buffers only): a solve then launches
// them without capturing or instantiating anything.
void capture_graphs(smpm_handle *H) {
  hipStream_t st = H->ws;
  if (H->precision == SMPM_FP64) {
    if (!H->g_head)
      H->g_head = capture(st, [&] {
        stage_rhs(H, st);
        Inner<double>::pre(H, st);
      });
    if (!H->g_tail)
      H->g_tail = capture(st, [&] {
        Inner<double>::post(H, st);
        residual64(H, st, H->method == SMPM_METHOD_DBJ);
        finish_u(H, st);
      });
    Inner<double>::capture_loops(H, st);
  } else {
    if (!H->g_stage) H->g_stage = capture(st, [&] { stage_rhs(H, st); });
    if (!H->g_resid) H->g_resid = capture(st, [&] { residual64(H, st); });
    if (!H->g_finish) H->g_finish = capture(st, [&] { finish_u(H, st); });
    Inner<float>::capture_loops(H, st);
  }
  HIPCHECK(hipStreamSynchronize(st));
}

// The FFT path of the y transform: m_y a power of two with at least one
// column per workgroup's staging (else the dense DFT GEMM).
bool fft_ok(int my) { return my >= 2 && (my & (my - 1)) == 0 && my <= kFftSlots; }

// y transform of ncol columns: forward (planes -> Re/Im of m_y/2 + 1 modes,
// scaled by 1/m_y) or inverse, by FFT where m_y allows, else by the DFT GEMM.
void transform_y(smpm_handle *H, bool inverse, const double *in, double *out, int64_t ncol, hipStream_t st) {
  const int my = H->my, nk2 = 2 * (my / 2 + 1);
  if (H->fft_tw) {
    int logmy = 0;
    while ((1 << logmy) < my) ++logmy;
    if (my >= 16 && my <= 128) {   // two steps through LDS
      const dim3 grid((unsigned)((ncol + 2 * (kFftPackSlots / my) - 1) / (2 * (kFftPackSlots / my))));
      const double2 *tw = (const double2 *)H->fft_tw;
      switch (logmy * 2 + (inverse ? 1 : 0)) {
#define SMPM_FFT4_CASE(L)                                                                                  \
  case 2 * L:                                                                                              \
    hipLaunchKernelGGL((k_fft_y_4s<L, false>), grid, dim3(256), 0, st, in, out, ncol, tw);                \
    return;                                                                                                \
  case 2 * L + 1:                                                                                          \
    hipLaunchKernelGGL((k_fft_y_4s<L, true>), grid, dim3(256), 0, st, in, out, ncol, tw);                 \
    return;
        SMPM_FFT4_CASE(4) SMPM_FFT4_CASE(5) SMPM_FFT4_CASE(6) SMPM_FFT4_CASE(7)
#undef SMPM_FFT4_CASE
        default:
          break;
      }
    }
    if (my >= 8 && my <= kFftPackSlots) {   // two real columns per complex FFT, sizes fixed at compile time
      const dim3 grid((unsigned)((ncol + 2 * (kFftPackSlots / my) - 1) / (2 * (kFftPackSlots / my))));
      const double2 *tw = (const double2 *)H->fft_tw;
      switch (logmy * 2 + (inverse ? 1 : 0)) {
#define SMPM_FFT_CASE(L)                                                                                   \
  case 2 * L:                                                                                              \
    hipLaunchKernelGGL((k_fft_y_pack<L, false>), grid, dim3(256), 0, st, in, out, ncol, tw);              \
    return;                                                                                                \
  case 2 * L + 1:                                                                                          \
    hipLaunchKernelGGL((k_fft_y_pack<L, true>), grid, dim3(256), 0, st, in, out, ncol, tw);               \
    return;
        SMPM_FFT_CASE(3) SMPM_FFT_CASE(4) SMPM_FFT_CASE(5) SMPM_FFT_CASE(6) SMPM_FFT_CASE(7) SMPM_FFT_CASE(8)
        SMPM_FFT_CASE(9) SMPM_FFT_CASE(10) SMPM_FFT_CASE(11)
#undef SMPM_FFT_CASE
        default:
          break;
      }
    }
    const int CT = kFftSlots / my;
    const dim3 grid((unsigned)((ncol + CT - 1) / CT));
    const size_t shm = sizeof(double2) * kFftSlots;
    if (inverse)
      hipLaunchKernelGGL(k_fft_y<true>, grid, dim3(256), shm, st, in, out, my, logmy, ncol, (const double2 *)H->fft_tw);
    else
      hipLaunchKernelGGL(k_fft_y<false>, grid, dim3(256), shm, st, in, out, my, logmy, ncol, (const double2 *)H->fft_tw);
    return;
  }
  const int M = inverse ? my : nk2, K = inverse ? nk2 : my;
  const dim3 grid((unsigned)((ncol + 63) / 64), (unsigned)(((M + 15) / 16 + kDftTiles - 1) / kDftTiles));
  hipLaunchKernelGGL(k_dft_gemm, grid, dim3(256), 0, st, inverse ? H->dft_i : H->dft_f, M, K, in, out, ncol);
}

// Real DFT matrices and coefficient buffers of a Fourier handle:
// forward  f_m = (1/m_y) sum_j f_j (cos - i sin)(2 pi m j / m_y);
// inverse  u_j = sum_m w_m (Re u_m cos - Im u_m sin)(2 pi m j / m_y),
//          w_0 = 1, w_{m_y/2} = 1 for even m_y, else 2.
void fourier_tables(smpm_handle *H, hipStream_t s0) {
  const int my = H->my, nk = my / 2 + 1;
  std::vector<double> F((size_t)2 * nk * my), I((size_t)my * 2 * nk);
  for (int m = 0; m < nk; ++m) {
    const double w = (m == 0 || (my % 2 == 0 && m == my / 2)) ? 1.0 : 2.0;
    for (int j = 0; j < my; ++j) {
      const double th = 2.0 * M_PI * (double)(((int64_t)m * j) % my) / my;
      F[(size_t)(2 * m) * my + j] = std::cos(th) / my;
      F[(size_t)(2 * m + 1) * my + j] = -std::sin(th) / my;
      I[(size_t)j * 2 * nk + 2 * m] = w * std::cos(th);
      I[(size_t)j * 2 * nk + 2 * m + 1] = -w * std::sin(th);
    }
  }
  H->dft_f = dupload(H->owned, F, s0);
  H->dft_i = dupload(H->owned, I, s0);
  if (fft_ok(my)) {
    std::vector<double> tw((size_t)my);   // (cos, -sin) pairs, angle reduced like the DFT tables
    for (int k = 0; k < my / 2; ++k) {
      const double th = 2.0 * M_PI * (double)k / my;
      tw[2 * k] = std::cos(th);
      tw[2 * k + 1] = -std::sin(th);
    }
    H->fft_tw = reinterpret_cast<double2 *>(dupload(H->owned, tw, s0));
  }
  H->fhat = dalloc<double>(H->owned, H->tot_r);
  H->uhat = dalloc<double>(H->owned, H->tot_r);
  H->ghat = dalloc<double>(H->owned, H->tot_g);
  HIPCHECK(hipStreamSynchronize(s0));
}

smpm_status validate_opts(const smpm_opts *o, smpm_handle *H) {
  smpm_opts d{};
  if (o) d = *o;
  H->opts = d;
  H->tol = d.tol > 0 ? d.tol : 1e-10;
  H->maxit = d.max_iter > 0 ? d.max_iter : 300;
  H->nrhs = d.nrhs > 0 ? d.nrhs : 1;
  H->precision = d.precision;
  H->method = d.method;
  H->inner_tol = d.inner_tol > 0 ? d.inner_tol : 1e-4;
  H->max_sweeps = d.max_sweeps > 0 ? d.max_sweeps : (d.precision == SMPM_FP16S_IR ? 40 : 12);
  H->host_only = (d.flags & SMPM_FLAG_HOST_ONLY) != 0;
  H->no_tune = (d.flags & SMPM_FLAG_NO_TUNE) != 0;
  H->one_krylov = (d.flags & SMPM_FLAG_ONE_KRYLOV) != 0;
  H->zlabel = d.zlabel;
  if (d.zlabel != 0 && d.zlabel != 1) return fail(SMPM_EINVAL, "zlabel must be 0 (per interface) or 1 (per element)");
  if (H->one_krylov && H->method != SMPM_METHOD_DBJ) return fail(SMPM_EINVAL, "one Krylov space needs the DBJ method");
  if (d.tol < 0 || d.max_iter < 0 || d.nrhs < 0 || d.inner_tol < 0 || d.max_sweeps < 0)
    return fail(SMPM_EINVAL, "negative option value");
  if (H->maxit > 2000) return fail(SMPM_EINVAL, "max_iter above 2000");
  if (H->precision != SMPM_FP64 && H->precision != SMPM_FP32_IR && H->precision != SMPM_FP16S_IR)
    return fail(SMPM_EINVAL, "unknown precision");
  H->op16 = H->precision == SMPM_FP16S_IR;
  if (H->method < SMPM_METHOD_DBJ || H->method > SMPM_METHOD_2LAS)
    return fail(SMPM_EINVAL, "unknown method (DBJ, BJ, SCHUR, 2LAS)");
  return SMPM_OK;
}

smpm_status setup_common(const smpm_grid *grids, const double *k, int nsys, bool one_grid,
                         const smpm_opts *opts, void *stream, smpm_handle **out) {
  if (!out) return fail(SMPM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grids || !k || nsys < 1) return fail(SMPM_EINVAL, "grids/k NULL or count < 1");
  std::unique_ptr<smpm_handle> H(new smpm_handle());
  smpm_status st = validate_opts(opts, H.get());
  if (st != SMPM_OK) return st;
  for (int i = 0; i < nsys; ++i) {
    const smpm_grid &g = one_grid ? grids[0] : grids[i];
    if (!g.xb || !g.zb) return fail(SMPM_EINVAL, "grid breakpoints NULL");
    if (g.mx < 2 || g.mz < 1 || g.order < 1) return fail(SMPM_EINVAL, "need mx >= 2, mz >= 1, order >= 1");
    if ((int64_t)(g.order + 1) * g.mz > kMaxN) return fail(SMPM_EINVAL, "n * m_z above the supported 544");
    if (g.order + 1 > kMaxNodes) return fail(SMPM_EINVAL, "order above 21 is not supported");
    if (g.mx - 1 > 1024) return fail(SMPM_EINVAL, "more than 1025 strips");
    if ((int64_t)(g.mx - 1) * (H->zlabel ? g.mz : 1) > 4096)
      return fail(SMPM_EINVAL, "coarse space above 4096 unknowns");
    if (!(k[i] >= 0.0) || !std::isfinite(k[i])) return fail(SMPM_EINVAL, "wavenumbers must be finite and >= 0");
  }
  H->sys.resize(nsys);
  std::vector<std::string> errs(nsys);
  std::vector<int> codes(nsys, SMPM_OK);
  SetupOptions so;
  so.tau = H->opts.tau;
  so.zlabel = H->zlabel;
  so.threads = nsys > 1 ? 1 : 0;   // parallel over systems, or over strip classes of one system
  // the large dense setup steps on the device, unless asked not to
  std::unique_ptr<DeviceDense, void (*)(DeviceDense *)> dense(
      H->host_only || (H->opts.flags & SMPM_FLAG_HOST_SETUP)
          ? nullptr
          : device_dense_create((H->opts.flags & SMPM_FLAG_DEVICE_SETUP) != 0),
      device_dense_destroy);
  so.dense = device_dense_backend(dense.get());
  // the u_S elimination runs beside the other steps: a back end of its own
  std::unique_ptr<DeviceDense, void (*)(DeviceDense *)> dense_null(
      dense ? device_dense_create((H->opts.flags & SMPM_FLAG_DEVICE_SETUP) != 0) : nullptr, device_dense_destroy);
  so.dense_null = device_dense_backend(dense_null.get());
  // Grids with 16 interfaces or more reach the back ends (the u_S
  // elimination, then the large batches of one system): their start-up
  // runs on worker threads beside the host steps.  Batches of systems build
  // on one host thread each, whose blocks stay small, so there only the u_S
  // back end starts early.  Declared after the back ends, so the futures are
  // joined before those are destroyed.
  bool wide = false, any_singular = false;
  int nmax = 0;   // largest N = (order + 1) m_z
  for (int i = 0; i < nsys; ++i) {
    const smpm_grid &g = one_grid ? grids[0] : grids[i];
    wide = wide || g.mx - 1 >= 16;
    any_singular = any_singular || k[i] == 0.0;
    nmax = std::max(nmax, (g.order + 1) * g.mz);
  }
  std::future<void> warm_dense, warm_null;
  if (wide && nsys == 1 && so.dense && so.dense->warm)   // the block-Jacobi blocks are 4 N square
    warm_dense = std::async(std::launch::async, so.dense->warm, grids[0].order + 1, grids[0].mz, 4 * nmax, 0);
  if (wide && any_singular && so.dense_null && so.dense_null->warm)
    warm_null = std::async(std::launch::async, so.dense_null->warm, 0, 0, 0, nmax);
  parallel_for(nsys, nsys > 1 ? 0 : 1, [&](int i) {
    const smpm_grid &g = one_grid ? grids[0] : grids[i];
    try {
      build_system(H->sys[i], g.mx, g.mz, g.order, g.xb, g.zb, k[i], so);
    } catch (const std::invalid_argument &e) {
      codes[i] = SMPM_EINVAL; errs[i] = e.what();
    } catch (const std::domain_error &e) {
      codes[i] = SMPM_ESINGULAR; errs[i] = e.what();
    } catch (const std::bad_alloc &) {
      codes[i] = SMPM_ENOMEM; errs[i] = "host allocation failed in setup";
    } catch (const std::exception &e) {
      codes[i] = SMPM_ESINGULAR; errs[i] = e.what();
    }
  });
  for (int i = 0; i < nsys; ++i)
    if (codes[i] != SMPM_OK) return fail((smpm_status)codes[i], "system " + std::to_string(i) + ": " + errs[i]);
  if (!H->host_only) {
    const bool times = std::getenv("SMPM_SETUP_TIMES") != nullptr;
    auto t0 = std::chrono::steady_clock::now();
    auto lap = [&](const char *what) {
      if (!times) return;
      HIPCHECK(hipDeviceSynchronize());
      const auto now = std::chrono::steady_clock::now();
      std::fprintf(stderr, "setup %-28s %8.1f ms\n", what, std::chrono::duration<double, std::milli>(now - t0).count());
      t0 = now;
    };
    try {
      upload(H.get(), (hipStream_t)stream);
      lap("upload");
      tune(H.get(), (hipStream_t)stream);
      lap("schedule tuning");
      capture_graphs(H.get());
      lap("graph capture");
    } catch (const std::bad_alloc &) {
      return fail(SMPM_ENOMEM, "device allocation failed in setup");
    } catch (const std::exception &e) {
      return fail(SMPM_EHIP, e.what());
    }
  }
  *out = H.release();
  return SMPM_OK;
}

}  // namespace

extern "C" {

smpm_status smpm_setup(const smpm_grid *grid, const double *k, int32_t nk, const smpm_opts *opts,
                       void *hip_stream, smpm_handle **out) {
  return setup_common(grid, k, nk, true, opts, hip_stream, out);
}

smpm_status smpm_setup_batch(const smpm_grid *grids, const double *k, int32_t nprob, const smpm_opts *opts,
                             void *hip_stream, smpm_handle **out) {
  return setup_common(grids, k, nprob, false, opts, hip_stream, out);
}

smpm_status smpm_setup_fourier(const smpm_grid *grid, int32_t my, double ly, const smpm_opts *opts,
                               void *hip_stream, smpm_handle **out) {
  if (!out) return fail(SMPM_EINVAL, "out is NULL");
  *out = nullptr;
  if (my < 2 || !(ly > 0.0) || !std::isfinite(ly)) return fail(SMPM_EINVAL, "need m_y >= 2 and l_y > 0");
  smpm_opts o{};
  if (opts) o = *opts;
  if (o.nrhs != 0 && o.nrhs != 2) return fail(SMPM_EINVAL, "a Fourier handle has nrhs = 2 (Re, Im)");
  o.nrhs = 2;
  const int nk = my / 2 + 1;
  std::vector<double> k(nk);
  for (int m = 0; m < nk; ++m) k[m] = 2.0 * M_PI * m / ly;
  smpm_handle *H = nullptr;
  smpm_status st = setup_common(grid, k.data(), nk, true, &o, hip_stream, &H);
  if (st != SMPM_OK) return st;
  H->my = my;
  H->ly = ly;
  if (!H->host_only) {
    try {
      fourier_tables(H, (hipStream_t)hip_stream);
    } catch (const std::exception &e) {
      delete H;
      return fail(SMPM_ENOMEM, e.what());
    }
  }
  *out = H;
  return SMPM_OK;
}

smpm_status smpm_save(const smpm_handle *H, const char *path) {
  if (!H || !path) return fail(SMPM_EINVAL, "handle or path is NULL");
  try {
    TableHeader h;
    h.zlabel = H->zlabel;
    h.my = H->my;
    h.ly = H->ly;
    save_tables(path, h, H->sys);
  } catch (const std::exception &e) {
    return fail(SMPM_EINVAL, e.what());
  }
  return SMPM_OK;
}

smpm_status smpm_load(const char *path, const smpm_opts *opts, void *hip_stream, smpm_handle **out) {
  if (!out || !path) return fail(SMPM_EINVAL, "out or path is NULL");
  *out = nullptr;
  TableHeader h;
  std::vector<System> sys;
  try {
    load_tables(path, h, sys);
  } catch (const std::bad_alloc &) {
    return fail(SMPM_ENOMEM, "host allocation failed while loading tables");
  } catch (const std::exception &e) {
    return fail(SMPM_EINVAL, e.what());
  }
  smpm_opts o{};
  if (opts) o = *opts;
  else o.zlabel = h.zlabel;
  if (o.zlabel != h.zlabel) return fail(SMPM_EINVAL, "zlabel differs from the one the tables were built for");
  if (h.my > 0) {
    if (o.nrhs != 0 && o.nrhs != 2) return fail(SMPM_EINVAL, "a Fourier handle has nrhs = 2 (Re, Im)");
    o.nrhs = 2;
  }
  std::unique_ptr<smpm_handle> H(new smpm_handle());
  smpm_status st = validate_opts(&o, H.get());
  if (st != SMPM_OK) return st;
  H->sys = std::move(sys);
  H->my = h.my;
  H->ly = h.ly;
  if (!H->host_only) {
    try {
      upload(H.get(), (hipStream_t)hip_stream);
      tune(H.get(), (hipStream_t)hip_stream);
      capture_graphs(H.get());
      if (H->my > 0) fourier_tables(H.get(), (hipStream_t)hip_stream);
    } catch (const std::bad_alloc &) {
      return fail(SMPM_ENOMEM, "device allocation failed while loading tables");
    } catch (const std::exception &e) {
      return fail(SMPM_EHIP, e.what());
    }
  }
  *out = H.release();
  return SMPM_OK;
}

smpm_status smpm_solve_fourier(smpm_handle *H, const double *f, const double *g, double *u, void *hip_stream,
                               smpm_stats *stats) {
  if (!H) return fail(SMPM_EINVAL, "handle is NULL");
  if (H->my == 0) return fail(SMPM_EINVAL, "not a Fourier handle (smpm_setup_fourier)");
  if (H->host_only) return fail(SMPM_EUNSUPPORTED, "host-only handle");
  if (!f || !u) return fail(SMPM_EINVAL, "f or u is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  const int nk2 = 2 * (H->my / 2 + 1);
  const System &s0 = H->sys[0];
  const int64_t r = s0.r, gsz = 2LL * s0.n * (s0.mx + s0.mz);
  (void)nk2;
  transform_y(H, false, f, H->fhat, r, st);
  if (g) transform_y(H, false, g, H->ghat, gsz, st);
  if (hipGetLastError() != hipSuccess) return fail(SMPM_EHIP, "transform launch failed");
  const smpm_status status = smpm_solve(H, H->fhat, g ? H->ghat : nullptr, H->uhat, hip_stream, stats);
  if (status == SMPM_OK || status == SMPM_ENOTCONV || status == SMPM_ENONFINITE) {
    transform_y(H, true, H->uhat, u, r, st);
    if (hipGetLastError() != hipSuccess) return fail(SMPM_EHIP, "transform launch failed");
  }
  return status;
}

smpm_status smpm_transform_y(smpm_handle *H, int32_t inverse, const double *in, double *out, void *hip_stream) {
  if (!H) return fail(SMPM_EINVAL, "handle is NULL");
  if (H->my == 0) return fail(SMPM_EINVAL, "not a Fourier handle (smpm_setup_fourier)");
  if (H->host_only) return fail(SMPM_EUNSUPPORTED, "host-only handle");
  if (!in || !out || in == out) return fail(SMPM_EINVAL, "in or out is NULL, or they are the same array");
  transform_y(H, inverse != 0, in, out, H->sys[0].r, (hipStream_t)hip_stream);
  if (hipGetLastError() != hipSuccess) return fail(SMPM_EHIP, "transform launch failed");
  return SMPM_OK;
}

// Relative Schur residual of instance i from the reduced pairs (|r|^2,
// u_S . r) and (|b~|^2, .): at k = 0 the part of r in range(S) = u_S-perp,
// |r|^2 - (u_S . r)^2 (u_S has unit norm), since the regularized system's
// residual lies there in exact arithmetic and its u_S component is the
// rounding of u_S and of S x_S, which no iterate reduces (reported apart).
static double range_residual(const smpm_handle *H, int i) {
  const double nb = std::sqrt(H->h_nb[2 * i]);
  if (!(nb > 0)) return 0.0;
  double rr = H->h_pairs[2 * i];
  if (H->sys[H->h_ins[i].sys].singular) rr = std::max(rr - H->h_pairs[2 * i + 1] * H->h_pairs[2 * i + 1], 0.0);
  return std::sqrt(rr) / nb;
}

smpm_status smpm_solve(smpm_handle *H, const double *f, const double *g, double *u, void *hip_stream,
                       smpm_stats *stats) {
  if (!H) return fail(SMPM_EINVAL, "handle is NULL");
  if (H->host_only) return fail(SMPM_EUNSUPPORTED, "host-only handle");
  if (!f || !u) return fail(SMPM_EINVAL, "f or u is NULL");
  hipStream_t caller = (hipStream_t)hip_stream;
  hipStream_t st = H->ws;
  const auto t0 = std::chrono::steady_clock::now();
  smpm_stats S{};
  S.instances = H->ninst;
  try {
    HIPCHECK(hipEventRecord(H->ev_in, caller));
    HIPCHECK(hipStreamWaitEvent(st, H->ev_in, 0));
    const bool useP = H->method == SMPM_METHOD_DBJ;
    bool nonfinite = false, notconv = false;
    int sweeps = 0, batch_run = 0;
    if (H->precision == SMPM_FP64) {
      // Head graph, the predicted iterations, then the tail graph (the
      // loop's end, the final FP64 check of the Schur residual, the
      // recovery of u) and the report, with one synchronization.  The tail
      // only overwrites its outputs and leaves the Krylov state alone, so
      // if an instance is still iterating the loop resumes and the tail is
      // enqueued again.
      capture_graphs(H);   // done at setup: nothing to capture here
      read_rhs(H, f, g, st);
      HIPCHECK(hipGraphLaunch(H->g_head, st));
      int launched = Inner<double>::predicted(H, 0, st);
      const bool had_pred = H->pred_iters[0] >= 0;
      for (int pass = 0;; ++pass) {
        if (pass == 1 && had_pred) H->pred_margin[0] = 1;   // the prediction fell short
        HIPCHECK(hipGraphLaunch(H->g_tail, st));
        write_u(H, u, st);   // again after a later tail if the loop resumes
        HIPCHECK(hipMemcpyAsync(H->h_rep, H->gs, H->rep_bytes, hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        const GState *hg = reinterpret_cast<const GState *>(H->h_rep);
        bool active = false;
        for (int i = 0; i < H->ninst; ++i) active |= hg[i].active != 0;
        if (!active || launched >= H->maxit) break;
        const int n = std::min(kIterChunk, H->maxit - launched);
        Inner<double>::iterations(H, n, st);
        Inner<double>::until_done(H, launched + n, st);
        launched = H->maxit;   // every instance has stopped: this tail is the last
      }
      const size_t gs_b = sizeof(GState) * H->ninst;
      std::memcpy(H->h_gs_hist, H->h_rep, gs_b);
      std::memcpy(H->h_pairs, H->h_rep + gs_b, sizeof(double) * 2 * H->ninst);
      std::memcpy(H->h_defect, H->h_rep + gs_b + sizeof(double) * 2 * H->ninst, sizeof(double) * H->ninst);
      std::memcpy(H->h_nb, H->h_rep + gs_b + sizeof(double) * 3 * H->ninst, sizeof(double) * 2 * H->ninst);
      sweeps = 1;
      S.schur_matvecs += H->ninst * ((useP ? 1 : 0) + 1);
    } else {
      capture_graphs(H);   // done at setup: nothing to capture here
      read_rhs(H, f, g, st);
      HIPCHECK(hipGraphLaunch(H->g_stage, st));
      HIPCHECK(hipMemcpyAsync(H->h_nb, H->pairs, sizeof(double) * 2 * H->ninst, hipMemcpyDeviceToHost, st));
      // As many sweeps as the previous solve took, each with its predicted
      // inner iterations, enqueued back to back without a host check; the
      // residual is checked after them and the checked sweeps below go on
      // if it is not small enough.
      const int batch = std::min(H->pred_nsweeps, H->max_sweeps);
      batch_run = batch;
      for (; sweeps < batch; ++sweeps) {
        if (sweeps > 0) {
          HIPCHECK(hipGraphLaunch(H->g_resid, st));
          S.schur_matvecs += H->ninst;
        }
        Inner<float>::run_fixed(H, sweeps, st);
        S.schur_matvecs += useP ? H->ninst : 0;
      }
      double prev_worst = 1.0, prev2_worst = 1.0;
      for (;; ++sweeps) {
        if (sweeps > 0) {
          HIPCHECK(hipGraphLaunch(H->g_resid, st));
          S.schur_matvecs += H->ninst;
          HIPCHECK(hipMemcpyAsync(H->h_pairs, H->pairs, sizeof(double) * 2 * H->ninst, hipMemcpyDeviceToHost, st));
          HIPCHECK(hipStreamSynchronize(st));
          bool done = true;
          double worst = 0.0;
          for (int i = 0; i < H->ninst; ++i) {
            const double rel = range_residual(H, i);
            if (!std::isfinite(rel)) nonfinite = true;
            if (rel > H->tol) done = false;
            worst = std::max(worst, rel);
          }
          if (done || nonfinite) break;
          // stagnation: a sweep that does not cut the worst residual by 10%
          // will not reach the tolerance (the inner operator is too inexact)
          if (worst > kStagnation * prev_worst) { notconv = true; break; }
          // nor will one whose rate over the last two sweeps, kept up, needs
          // more sweeps than are left
          if (sweeps >= 3 && worst > 0.0) {
            const double need = 2.0 * std::log(H->tol / worst) / std::log(worst / prev2_worst);
            if (sweeps + need > H->max_sweeps) { notconv = true; break; }
          }
          prev2_worst = prev_worst;
          prev_worst = worst;
        }
        if (sweeps >= H->max_sweeps) { notconv = true; break; }
        Inner<float>::run(H, sweeps, st);
        S.schur_matvecs += useP ? H->ninst : 0;
      }
      HIPCHECK(hipMemcpyAsync(H->h_defect, H->defect, sizeof(double) * H->ninst, hipMemcpyDeviceToHost, st));
      HIPCHECK(hipGraphLaunch(H->g_finish, st));
      write_u(H, u, st);
    }
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipEventRecord(H->ev_out, st));
    HIPCHECK(hipStreamWaitEvent(caller, H->ev_out, 0));
    HIPCHECK(hipStreamSynchronize(st));
    // iteration statistics of every inner solve
    const int P = H->precision == SMPM_FP64 ? 0 : 1;
    const int nslots = H->precision == SMPM_FP64 ? 1 : std::min(sweeps, H->max_sweeps);
    int itmax_all = 0;
    if (P == 1) H->pred_sweep.assign(nslots, -1);
    for (int sw = 0; sw < nslots; ++sw)
      for (int i = 0; i < H->ninst; ++i) {
        const GState &gsi = H->h_gs_hist[(size_t)sw * H->ninst + i];
        S.iters_total += gsi.iter;
        S.schur_matvecs += gsi.iter;
        S.iters_max = std::max(S.iters_max, gsi.iter);
        itmax_all = std::max(itmax_all, gsi.iter);
        // an inner solve cut short by its prediction gets a chunk more next time
        if (P == 1) H->pred_sweep[sw] = std::max(H->pred_sweep[sw], gsi.iter + (gsi.active ? kIterChunk : 0));
        if (gsi.status == 3) nonfinite = true;
        if (gsi.status == 2 && H->precision == SMPM_FP64) notconv = true;
      }
    H->pred_iters[P] = itmax_all;
    S.sweeps_max = H->precision == SMPM_FP64 ? 1 : sweeps;
    double relmax = 0.0, defmax = 0.0, nullmax = 0.0;
    int conv = 0;
    for (int i = 0; i < H->ninst; ++i) {
      const double nb = std::sqrt(H->h_nb[2 * i]);
      const double rel = range_residual(H, i);
      if (!std::isfinite(rel)) nonfinite = true;
      relmax = std::max(relmax, rel);
      if (H->sys[H->h_ins[i].sys].singular) {
        defmax = std::max(defmax, H->h_defect[i]);
        if (nb > 0) nullmax = std::max(nullmax, std::fabs(H->h_pairs[2 * i + 1]) / nb);
      }
      if (rel <= H->tol * 1.001) ++conv;
    }
    S.rel_residual_max = relmax;
    S.null_residual_max = nullmax;
    S.compat_defect_max = defmax;
    S.converged = conv;
    S.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = S;
    // the next refinement solve runs this many sweeps unchecked: only after
    // a converged one
    // After checked sweeps beyond the unchecked ones (some inner solve was cut
    // short by its prediction), keep the unchecked count: the grown per-sweep
    // predictions and the margin make those sweeps suffice next time.
    if (P == 1) {
      const bool extra = batch_run > 0 && sweeps > batch_run;
      if (extra) H->pred_margin[1] = 1;
      H->pred_nsweeps = (nonfinite || notconv) ? 0 : (extra ? batch_run : nslots);
    }
    if (nonfinite) return fail(SMPM_ENONFINITE, "non-finite value in the inputs or iterates");
    if (notconv) return fail(SMPM_ENOTCONV, "iteration limit reached before the tolerance");
  } catch (const std::exception &e) {
    if (stats) *stats = S;
    return fail(SMPM_EHIP, e.what());
  }
  return SMPM_OK;
}

smpm_status smpm_apply(smpm_handle *H, smpm_op op, int32_t sysi, const void *x, void *y, int32_t precision,
                       void *hip_stream) {
  if (!H) return fail(SMPM_EINVAL, "handle is NULL");
  if (H->host_only) return fail(SMPM_EUNSUPPORTED, "host-only handle");
  if (sysi < 0 || sysi >= (int)H->sys.size()) return fail(SMPM_EINVAL, "system index out of range");
  if (!x || !y) return fail(SMPM_EINVAL, "x or y is NULL");
  if (precision != SMPM_FP64 && !(precision == SMPM_FP32_IR && (op == SMPM_OP_SCHUR || op == SMPM_OP_BJINV)))
    return fail(SMPM_EINVAL, "only SCHUR and BJINV have FP32 variants");
  hipStream_t st = (hipStream_t)hip_stream;
  const int inst = sysi * H->nrhs;
  const InstDev &I = H->h_ins[inst];
  const System &s = H->sys[sysi];
  int nxc = 0, nhc = 0;
  const int2 *wx = xwork(H, inst, nxc);
  const int2 *wh = hwork(H, inst, nhc);
  const size_t bx = sizeof(double) * s.kS, br = sizeof(double) * s.r;
  try {
    switch (op) {
      case SMPM_OP_SCHUR:
      case SMPM_OP_BJINV: {
        const int kop = op == SMPM_OP_SCHUR ? 0 : 1;
        if (precision == SMPM_FP64) {
          HIPCHECK(hipMemcpyAsync(H->t64 + I.x_off, x, bx, hipMemcpyDeviceToDevice, st));
          gemv<double, double, double>(H, kop, H->t64, 0, nullptr, H->y64, nullptr, nullptr, st, inst);
          HIPCHECK(hipMemcpyAsync(y, H->y64 + I.x_off, bx, hipMemcpyDeviceToDevice, st));
        } else {
          HIPCHECK(hipMemcpyAsync(H->t32 + I.x_off, x, sizeof(float) * s.kS, hipMemcpyDeviceToDevice, st));
          gemv<float, float, float>(H, kop, H->t32, 0, nullptr, H->y32, nullptr, nullptr, st, inst);
          HIPCHECK(hipMemcpyAsync(y, H->y32 + I.x_off, sizeof(float) * s.kS, hipMemcpyDeviceToDevice, st));
        }
        break;
      }
      case SMPM_OP_DEFLATE_P: {   // P x = x - (S Z) G Z^T x
        HIPCHECK(hipMemcpyAsync(H->t64 + I.x_off, x, bx, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(k_zt<double>, dim3(nhc), dim3(kBlock), 0, st, H->d_sys, H->d_ins, wh, (const double *)H->t64, 0,
                           (const double *)nullptr, (const GState *)nullptr, H->hs);
        hipLaunchKernelGGL(k_coarse, dim3(1, ctiles(H)), dim3(kBlock), sizeof(double) * H->dmax, st, H->d_sys, H->d_ins + inst, (const double *)H->hs,
                           (const double *)nullptr, (double *)nullptr, H->cv, (const GState *)nullptr);
        hipLaunchKernelGGL(k_xupdate<double>, dim3(nxc), dim3(kBlock), 0, st, H->d_sys, H->d_ins, wx, 3,
                           (const double *)H->t64, (const double *)H->cv, H->y64, (double *)nullptr,
                           (const double *)nullptr);
        HIPCHECK(hipMemcpyAsync(y, H->y64 + I.x_off, bx, hipMemcpyDeviceToDevice, st));
        break;
      }
      case SMPM_OP_DEFLATE_Q: {   // Q x = x - Z G Z^T S x
        HIPCHECK(hipMemcpyAsync(H->t64 + I.x_off, x, bx, hipMemcpyDeviceToDevice, st));
        gemv<double, double, double>(H, 0, H->t64, 0, nullptr, H->y64, H->zlabel == 0 ? H->hs : nullptr, nullptr, st,
                                     inst);
        if (H->zlabel != 0)
          hipLaunchKernelGGL(k_zt<double>, dim3(nhc), dim3(kBlock), 0, st, H->d_sys, H->d_ins, wh,
                             (const double *)H->y64, 0, (const double *)nullptr, (const GState *)nullptr, H->hs);
        hipLaunchKernelGGL(k_coarse, dim3(1, ctiles(H)), dim3(kBlock), sizeof(double) * H->dmax, st, H->d_sys, H->d_ins + inst, (const double *)H->hs,
                           (const double *)nullptr, (double *)nullptr, H->cv, (const GState *)nullptr);
        hipLaunchKernelGGL(k_xupdate<double>, dim3(nxc), dim3(kBlock), 0, st, H->d_sys, H->d_ins, wx, 4,
                           (const double *)H->t64, (const double *)H->cv, H->z64, (double *)nullptr,
                           (const double *)nullptr);
        HIPCHECK(hipMemcpyAsync(y, H->z64 + I.x_off, bx, hipMemcpyDeviceToDevice, st));
        break;
      }
      case SMPM_OP_AINV:
        HIPCHECK(hipMemcpyAsync(H->F + I.f_off, x, br, hipMemcpyDeviceToDevice, st));
        ainv(H, H->F, H->v, st, inst);
        HIPCHECK(hipMemcpyAsync(y, H->v + I.f_off, br, hipMemcpyDeviceToDevice, st));
        break;
      case SMPM_OP_B:
        HIPCHECK(hipMemcpyAsync(H->v + I.f_off, x, br, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(k_bS, dim3(nhc), dim3(kBlock), 0, st, H->d_sys, H->d_ins, wh, (const double *)H->v, H->y64, H->hs);
        HIPCHECK(hipMemcpyAsync(y, H->y64 + I.x_off, bx, hipMemcpyDeviceToDevice, st));
        break;
      case SMPM_OP_SCHUR_RHS:
        return fail(SMPM_EINVAL, "SCHUR_RHS is applied through smpm_solve's staging only");
      default:
        return fail(SMPM_EINVAL, "unknown operator");
    }
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(st));
  } catch (const std::exception &e) {
    return fail(SMPM_EHIP, e.what());
  }
  return SMPM_OK;
}

smpm_status smpm_schur_apply_all(smpm_handle *H, const void *x, void *y, int32_t precision, void *hip_stream) {
  if (!H) return fail(SMPM_EINVAL, "handle is NULL");
  if (H->host_only) return fail(SMPM_EUNSUPPORTED, "host-only handle");
  if (!x || !y) return fail(SMPM_EINVAL, "x or y is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  if (precision == SMPM_FP64)
    gemv<double, double, double>(H, 0, (const double *)x, 0, nullptr, (double *)y, nullptr, nullptr, st);
  else if (precision == SMPM_FP32_IR)
    gemv<float, float, float>(H, 0, (const float *)x, 0, nullptr, (float *)y, nullptr, nullptr, st);
  else if (precision == SMPM_FP16S_IR && H->op16)
    gemv<float, float, float>(H, 0, (const float *)x, 0, nullptr, (float *)y, nullptr, nullptr, st, -1, true);
  else
    return fail(SMPM_EINVAL, "unknown precision");
  if (hipGetLastError() != hipSuccess) return fail(SMPM_EHIP, "kernel launch failed");
  return SMPM_OK;
}

smpm_status smpm_apply_all(smpm_handle *H, smpm_op op, const void *x, void *y, int32_t precision,
                           void *hip_stream) {
  if (!H) return fail(SMPM_EINVAL, "handle is NULL");
  if (H->host_only) return fail(SMPM_EUNSUPPORTED, "host-only handle");
  if (!x || !y || x == y) return fail(SMPM_EINVAL, "x or y is NULL, or x and y are the same array");
  const bool p16 = precision == SMPM_FP16S_IR;
  if (precision != SMPM_FP64 && precision != SMPM_FP32_IR && !p16) return fail(SMPM_EINVAL, "unknown precision");
  if (p16 && !H->op16) return fail(SMPM_EINVAL, "FP16 tables exist on SMPM_FP16S_IR handles only");
  if (op == SMPM_OP_AINV && precision != SMPM_FP64) return fail(SMPM_EINVAL, "AINV is FP64 only");
  hipStream_t st = (hipStream_t)hip_stream;
  try {
    switch (op) {
      case SMPM_OP_SCHUR:
      case SMPM_OP_BJINV: {
        const int kop = op == SMPM_OP_SCHUR ? 0 : 1;
        if (precision == SMPM_FP64)
          gemv<double, double, double>(H, kop, (const double *)x, 0, nullptr, (double *)y, nullptr, nullptr, st);
        else
          gemv<float, float, float>(H, kop, (const float *)x, 0, nullptr, (float *)y, nullptr, nullptr, st, -1, p16);
        break;
      }
      case SMPM_OP_SCHUR_BJINV: {   // the GMRES iteration's operator, as the solve applies it
        const int pr = precision == SMPM_FP64 ? 0 : (p16 ? 2 : 1);
        if (precision == SMPM_FP64) {
          if (H->use_fused[pr]) {
            gemv<double, double, double>(H, 2, (const double *)x, 0, nullptr, (double *)y, nullptr, nullptr, st);
          } else {
            gemv<double, double, double>(H, 1, (const double *)x, 0, nullptr, H->z64, nullptr, nullptr, st);
            gemv<double, double, double>(H, 0, (const double *)H->z64, 0, nullptr, (double *)y, nullptr, nullptr, st);
          }
        } else if (H->use_fused[pr]) {
          gemv<float, float, float>(H, 2, (const float *)x, 0, nullptr, (float *)y, nullptr, nullptr, st, -1, p16);
        } else {
          gemv<float, float, float>(H, 1, (const float *)x, 0, nullptr, H->z32, nullptr, nullptr, st, -1, p16);
          gemv<float, float, float>(H, 0, (const float *)H->z32, 0, nullptr, (float *)y, nullptr, nullptr, st, -1, p16);
        }
        break;
      }
      case SMPM_OP_AINV:
        ainv(H, (const double *)x, (double *)y, st);
        break;
      default:
        return fail(SMPM_EINVAL, "smpm_apply_all takes SCHUR, BJINV, SCHUR_BJINV or AINV");
    }
    HIPCHECK(hipGetLastError());
  } catch (const std::exception &e) {
    return fail(SMPM_EHIP, e.what());
  }
  return SMPM_OK;
}

int32_t smpm_num_systems(const smpm_handle *H) { return H ? (int32_t)H->sys.size() : 0; }

smpm_status smpm_query(const smpm_handle *H, int32_t sysi, smpm_info *info) {
  if (!H || !info) return fail(SMPM_EINVAL, "NULL argument");
  if (sysi < 0 || sysi >= (int)H->sys.size()) return fail(SMPM_EINVAL, "system index out of range");
  const System &s = H->sys[sysi];
  smpm_info o{};
  o.n = s.n; o.mx = s.mx; o.mz = s.mz; o.nrhs = H->nrhs; o.r = s.r; o.kS = s.kS; o.d = s.d;
  o.kwave = s.kwave; o.tau = s.tau;
  int64_t f = 0, g = 0, x = 0;
  for (int q = 0; q < sysi; ++q) {
    const System &p = H->sys[q];
    f += p.r * H->nrhs; g += 2LL * p.n * (p.mx + p.mz) * H->nrhs; x += p.kS * H->nrhs;
  }
  o.f_offset = f; o.g_offset = g; o.x_offset = x;
  o.unique_W = s.nW; o.unique_M = s.nM;
  o.bytes_W64 = (int64_t)s.nW * s.N * 2 * s.N * 8;   // distinct Schur half blocks, FP64
  o.bytes_M64 = (int64_t)s.nM * s.N * 4 * s.N * 8;   // distinct block-Jacobi row chunks, FP64
  for (int op = 0; op < 2; ++op)
    for (int pr = 0; pr < 2; ++pr)
      o.gemm_sched[2 * op + pr] = H->gl[op][0].n > 0 ? H->sched[op][pr == 1 && H->op16 ? 2 : pr] : -1;
  for (int k = 0; k < 3; ++k)
    for (int w = 0; w < 2; ++w) o.elem_sched[2 * k + w] = H->n_cg_all[k][w] > 0 ? H->cg_sched[k][w] : -1;
  for (int k = 0; k < 3; ++k) o.elem_alt[k] = H->cg_alt_sched[k];
  for (int pr = 0; pr < 3; ++pr) {
    o.fused_op[pr] = H->use_fused[pr] ? 1 : 0;
    o.fused_sched[pr] = H->gl[2][0].n > 0 ? H->sched[2][pr] : -1;
  }
  o.setup_device = s.dev_steps;
  o.rhs_gemm[0] = H->use_ba ? H->ba_sched : -1;
  o.rhs_gemm[1] = H->use_ba ? (H->ba_list ? 16 : kGemmVecs) : -1;
  for (int op = 0; op < 2; ++op)
    for (int pr = 0; pr < 2; ++pr) {
      const int p = pr == 1 && H->op16 ? 2 : pr;
      o.gemm_list[2 * op + pr] = H->gl[op][0].n > 0 ? (H->g_list[op][p] ? 16 : kGemmVecs) : -1;
    }
  // Algorithmic operator sizes: nonzero entries only (a Schur block's
  // column half for a window half outside the interface range is stored as
  // zeros and not counted), distinct blocks once.
  const int N = s.N, nh = s.nh;
  const size_t wsz = (size_t)N * 2 * N;
  for (int b = 0; b < s.nW; ++b)
    for (int c = 0; c < 2; ++c) {
      bool nz = false;
      for (int i = 0; i < N && !nz; ++i)
        for (int q = 0; q < N && !nz; ++q) nz = s.Wblk[b * wsz + (size_t)i * 2 * N + c * N + q] != 0.0;
      if (nz) o.nnz_W_unique += (int64_t)N * N;
    }
  std::vector<int> mK(s.nM / 4, 0), fK(s.nF, 0);
  for (int h = 0; h < nh; ++h) {
    for (int p = 0; p < 2; ++p) {
      const int wh = s.w_win[h] + p;
      if (wh >= 0 && wh < nh) o.nnz_W_total += (int64_t)N * N;
    }
    o.nnz_M_total += (int64_t)N * s.m_K[h];
    mK[s.m_id[h] / 4] = s.m_K[h];
    if (s.nF > 0) {
      o.nnz_F_total += (int64_t)N * s.f_K[h];
      fK[s.f_id[h]] = s.f_K[h];
    }
  }
  for (int K : mK) o.nnz_M_unique += (int64_t)K * K;
  for (int K : fK) o.nnz_F_unique += (int64_t)N * K;
  o.strip_classes = (int32_t)s.classes.size();
  const size_t bsz = (size_t)s.n2 * s.n2;
  for (const StripClass &c : s.classes)   // element inverses equal bit for bit are stored once
    for (int e = 0; e < s.mz; ++e) {
      bool seen = false;
      for (int f = 0; f < e && !seen; ++f)
        seen = !std::memcmp(c.Dinv.data() + f * bsz, c.Dinv.data() + e * bsz, sizeof(double) * bsz);
      if (!seen) ++o.elem_unique;
    }
  *info = o;
  return SMPM_OK;
}

smpm_status smpm_export(const smpm_handle *H, smpm_table what, int32_t sysi, double *out, int64_t count) {
  if (!H || !out) return fail(SMPM_EINVAL, "NULL argument");
  if (sysi < 0 || sysi >= (int)H->sys.size()) return fail(SMPM_EINVAL, "system index out of range");
  const System &s = H->sys[sysi];
  auto need = [&](int64_t n) -> bool { return count == n; };
  switch (what) {
    case SMPM_TABLE_SCHUR_DENSE: {
      if (!need(s.kS * s.kS)) return fail(SMPM_EINVAL, "count must be k_S^2");
      std::fill(out, out + count, 0.0);
      for (int h = 0; h < s.nh; ++h)
        for (int i = 0; i < s.N; ++i) {
          const int64_t row = (int64_t)h * s.N + i;
          out[row * s.kS + row] += 1.0;
          for (int c = 0; c < 2 * s.N; ++c) {
            const int64_t col = (int64_t)s.w_win[h] * s.N + c;
            if (col < 0 || col >= s.kS) continue;
            out[row * s.kS + col] += s.Wblk[(size_t)s.w_id[h] * s.N * 2 * s.N + (size_t)i * 2 * s.N + c];
          }
        }
      return SMPM_OK;
    }
    case SMPM_TABLE_BJINV_DENSE: {
      if (!need(s.kS * s.kS)) return fail(SMPM_EINVAL, "count must be k_S^2");
      std::fill(out, out + count, 0.0);
      for (int h = 0; h < s.nh; ++h)
        for (int i = 0; i < s.N; ++i) {
          const int64_t row = (int64_t)h * s.N + i;
          for (int c = 0; c < s.m_K[h]; ++c) {
            const int64_t col = (int64_t)s.m_win[h] * s.N + c;
            out[row * s.kS + col] = s.Mblk[(size_t)s.m_id[h] * s.N * 4 * s.N + (size_t)i * 4 * s.N + c];
          }
        }
      return SMPM_OK;
    }
    case SMPM_TABLE_SMINV_DENSE: {
      if (s.nF == 0) return fail(SMPM_EUNSUPPORTED, "no fused S M^-1 blocks (strips do not share blocks)");
      if (!need(s.kS * s.kS)) return fail(SMPM_EINVAL, "count must be k_S^2");
      std::fill(out, out + count, 0.0);
      for (int h = 0; h < s.nh; ++h)
        for (int i = 0; i < s.N; ++i) {
          const int64_t row = (int64_t)h * s.N + i;
          for (int c = 0; c < s.f_K[h]; ++c)
            out[row * s.kS + (int64_t)s.f_win[h] * s.N + c] = s.Fblk[((size_t)s.f_id[h] * s.N + i) * 8 * s.N + c];
        }
      return SMPM_OK;
    }
    case SMPM_TABLE_COARSE_C:
      if (!need((int64_t)s.d * s.d)) return fail(SMPM_EINVAL, "count must be d^2");
      std::copy(s.C.begin(), s.C.end(), out);
      return SMPM_OK;
    case SMPM_TABLE_U_S:
    case SMPM_TABLE_U_L:
    case SMPM_TABLE_U_C: {
      if (!s.singular) return fail(SMPM_EINVAL, "null vectors exist for k = 0 only");
      const std::vector<double> &v = what == SMPM_TABLE_U_S ? s.uS : what == SMPM_TABLE_U_L ? s.uL : s.uC;
      if (!need((int64_t)v.size())) return fail(SMPM_EINVAL, "count mismatch");
      std::copy(v.begin(), v.end(), out);
      return SMPM_OK;
    }
    case SMPM_TABLE_SZ: {
      if (!need(s.kS * s.d)) return fail(SMPM_EINVAL, "count must be k_S * d");
      std::fill(out, out + count, 0.0);
      for (int h = 0; h < s.nh; ++h)
        for (int p = 0; p < 2 * s.zm; ++p) {
          const int col = s.sz_col[(size_t)h * 2 * s.zm + p];
          if (col < 0) continue;
          for (int i = 0; i < s.N; ++i)
            out[((int64_t)h * s.N + i) * s.d + col] = s.SZh[((size_t)h * 2 * s.zm + p) * s.N + i];
        }
      return SMPM_OK;
    }
  }
  return fail(SMPM_EINVAL, "unknown table");
}

void smpm_destroy(smpm_handle *H) { delete H; }

const char *smpm_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Operator applies without any allocation, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).  The
// intermediate vectors of smpm_apply (the Z^T partial sums, the coarse
// vector, the S x of Q) live in one file-scope device array instead of the
// handle's workspace, and x and y are read and written in place.

namespace {

constexpr size_t kScratchDoubles = size_t(1) << 21;   // 16 MiB per device
constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[kScratchDoubles];

// The array's device address, looked up once per device with that device
// current (each device holds its own copy of the array).
double *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

double *scratch_address(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) throw std::runtime_error(std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  return g_scratch_ptr[dev];
}

// A base pointer whose element `off` is p[0]: the kernels address one
// instance's vectors through absolute batched offsets.
template <typename T>
T *rebase(T *p, int64_t off) {
  return reinterpret_cast<T *>(reinterpret_cast<uintptr_t>(p) - (uintptr_t)(off * (int64_t)sizeof(T)));
}

}  // namespace

extern "C" {

smpm_status smpm_apply_noalloc(smpm_handle *H, smpm_op op, int32_t sysi, const void *x, void *y,
                               int32_t precision, void *hip_stream) {
  if (!H) return fail(SMPM_EINVAL, "handle is NULL");
  if (H->host_only) return fail(SMPM_EUNSUPPORTED, "host-only handle");
  if (sysi < 0 || sysi >= (int)H->sys.size()) return fail(SMPM_EINVAL, "system index out of range");
  if (!x || !y || x == y) return fail(SMPM_EINVAL, "x or y is NULL, or x and y are the same array");
  if (op != SMPM_OP_SCHUR && op != SMPM_OP_BJINV && op != SMPM_OP_DEFLATE_P && op != SMPM_OP_DEFLATE_Q)
    return fail(SMPM_EINVAL, "smpm_apply_noalloc takes SCHUR, BJINV, DEFLATE_P or DEFLATE_Q");
  if (precision != SMPM_FP64 && !(precision == SMPM_FP32_IR && (op == SMPM_OP_SCHUR || op == SMPM_OP_BJINV)))
    return fail(SMPM_EINVAL, "only SCHUR and BJINV have FP32 variants");
  hipStream_t st = (hipStream_t)hip_stream;
  const int inst = sysi * H->nrhs;
  const InstDev &I = H->h_ins[inst];
  const System &s = H->sys[sysi];
  // scratch layout: [S x (k_S) | Z^T partial sums | coarse vector (d)]
  const int64_t nhs = (int64_t)s.nh * (s.zm > 1 ? s.zm : (s.N + 15) / 16);
  const int64_t need = s.kS + nhs + s.d;
  if (need > (int64_t)kScratchDoubles)
    return fail(SMPM_EINVAL, "system too large for the fixed scratch of smpm_apply_noalloc (" +
                                 std::to_string(need) + " > " + std::to_string(kScratchDoubles) + " doubles)");
  try {
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SMPM_EINVAL, "device index above the supported 64");
    double *sc = scratch_address(dev);
    double *zs = sc, *hs = sc + s.kS, *cv = hs + nhs;
    double *hsb = rebase(hs, I.hs_off), *cvb = rebase(cv, I.c_off);
    int nxc = 0, nhc = 0;
    const int2 *wx = xwork(H, inst, nxc);
    const int2 *wh = hwork(H, inst, nhc);
    switch (op) {
      case SMPM_OP_SCHUR:
      case SMPM_OP_BJINV: {
        const int kop = op == SMPM_OP_SCHUR ? 0 : 1;
        if (precision == SMPM_FP64)
          gemv<double, double, double>(H, kop, rebase((const double *)x, I.x_off), 0, nullptr,
                                       rebase((double *)y, I.x_off), nullptr, nullptr, st, inst);
        else
          gemv<float, float, float>(H, kop, rebase((const float *)x, I.x_off), 0, nullptr,
                                    rebase((float *)y, I.x_off), nullptr, nullptr, st, inst);
        break;
      }
      case SMPM_OP_DEFLATE_P: {   // P x = x - (S Z) G Z^T x
        const double *xb = rebase((const double *)x, I.x_off);
        hipLaunchKernelGGL(k_zt<double>, dim3(nhc), dim3(kBlock), 0, st, H->d_sys, H->d_ins, wh, xb, 0,
                           (const double *)nullptr, (const GState *)nullptr, hsb);
        hipLaunchKernelGGL(k_coarse, dim3(1, ctiles(H)), dim3(kBlock), sizeof(double) * H->dmax, st, H->d_sys,
                           H->d_ins + inst, (const double *)hsb, (const double *)nullptr, (double *)nullptr, cvb,
                           (const GState *)nullptr);
        hipLaunchKernelGGL(k_xupdate<double>, dim3(nxc), dim3(kBlock), 0, st, H->d_sys, H->d_ins, wx, 3, xb,
                           (const double *)cvb, rebase((double *)y, I.x_off), (double *)nullptr,
                           (const double *)nullptr);
        break;
      }
      case SMPM_OP_DEFLATE_Q: {   // Q x = x - Z G Z^T S x
        const double *xb = rebase((const double *)x, I.x_off);
        double *zb = rebase(zs, I.x_off);
        gemv<double, double, double>(H, 0, xb, 0, nullptr, zb, H->zlabel == 0 ? hsb : nullptr, nullptr, st, inst);
        if (H->zlabel != 0)
          hipLaunchKernelGGL(k_zt<double>, dim3(nhc), dim3(kBlock), 0, st, H->d_sys, H->d_ins, wh,
                             (const double *)zb, 0, (const double *)nullptr, (const GState *)nullptr, hsb);
        hipLaunchKernelGGL(k_coarse, dim3(1, ctiles(H)), dim3(kBlock), sizeof(double) * H->dmax, st, H->d_sys,
                           H->d_ins + inst, (const double *)hsb, (const double *)nullptr, (double *)nullptr, cvb,
                           (const GState *)nullptr);
        hipLaunchKernelGGL(k_xupdate<double>, dim3(nxc), dim3(kBlock), 0, st, H->d_sys, H->d_ins, wx, 4, xb,
                           (const double *)cvb, rebase((double *)y, I.x_off), (double *)nullptr,
                           (const double *)nullptr);
        break;
      }
      default:
        break;
    }
    HIPCHECK(hipGetLastError());
  } catch (const std::exception &e) {
    return fail(SMPM_EHIP, e.what());
  }
  return SMPM_OK;
}

}  // extern "C"
