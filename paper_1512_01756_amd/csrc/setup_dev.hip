// Device back end of the heavy dense setup steps (Sec. 2.3, 2.4 and 3.2
// tables): the multi-right-hand-side strip solves behind the Schur blocks W,
// batched in-place inverses (block-Jacobi blocks, the coarse matrix) and the
// block-tridiagonal elimination and solves of the u_S inverse iteration, on
// rocSOLVER / rocBLAS.  The host setup calls it through DenseBackend; every
// input and result stays in the host tables' row-major layout, so the two
// paths are interchangeable step by step.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "host.hpp"
#include "setup_dev.hpp"

namespace smpm {

namespace {

void hcheck(hipError_t e, const char *what) {
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

void rcheck(rocblas_status s, const char *what) {
  if (s != rocblas_status_success)
    throw std::runtime_error(std::string(what) + ": rocBLAS status " + std::to_string((int)s));
}

template <typename T>
struct DBuf {
  T *p = nullptr;
  explicit DBuf(size_t n) { hcheck(hipMalloc((void **)&p, sizeof(T) * std::max<size_t>(n, 1)), "hipMalloc"); }
  ~DBuf() {
    if (p) (void)hipFree(p);
  }
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
};

// Cyclic reduction of the block-tridiagonal T (d blocks of M = 2N), all
// column-major on the device.  Level 0 holds T: diagonal blocks A_i, the
// coupling to block i - 1 (B_i) and to block i + 1 (C_i).  One level
// eliminates the odd positions k of the current list: A_k is factored (LU with
// pivots), B_k <- Y_k = A_k^-1 B_k and C_k <- Z_k = A_k^-1 C_k; the even
// positions e become the next level, with A_e - B_e Z_{e-1} - C_e Y_{e+1},
// -B_e Y_{e-1} and -C_e Z_{e+1}.  Every step of a level is one
// strided-batched call over its odd or even blocks, so the d sequential steps
// of a block elimination become log2(d) levels.  The last level is one block,
// factored.
struct CrLevel {
  int m;                             // blocks on this level
  DBuf<double> A, B, C, b;           // m blocks of M x M each; b: m blocks of M (solves)
  DBuf<rocblas_int> ipiv, info;
  CrLevel(int m_, int M)
      : m(m_), A((size_t)m_ * M * M), B((size_t)m_ * M * M), C((size_t)m_ * M * M), b((size_t)m_ * M),
        ipiv((size_t)m_ * M), info(m_) {}
};
struct TriFact {
  int d, N, M;
  std::vector<std::unique_ptr<CrLevel>> lv;
};

// Right-hand sides of element e's boundary injections for cn classes, laid
// out like the host strip solve's X rows of element e ([node l][column j],
// j fastest): 1 at (l = b n, j = e n + b) and (l = b n + n - 1, j = N + e n + b),
// 0 elsewhere.
__global__ void k_inject(double *__restrict__ R, int64_t total, int n, int N, int e) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int nr = 2 * N, n2 = n * n;
  const int64_t per = (int64_t)n2 * nr;
  const int64_t rem = idx % per;
  const int l = (int)(rem / nr), j = (int)(rem % nr);
  const int b = l / n, a = l - b * n;
  double v = 0.0;
  if (a == 0 && j == e * n + b) v = 1.0;
  if (a == n - 1 && j == N + e * n + b) v = 1.0;
  R[idx] = v;
}

}  // namespace

struct DeviceDense {
  std::mutex mu;
  int dev = 0;   // the caller's device at creation: the worker threads of the setup start on device 0
  hipStream_t st = nullptr;
  rocblas_handle h = nullptr;
  DenseBackend be;

  // The stream and the rocBLAS handle are made on first use, so setups that
  // never reach the device back end do not pay for them.  Every entry makes
  // the creating thread's device current on the thread that calls it.
  void ensure() {
    hcheck(hipSetDevice(dev), "hipSetDevice");
    if (h) return;
    hcheck(hipStreamCreate(&st), "hipStreamCreate");
    rcheck(rocblas_create_handle(&h), "rocblas_create_handle");
    rcheck(rocblas_set_stream(h, st), "rocblas_set_stream");
  }

  ~DeviceDense() {
    if (h) (void)rocblas_destroy_handle(h);
    if (st) (void)hipStreamDestroy(st);
  }

  // The stream, the rocBLAS handle and the library kernels, ready before
  // the first step: the first call of a rocSOLVER or rocBLAS routine at a
  // new size class loads its kernels (0.15 s and more each), so the steps
  // run once on small stand-ins of their real sizes (the strip solves of one
  // class of zeros; two inverses of 2 x 2 and of inv_n x inv_n; the
  // elimination over four interfaces of N-row halves and one solve).
  void warm(int n, int mz, int inv_n, int tri_N) {
    try {
      {
        std::lock_guard<std::mutex> lk(mu);
        ensure();
      }
      if (n > 0 && mz > 0) {   // one strip class of zeros
        const int n2 = n * n, N = n * mz;
        std::vector<double> G((size_t)mz * n2 * n2, 0.0), lo((size_t)mz * n, 0.0), up((size_t)mz * n, 0.0),
            bw(n, 0.0), bev(n, 0.0), Wq(4 * (size_t)N * N);
        const double *Gp[1] = {G.data()}, *bwp[1] = {bw.data()}, *bep[1] = {bev.data()};
        double *Wp[4] = {Wq.data(), Wq.data() + (size_t)N * N, Wq.data() + 2 * (size_t)N * N,
                         Wq.data() + 3 * (size_t)N * N};
        strip_schur(1, n, mz, Gp, lo.data(), up.data(), bwp, bep, Wp);
      }
      for (const int n : {2, inv_n}) {
        if (n <= 0) continue;
        std::vector<double> a(2 * (size_t)n * n, 0.0);
        for (int q = 0; q < 2; ++q)
          for (int i = 0; i < n; ++i) a[(size_t)q * n * n + (size_t)i * n + i] = 2.0 + q;
        double *mats[2] = {a.data(), a.data() + (size_t)n * n};
        invert(n, 2, mats);
      }
      if (tri_N > 0) {
        const int d = 4, M = 2 * tri_N;
        std::vector<double> Td((size_t)d * M * M, 0.0), Lo((size_t)d * tri_N * tri_N, 0.0),
            Up((size_t)d * tri_N * tri_N, 0.0), v((size_t)d * M, 1.0);
        for (int q = 0; q < d; ++q)
          for (int i = 0; i < M; ++i) Td[(size_t)q * M * M + (size_t)i * M + i] = 2.0;
        void *f = tri_factor(d, tri_N, Td.data(), Lo.data(), Up.data());
        tri_solve(f, v.data());
        std::lock_guard<std::mutex> lk(mu);
        (void)hipSetDevice(dev);
        delete static_cast<TriFact *>(f);
      }
    } catch (...) {
    }
  }

  // Row-major A is column-major A^T, and inv(A^T) = inv(A)^T: inverting the
  // column-major view in place leaves inv(A) in the row-major layout.
  void invert(int n, int count, double *const *mats) {
    std::lock_guard<std::mutex> lk(mu);
    ensure();
    const size_t nn = (size_t)n * n;
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(count, (int64_t)(1ull << 30) / (int64_t)(nn * 8)));
    DBuf<double> A(nn * chunk);
    DBuf<rocblas_int> ipiv((size_t)n * chunk), info(chunk);
    std::vector<rocblas_int> hinfo(chunk);
    for (int c0 = 0; c0 < count; c0 += chunk) {
      const int cn = std::min(chunk, count - c0);
      for (int q = 0; q < cn; ++q)
        hcheck(hipMemcpyAsync(A.p + q * nn, mats[c0 + q], nn * 8, hipMemcpyHostToDevice, st), "upload");
      rcheck(rocsolver_dgetrf_strided_batched(h, n, n, A.p, n, (rocblas_stride)nn, ipiv.p, n, info.p, cn), "getrf");
      hcheck(hipMemcpyAsync(hinfo.data(), info.p, sizeof(rocblas_int) * cn, hipMemcpyDeviceToHost, st), "info");
      hcheck(hipStreamSynchronize(st), "getrf");
      for (int q = 0; q < cn; ++q)
        if (hinfo[q] != 0) throw std::domain_error("singular matrix in the setup");
      rcheck(rocsolver_dgetri_strided_batched(h, n, A.p, n, (rocblas_stride)nn, ipiv.p, n, info.p, cn), "getri");
      hcheck(hipMemcpyAsync(hinfo.data(), info.p, sizeof(rocblas_int) * cn, hipMemcpyDeviceToHost, st), "info");
      for (int q = 0; q < cn; ++q)
        hcheck(hipMemcpyAsync(mats[c0 + q], A.p + q * nn, nn * 8, hipMemcpyDeviceToHost, st), "download");
      hcheck(hipStreamSynchronize(st), "getri");
      for (int q = 0; q < cn; ++q)
        if (hinfo[q] != 0) throw std::domain_error("singular matrix in the setup");
    }
  }

  // Block elimination T~_0 = T_0, T~_i = T_i - Lo_i X_{i-1}[0..N], X_i =
  // T~_i^-1 [0; Up_i], in order over the interfaces (each step needs the
  // previous one); the d steps are enqueued back to back on one stream.
  void *tri_factor(int d, int N, const double *Td, const double *Lo, const double *Up) {
    std::lock_guard<std::mutex> lk(mu);
    ensure();
    const int M = 2 * N;
    const size_t MM = (size_t)M * M;
    std::unique_ptr<TriFact> f(new TriFact{d, N, M, {}});
    const double one = 1.0, minus = -1.0, zero = 0.0;
    const rocblas_operation nn = rocblas_operation_none;
    // SMPM_SETUP_TIMES: the upload and each level, synchronized, to stderr
    const bool times = std::getenv("SMPM_SETUP_TIMES") != nullptr;
    auto t0 = std::chrono::steady_clock::now();
    auto lap = [&](const char *what, int m) {
      if (!times) return;
      hcheck(hipStreamSynchronize(st), "lap");
      const auto t1 = std::chrono::steady_clock::now();
      std::fprintf(stderr, "  u_S reduction: %-24s m = %4d  %8.1f ms\n", what, m,
                   std::chrono::duration<double, std::milli>(t1 - t0).count());
      t0 = t1;
    };
    // level 0: T's blocks.  The host's row-major blocks go up as they are and
    // are transposed on the device (a row-major block is the column-major
    // transpose); B_i and C_i are zero but for one N x N quadrant (rows and
    // columns 0..N of B_i, N..2N of C_i).
    f->lv.emplace_back(new CrLevel(d, M));
    {
      CrLevel &L0 = *f->lv[0];
      const size_t NN = (size_t)N * N;
      DBuf<double> raw((size_t)d * MM), lo((size_t)d * NN), up((size_t)d * NN);
      hcheck(hipMemcpyAsync(raw.p, Td, sizeof(double) * d * MM, hipMemcpyHostToDevice, st), "upload T");
      hcheck(hipMemcpyAsync(lo.p, Lo, sizeof(double) * d * NN, hipMemcpyHostToDevice, st), "upload Lo");
      hcheck(hipMemcpyAsync(up.p, Up, sizeof(double) * d * NN, hipMemcpyHostToDevice, st), "upload Up");
      hcheck(hipMemsetAsync(L0.B.p, 0, sizeof(double) * d * MM, st), "zero B");
      hcheck(hipMemsetAsync(L0.C.p, 0, sizeof(double) * d * MM, st), "zero C");
      const rocblas_operation tt = rocblas_operation_transpose;
      rcheck(rocblas_dgeam_strided_batched(h, tt, nn, M, M, &one, raw.p, M, MM, &zero, raw.p, M, MM, L0.A.p, M, MM, d),
             "transpose A");
      rcheck(rocblas_dgeam_strided_batched(h, tt, nn, N, N, &one, lo.p + NN, N, NN, &zero, lo.p + NN, N, NN,
                                           L0.B.p + MM, M, MM, d - 1),
             "transpose B");
      rcheck(rocblas_dgeam_strided_batched(h, tt, nn, N, N, &one, up.p, N, NN, &zero, up.p, N, NN,
                                           L0.C.p + (size_t)N * M + N, M, MM, d - 1),
             "transpose C");
      hcheck(hipStreamSynchronize(st), "level 0");   // before the staging buffers go
    }
    lap("upload", d);
    while (f->lv.back()->m > 1) {
      CrLevel &L = *f->lv.back();
      const int m = L.m, mo = m / 2, me = (m + 1) / 2;
      // odd blocks: A_k = LU, Y_k = A_k^-1 B_k, Z_k = A_k^-1 C_k
      rcheck(rocsolver_dgetrf_strided_batched(h, M, M, L.A.p + MM, M, 2 * MM, L.ipiv.p + M, 2 * M, L.info.p, mo),
             "getrf (odd blocks)");
      lap("getrf", m);
      rcheck(rocsolver_dgetrs_strided_batched(h, nn, M, M, L.A.p + MM, M, 2 * MM, L.ipiv.p + M, 2 * M, L.B.p + MM, M,
                                              2 * MM, mo),
             "getrs Y");
      rcheck(rocsolver_dgetrs_strided_batched(h, nn, M, M, L.A.p + MM, M, 2 * MM, L.ipiv.p + M, 2 * M, L.C.p + MM, M,
                                              2 * MM, mo),
             "getrs Z");
      lap("getrs", m);
      f->lv.emplace_back(new CrLevel(me, M));
      CrLevel &Nx = *f->lv.back();
      hcheck(hipMemsetAsync(Nx.B.p, 0, sizeof(double) * me * MM, st), "zero B'");
      hcheck(hipMemsetAsync(Nx.C.p, 0, sizeof(double) * me * MM, st), "zero C'");
      // even blocks e = 2q: A_e -= B_e Z_{e-1} (q >= 1), A_e -= C_e Y_{e+1} (q < mo)
      if (me > 1)
        rcheck(rocblas_dgemm_strided_batched(h, nn, nn, M, M, M, &minus, L.B.p + 2 * MM, M, 2 * MM, L.C.p + MM, M,
                                             2 * MM, &one, L.A.p + 2 * MM, M, 2 * MM, me - 1),
               "gemm A -= B Z");
      rcheck(rocblas_dgemm_strided_batched(h, nn, nn, M, M, M, &minus, L.C.p, M, 2 * MM, L.B.p + MM, M, 2 * MM, &one,
                                           L.A.p, M, 2 * MM, mo),
             "gemm A -= C Y");
      // B'_q = -B_e Y_{e-1} (q >= 1), C'_q = -C_e Z_{e+1} (q < mo)
      if (me > 1)
        rcheck(rocblas_dgemm_strided_batched(h, nn, nn, M, M, M, &minus, L.B.p + 2 * MM, M, 2 * MM, L.B.p + MM, M,
                                             2 * MM, &zero, Nx.B.p + MM, M, MM, me - 1),
               "gemm B'");
      rcheck(rocblas_dgemm_strided_batched(h, nn, nn, M, M, M, &minus, L.C.p, M, 2 * MM, L.C.p + MM, M, 2 * MM, &zero,
                                           Nx.C.p, M, MM, mo),
             "gemm C'");
      hcheck(hipMemcpy2DAsync(Nx.A.p, sizeof(double) * MM, L.A.p, sizeof(double) * 2 * MM, sizeof(double) * MM, me,
                              hipMemcpyDeviceToDevice, st),
             "next level A");
      lap("gemms, next level", m);
    }
    CrLevel &Lc = *f->lv.back();
    rcheck(rocsolver_dgetrf_strided_batched(h, M, M, Lc.A.p, M, MM, Lc.ipiv.p, M, Lc.info.p, 1), "getrf (last)");
    for (size_t l = 0; l < f->lv.size(); ++l) {
      CrLevel &L = *f->lv[l];
      const int cnt = l + 1 == f->lv.size() ? 1 : L.m / 2;
      std::vector<rocblas_int> hinfo(cnt);
      hcheck(hipMemcpyAsync(hinfo.data(), L.info.p, sizeof(rocblas_int) * cnt, hipMemcpyDeviceToHost, st), "info");
      hcheck(hipStreamSynchronize(st), "reduction");
      for (int k = 0; k < cnt; ++k)
        if (hinfo[k] != 0) throw std::runtime_error("singular block in the inverse iteration for u_S");
    }
    return f.release();
  }

  // v <- T^-1 v through the levels: forward, w_k = A_k^-1 b_k on the odd
  // blocks and b_e -= B_e w_{e-1} + C_e w_{e+1} on the even ones, which become
  // the next level's right-hand side; the last block solved; backward, the
  // even blocks take the next level's solution and the odd ones
  // x_k = w_k - Y_k x_{k-1} - Z_k x_{k+1}.
  void tri_solve(void *fp, double *v) {
    std::lock_guard<std::mutex> lk(mu);
    hcheck(hipSetDevice(dev), "hipSetDevice");
    TriFact *f = static_cast<TriFact *>(fp);
    const int M = f->M;
    const size_t MM = (size_t)M * M;
    const double one = 1.0, minus = -1.0;
    const rocblas_operation nn = rocblas_operation_none;
    const int nl = (int)f->lv.size();
    hcheck(hipMemcpyAsync(f->lv[0]->b.p, v, sizeof(double) * f->d * M, hipMemcpyHostToDevice, st), "upload v");
    for (int l = 0; l + 1 < nl; ++l) {
      CrLevel &L = *f->lv[l], &Nx = *f->lv[l + 1];
      const int m = L.m, mo = m / 2, me = (m + 1) / 2;
      rcheck(rocsolver_dgetrs_strided_batched(h, nn, M, 1, L.A.p + MM, M, 2 * MM, L.ipiv.p + M, 2 * M, L.b.p + M, M,
                                              2 * M, mo),
             "getrs w");
      if (me > 1)
        rcheck(rocblas_dgemv_strided_batched(h, nn, M, M, &minus, L.B.p + 2 * MM, M, 2 * MM, L.b.p + M, 1, 2 * M, &one,
                                             L.b.p + 2 * M, 1, 2 * M, me - 1),
               "gemv b -= B w");
      rcheck(rocblas_dgemv_strided_batched(h, nn, M, M, &minus, L.C.p, M, 2 * MM, L.b.p + M, 1, 2 * M, &one, L.b.p, 1,
                                           2 * M, mo),
             "gemv b -= C w");
      hcheck(hipMemcpy2DAsync(Nx.b.p, sizeof(double) * M, L.b.p, sizeof(double) * 2 * M, sizeof(double) * M, me,
                              hipMemcpyDeviceToDevice, st),
             "next level b");
    }
    CrLevel &Lc = *f->lv.back();
    rcheck(rocsolver_dgetrs_strided_batched(h, nn, M, 1, Lc.A.p, M, MM, Lc.ipiv.p, M, Lc.b.p, M, M, 1), "getrs (last)");
    for (int l = nl - 2; l >= 0; --l) {
      CrLevel &L = *f->lv[l], &Nx = *f->lv[l + 1];
      const int m = L.m, mo = m / 2, me = (m + 1) / 2;
      hcheck(hipMemcpy2DAsync(L.b.p, sizeof(double) * 2 * M, Nx.b.p, sizeof(double) * M, sizeof(double) * M, me,
                              hipMemcpyDeviceToDevice, st),
             "even solution");
      rcheck(rocblas_dgemv_strided_batched(h, nn, M, M, &minus, L.B.p + MM, M, 2 * MM, L.b.p, 1, 2 * M, &one,
                                           L.b.p + M, 1, 2 * M, mo),
             "gemv x -= Y x");
      const int nz = (m % 2 == 1) ? mo : mo - 1;   // odd blocks with a right neighbour
      if (nz > 0)
        rcheck(rocblas_dgemv_strided_batched(h, nn, M, M, &minus, L.C.p + MM, M, 2 * MM, L.b.p + 2 * M, 1, 2 * M,
                                             &one, L.b.p + M, 1, 2 * M, nz),
               "gemv x -= Z x");
    }
    hcheck(hipMemcpyAsync(v, f->lv[0]->b.p, sizeof(double) * f->d * M, hipMemcpyDeviceToHost, st), "download v");
    hcheck(hipStreamSynchronize(st), "solve");
  }

  // W quarter blocks (DenseBackend::strip_schur), batched over classes.  The
  // host's row-major X (node rows x 2N columns) is the column-major X^T with
  // leading dimension 2N, and a row-major G_e is the column-major G_e^T, so
  // each step of the block-Thomas solve is one strided-batched call:
  //   forward, e = 0 .. m_z - 1:  R = injections of e;  R[(0, t)] -= sum_c
  //     lo_e[c] X_{e-1}[(c, t)] (a GEMV over the n row groups);  X_e = G_e R;
  //   backward, e = m_z - 2 .. 0:  q[t] = sum_c up_e[c] X_{e+1}[(c, t)];
  //     X_e -= G_e[:, (n-1, t)] q[t];
  // then Wq[r][col][(e, b)][.] = sum_a beta_r[a] X[(e, b, a)][col N + .], one
  // GEMV per element row (e, b).
  void strip_schur(int ncl, int n, int mz, const double *const *G, const double *lo, const double *up,
                   const double *const *betaW, const double *const *betaE, double *const *Wq) {
    std::lock_guard<std::mutex> lk(mu);
    ensure();
    const int n2 = n * n, N = n * mz, nr = 2 * N;
    const size_t gsz = (size_t)mz * n2 * n2, xsz = (size_t)mz * n2 * nr, rsz = (size_t)n2 * nr;
    const size_t per = (gsz + xsz + rsz + (size_t)n * nr + (size_t)N * nr + 2 * n) * sizeof(double);
    const int chunk = (int)std::max<size_t>(1, std::min<size_t>(ncl, (size_t)(2ull << 30) / per));
    DBuf<double> dG(gsz * chunk), dX(xsz * chunk), dR(rsz * chunk), dQ((size_t)n * nr * chunk),
        dY((size_t)N * nr * chunk), dlo((size_t)mz * n), dup((size_t)mz * n), dbeta((size_t)2 * n * chunk);
    hcheck(hipMemcpyAsync(dlo.p, lo, sizeof(double) * mz * n, hipMemcpyHostToDevice, st), "upload lo");
    hcheck(hipMemcpyAsync(dup.p, up, sizeof(double) * mz * n, hipMemcpyHostToDevice, st), "upload up");
    std::vector<double> hY((size_t)N * nr * chunk);
    const double one = 1.0, zero = 0.0, minus = -1.0;
    for (int c0 = 0; c0 < ncl; c0 += chunk) {
      const int cn = std::min(chunk, ncl - c0);
      for (int q = 0; q < cn; ++q) {
        hcheck(hipMemcpyAsync(dG.p + q * gsz, G[c0 + q], sizeof(double) * gsz, hipMemcpyHostToDevice, st), "upload G");
        hcheck(hipMemcpyAsync(dbeta.p + (size_t)2 * n * q, betaW[c0 + q], sizeof(double) * n, hipMemcpyHostToDevice, st),
               "upload beta");
        hcheck(hipMemcpyAsync(dbeta.p + (size_t)2 * n * q + n, betaE[c0 + q], sizeof(double) * n,
                              hipMemcpyHostToDevice, st),
               "upload beta");
      }
      const int64_t rtot = (int64_t)rsz * cn;
      for (int e = 0; e < mz; ++e) {
        hipLaunchKernelGGL(k_inject, dim3((unsigned)((rtot + 255) / 256)), dim3(256), 0, st, dR.p, rtot, n, N, e);
        hcheck(hipGetLastError(), "inject");
        if (e > 0)
          rcheck(rocblas_dgemv_strided_batched(h, rocblas_operation_none, n * nr, n, &minus, dX.p + (size_t)(e - 1) * rsz,
                                               n * nr, (rocblas_stride)xsz, dlo.p + (size_t)e * n, 1, 0, &one, dR.p, 1,
                                               (rocblas_stride)rsz, cn),
                 "gemv lo");
        rcheck(rocblas_dgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_none, nr, n2, n2, &one, dR.p,
                                             nr, (rocblas_stride)rsz, dG.p + (size_t)e * n2 * n2, n2,
                                             (rocblas_stride)gsz, &zero, dX.p + (size_t)e * rsz, nr,
                                             (rocblas_stride)xsz, cn),
               "gemm forward");
      }
      for (int e = mz - 2; e >= 0; --e) {
        rcheck(rocblas_dgemv_strided_batched(h, rocblas_operation_none, n * nr, n, &one, dX.p + (size_t)(e + 1) * rsz,
                                             n * nr, (rocblas_stride)xsz, dup.p + (size_t)e * n, 1, 0, &zero, dQ.p, 1,
                                             (rocblas_stride)((size_t)n * nr), cn),
               "gemv up");
        rcheck(rocblas_dgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_none, nr, n2, n, &minus, dQ.p,
                                             nr, (rocblas_stride)((size_t)n * nr),
                                             dG.p + (size_t)e * n2 * n2 + (size_t)(n - 1) * n, n2, (rocblas_stride)gsz,
                                             &one, dX.p + (size_t)e * rsz, nr, (rocblas_stride)xsz, cn),
               "gemm backward");
      }
      for (int r = 0; r < 2; ++r) {
        for (int q = 0; q < cn; ++q)
          rcheck(rocblas_dgemv_strided_batched(h, rocblas_operation_none, nr, n, &one, dX.p + q * xsz, nr,
                                               (rocblas_stride)((size_t)n * nr), dbeta.p + (size_t)2 * n * q + r * n, 1,
                                               0, &zero, dY.p + (size_t)q * N * nr, 1, (rocblas_stride)nr, N),
                 "gemv beta");
        hcheck(hipMemcpyAsync(hY.data(), dY.p, sizeof(double) * N * nr * cn, hipMemcpyDeviceToHost, st), "download W");
        hcheck(hipStreamSynchronize(st), "W blocks");
        for (int q = 0; q < cn; ++q)
          for (int col = 0; col < 2; ++col) {
            double *dst = Wq[4 * (c0 + q) + 2 * r + col];
            for (int p = 0; p < N; ++p)
              std::memcpy(dst + (size_t)p * N, &hY[((size_t)q * N + p) * nr + (size_t)col * N], sizeof(double) * N);
          }
      }
    }
  }
};

DeviceDense *device_dense_create(bool always) {
  // The runtime starts on the calling thread, with its current device, before
  // any worker thread of the setup reaches the back end; without a device
  // the setup runs every step on the host.
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  DeviceDense *dd = new DeviceDense();
  dd->dev = dev;
  dd->be.always = always;
  dd->be.invert = [dd](int n, int count, double *const *mats) { dd->invert(n, count, mats); };
  dd->be.tri_factor = [dd](int d, int N, const double *Td, const double *Lo, const double *Up) {
    return dd->tri_factor(d, N, Td, Lo, Up);
  };
  dd->be.tri_solve = [dd](void *f, double *v) { dd->tri_solve(f, v); };
  dd->be.warm = [dd](int n, int mz, int inv_n, int tri_N) { dd->warm(n, mz, inv_n, tri_N); };
  dd->be.tri_free = [dd](void *f) {
    std::lock_guard<std::mutex> lk(dd->mu);
    (void)hipSetDevice(dd->dev);
    delete static_cast<TriFact *>(f);
  };
  dd->be.strip_schur = [dd](int ncl, int n, int mz, const double *const *G, const double *lo, const double *up,
                            const double *const *bw, const double *const *be, double *const *Wq) {
    dd->strip_schur(ncl, n, mz, G, lo, up, bw, be, Wq);
  };
  return dd;
}

void device_dense_destroy(DeviceDense *dd) { delete dd; }

const DenseBackend *device_dense_backend(const DeviceDense *dd) { return dd ? &dd->be : nullptr; }

}  // namespace smpm
