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
#include <cstring>
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

// Factors of the block-tridiagonal T, all column-major on the device:
// T~_i (M x M, LU with pivots), Lo_i (N x N), X_i = T~_i^-1 T[i][i+1]
// (the M x N nonzero columns).
struct TriFact {
  int d, N, M;
  DBuf<double> T, Lo, X, v, tmp;
  DBuf<rocblas_int> ipiv, info;
  TriFact(int d_, int N_)
      : d(d_), N(N_), M(2 * N_), T((size_t)d_ * 4 * N_ * N_), Lo((size_t)d_ * N_ * N_),
        X((size_t)d_ * 2 * N_ * N_), v((size_t)d_ * 2 * N_), tmp(2 * N_), ipiv((size_t)d_ * 2 * N_), info(d_) {}
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
    TriFact *f = new TriFact(d, N);
    try {
      std::vector<double> buf((size_t)M * M), bl((size_t)N * N), bx((size_t)M * N);
      for (int i = 0; i < d; ++i) {
        const double *t = Td + (size_t)i * M * M;
        for (int r = 0; r < M; ++r)
          for (int c = 0; c < M; ++c) buf[(size_t)c * M + r] = t[(size_t)r * M + c];
        hcheck(hipMemcpy(f->T.p + (size_t)i * M * M, buf.data(), sizeof(double) * M * M, hipMemcpyHostToDevice),
               "upload T");
        const double *l = Lo + (size_t)i * N * N;
        for (int r = 0; r < N; ++r)
          for (int c = 0; c < N; ++c) bl[(size_t)c * N + r] = l[(size_t)r * N + c];
        hcheck(hipMemcpy(f->Lo.p + (size_t)i * N * N, bl.data(), sizeof(double) * N * N, hipMemcpyHostToDevice),
               "upload Lo");
        std::fill(bx.begin(), bx.end(), 0.0);
        if (i + 1 < d) {
          const double *u = Up + (size_t)i * N * N;
          for (int r = 0; r < N; ++r)
            for (int c = 0; c < N; ++c) bx[(size_t)c * M + N + r] = u[(size_t)r * N + c];
        }
        hcheck(hipMemcpy(f->X.p + (size_t)i * M * N, bx.data(), sizeof(double) * M * N, hipMemcpyHostToDevice),
               "upload X");
      }
      const double one = 1.0, minus = -1.0;
      for (int i = 0; i < d; ++i) {
        double *T = f->T.p + (size_t)i * M * M;
        if (i > 0)
          rcheck(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, N, N, N, &minus,
                               f->Lo.p + (size_t)i * N * N, N, f->X.p + (size_t)(i - 1) * M * N, M, &one, T + (size_t)N * M,
                               M),
                 "gemm");
        rcheck(rocsolver_dgetrf(h, M, M, T, M, f->ipiv.p + (size_t)i * M, f->info.p + i), "getrf");
        if (i + 1 < d)
          rcheck(rocsolver_dgetrs(h, rocblas_operation_none, M, N, T, M, f->ipiv.p + (size_t)i * M,
                                  f->X.p + (size_t)i * M * N, M),
                 "getrs");
      }
      std::vector<rocblas_int> hinfo(d);
      hcheck(hipMemcpyAsync(hinfo.data(), f->info.p, sizeof(rocblas_int) * d, hipMemcpyDeviceToHost, st), "info");
      hcheck(hipStreamSynchronize(st), "elimination");
      for (int i = 0; i < d; ++i)
        if (hinfo[i] != 0) throw std::runtime_error("singular block in the inverse iteration for u_S");
    } catch (...) {
      delete f;
      throw;
    }
    return f;
  }

  // v <- T^-1 v: forward y_i = v_i - Lo_i T~_{i-1}^-1 y_{i-1} (first N rows),
  // backward x_i = T~_i^-1 y_i - X_i x_{i+1}[N..2N].
  void tri_solve(void *fp, double *v) {
    std::lock_guard<std::mutex> lk(mu);
    hcheck(hipSetDevice(dev), "hipSetDevice");
    TriFact *f = static_cast<TriFact *>(fp);
    const int d = f->d, N = f->N, M = f->M;
    const double one = 1.0, minus = -1.0;
    double *dv = f->v.p;
    hcheck(hipMemcpy(dv, v, sizeof(double) * d * M, hipMemcpyHostToDevice), "upload v");
    for (int i = 1; i < d; ++i) {
      hcheck(hipMemcpyAsync(f->tmp.p, dv + (size_t)(i - 1) * M, sizeof(double) * M, hipMemcpyDeviceToDevice, st),
             "copy");
      rcheck(rocsolver_dgetrs(h, rocblas_operation_none, M, 1, f->T.p + (size_t)(i - 1) * M * M, M,
                              f->ipiv.p + (size_t)(i - 1) * M, f->tmp.p, M),
             "getrs");
      rcheck(rocblas_dgemv(h, rocblas_operation_none, N, N, &minus, f->Lo.p + (size_t)i * N * N, N, f->tmp.p, 1, &one,
                           dv + (size_t)i * M, 1),
             "gemv");
    }
    for (int i = d - 1; i >= 0; --i) {
      rcheck(rocsolver_dgetrs(h, rocblas_operation_none, M, 1, f->T.p + (size_t)i * M * M, M, f->ipiv.p + (size_t)i * M,
                              dv + (size_t)i * M, M),
             "getrs");
      if (i + 1 < d)
        rcheck(rocblas_dgemv(h, rocblas_operation_none, M, N, &minus, f->X.p + (size_t)i * M * N, M,
                             dv + (size_t)(i + 1) * M + N, 1, &one, dv + (size_t)i * M, 1),
               "gemv");
    }
    hcheck(hipMemcpyAsync(v, dv, sizeof(double) * d * M, hipMemcpyDeviceToHost, st), "download v");
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
