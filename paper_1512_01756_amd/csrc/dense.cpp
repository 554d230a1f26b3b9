// Small dense FP64 linear algebra for the host-side setup (row-major).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "host.hpp"

namespace smpm {

// Register-blocked kernel: 4 rows of C at a time, 64 columns per tile, so one
// load of B[k][j..j+63] feeds four FMAs.
void gemm(int M, int N, int K, double alpha, const double *A, int lda,
          const double *B, int ldb, double beta, double *C, int ldc) {
  if (beta != 1.0) {
    for (int i = 0; i < M; ++i) {
      double *c = C + (size_t)i * ldc;
      if (beta == 0.0) std::fill(c, c + N, 0.0);
      else for (int j = 0; j < N; ++j) c[j] *= beta;
    }
  }
  if (alpha == 0.0 || K == 0) return;
  const int JB = 64, KB = 256;
  for (int k0 = 0; k0 < K; k0 += KB) {
    const int k1 = std::min(K, k0 + KB);
    for (int j0 = 0; j0 < N; j0 += JB) {
      const int jn = std::min(N, j0 + JB) - j0;
      int i = 0;
      for (; i + 4 <= M; i += 4) {
        double acc[4][JB];
        for (int q = 0; q < 4; ++q)
          for (int j = 0; j < jn; ++j) acc[q][j] = 0.0;
        const double *a0 = A + (size_t)(i + 0) * lda;
        const double *a1 = A + (size_t)(i + 1) * lda;
        const double *a2 = A + (size_t)(i + 2) * lda;
        const double *a3 = A + (size_t)(i + 3) * lda;
        for (int k = k0; k < k1; ++k) {
          const double *__restrict b = B + (size_t)k * ldb + j0;
          const double x0 = a0[k], x1 = a1[k], x2 = a2[k], x3 = a3[k];
          for (int j = 0; j < jn; ++j) {
            const double bj = b[j];
            acc[0][j] += x0 * bj;
            acc[1][j] += x1 * bj;
            acc[2][j] += x2 * bj;
            acc[3][j] += x3 * bj;
          }
        }
        for (int q = 0; q < 4; ++q) {
          double *c = C + (size_t)(i + q) * ldc + j0;
          for (int j = 0; j < jn; ++j) c[j] += alpha * acc[q][j];
        }
      }
      for (; i < M; ++i) {
        double acc[JB];
        for (int j = 0; j < jn; ++j) acc[j] = 0.0;
        const double *a = A + (size_t)i * lda;
        for (int k = k0; k < k1; ++k) {
          const double *__restrict b = B + (size_t)k * ldb + j0;
          const double x = a[k];
          for (int j = 0; j < jn; ++j) acc[j] += x * b[j];
        }
        double *c = C + (size_t)i * ldc + j0;
        for (int j = 0; j < jn; ++j) c[j] += alpha * acc[j];
      }
    }
  }
}

bool getrf(int n, double *A, int lda, int *piv) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(A[(size_t)k * lda + k]);
    for (int i = k + 1; i < n; ++i) {
      const double v = std::fabs(A[(size_t)i * lda + k]);
      if (v > best) { best = v; p = i; }
    }
    piv[k] = p;
    if (best == 0.0) return false;
    if (p != k) {
      double *rk = A + (size_t)k * lda, *rp = A + (size_t)p * lda;
      for (int j = 0; j < n; ++j) std::swap(rk[j], rp[j]);
    }
    const double inv = 1.0 / A[(size_t)k * lda + k];
    const double *__restrict rk = A + (size_t)k * lda;
    for (int i = k + 1; i < n; ++i) {
      double *__restrict ri = A + (size_t)i * lda;
      const double l = ri[k] * inv;
      ri[k] = l;
      if (l != 0.0)
        for (int j = k + 1; j < n; ++j) ri[j] -= l * rk[j];
    }
  }
  return true;
}

void getrs(int n, int nrhs, const double *LU, int lda, const int *piv, double *B, int ldb) {
  for (int k = 0; k < n; ++k)
    if (piv[k] != k) {
      double *a = B + (size_t)k * ldb, *b = B + (size_t)piv[k] * ldb;
      for (int j = 0; j < nrhs; ++j) std::swap(a[j], b[j]);
    }
  for (int i = 1; i < n; ++i) {           // L y = P b (unit lower)
    double *__restrict bi = B + (size_t)i * ldb;
    const double *li = LU + (size_t)i * lda;
    for (int k = 0; k < i; ++k) {
      const double l = li[k];
      if (l == 0.0) continue;
      const double *__restrict bk = B + (size_t)k * ldb;
      for (int j = 0; j < nrhs; ++j) bi[j] -= l * bk[j];
    }
  }
  for (int i = n - 1; i >= 0; --i) {      // U x = y
    double *__restrict bi = B + (size_t)i * ldb;
    const double *ui = LU + (size_t)i * lda;
    for (int k = i + 1; k < n; ++k) {
      const double u = ui[k];
      if (u == 0.0) continue;
      const double *__restrict bk = B + (size_t)k * ldb;
      for (int j = 0; j < nrhs; ++j) bi[j] -= u * bk[j];
    }
    const double inv = 1.0 / ui[i];
    for (int j = 0; j < nrhs; ++j) bi[j] *= inv;
  }
}

void getrs_t(int n, int nrhs, const double *LU, int lda, const int *piv, double *B, int ldb) {
  // A = P^T L U  =>  A^T = U^T L^T P: solve U^T y = b, L^T z = y, x = P^T z.
  for (int i = 0; i < n; ++i) {
    double *__restrict bi = B + (size_t)i * ldb;
    for (int k = 0; k < i; ++k) {
      const double u = LU[(size_t)k * lda + i];
      if (u == 0.0) continue;
      const double *__restrict bk = B + (size_t)k * ldb;
      for (int j = 0; j < nrhs; ++j) bi[j] -= u * bk[j];
    }
    const double inv = 1.0 / LU[(size_t)i * lda + i];
    for (int j = 0; j < nrhs; ++j) bi[j] *= inv;
  }
  for (int i = n - 2; i >= 0; --i) {
    double *__restrict bi = B + (size_t)i * ldb;
    for (int k = i + 1; k < n; ++k) {
      const double l = LU[(size_t)k * lda + i];
      if (l == 0.0) continue;
      const double *__restrict bk = B + (size_t)k * ldb;
      for (int j = 0; j < nrhs; ++j) bi[j] -= l * bk[j];
    }
  }
  for (int k = n - 1; k >= 0; --k)
    if (piv[k] != k) {
      double *a = B + (size_t)k * ldb, *b = B + (size_t)piv[k] * ldb;
      for (int j = 0; j < nrhs; ++j) std::swap(a[j], b[j]);
    }
}

bool invert(int n, double *A, int lda) {
  std::vector<double> LU((size_t)n * n);
  std::vector<int> piv(n);
  for (int i = 0; i < n; ++i) std::memcpy(&LU[(size_t)i * n], A + (size_t)i * lda, sizeof(double) * n);
  if (!getrf(n, LU.data(), n, piv.data())) return false;
  for (int i = 0; i < n; ++i) {
    double *ai = A + (size_t)i * lda;
    std::fill(ai, ai + n, 0.0);
    ai[i] = 1.0;
  }
  getrs(n, n, LU.data(), n, piv.data(), A, lda);
  return true;
}

int default_threads() {
  unsigned hc = std::thread::hardware_concurrency();
  if (hc == 0) hc = 4;
  return (int)std::min(hc, 16u);
}

void parallel_for(int count, int threads, const std::function<void(int)> &fn) {
  if (count <= 0) return;
  if (threads <= 0) threads = default_threads();
  threads = std::min(threads, count);
  if (threads <= 1) {
    for (int i = 0; i < count; ++i) fn(i);
    return;
  }
  std::atomic<int> next(0);
  std::vector<std::thread> pool;
  std::vector<std::exception_ptr> errs(threads);
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&, t]() {
      try {
        for (int i = next++; i < count; i = next++) fn(i);
      } catch (...) {
        errs[t] = std::current_exception();
      }
    });
  for (auto &th : pool) th.join();
  for (auto &e : errs)
    if (e) std::rethrow_exception(e);
}

}  // namespace smpm
