// Host-side data of the SMPM Schur solver: per-system operator tables built
// in FP64 at setup time and uploaded once.  No device code here.
#pragma once
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace smpm {

// ---- dense FP64 helpers (row-major) ---------------------------------------
// C[M x N] = beta * C + alpha * A[M x K] * B[K x N]; leading dimensions in
// elements.  Serial; callers parallelize over independent tasks.
void gemm(int M, int N, int K, double alpha, const double *A, int lda,
          const double *B, int ldb, double beta, double *C, int ldc);
// LU with partial pivoting, in place; returns false on an exactly zero pivot.
bool getrf(int n, double *A, int lda, int *piv);
// Solve A X = B with the factors of getrf; B is n x nrhs, leading dim ldb.
void getrs(int n, int nrhs, const double *LU, int lda, const int *piv, double *B, int ldb);
// Same with A^T.
void getrs_t(int n, int nrhs, const double *LU, int lda, const int *piv, double *B, int ldb);
// In-place inverse of an n x n matrix; false if singular.
bool invert(int n, double *A, int lda);

// Run fn(i) for i in [0, count) on up to `threads` worker threads.
void parallel_for(int count, int threads, const std::function<void(int)> &fn);
int default_threads();

// ---- GLL ------------------------------------------------------------------
struct GLL {
  int n;
  std::vector<double> x, w, D;   // nodes, weights, D row-major n x n
};
GLL make_gll(int n);

// ---- one strip class: strips with identical width and boundary type --------
struct StripClass {
  double hx;
  bool west_if, east_if;            // west / east side is an inter-strip interface
  // block-Thomas factors over the m_z elements: G[e] = (D~_e)^-1, n2 x n2,
  // row-major on the host.
  std::vector<double> G;
  // Element-parallel form for the device (Woodbury in z): A_j = D + P Lambda
  // with D = blockdiag(Dg_e) and P Lambda the z-interface coupling.
  // Dinv[e] = Dg_e^-1 (n2 x n2 row-major); Kinv = (I + Lambda D^-1 P)^-1,
  // nq = 2 n (m_z - 1) square, row-major.  q ordering: interface i (between
  // elements i and i+1): [lo: rows (0, t) of i+1 | up: rows (n-1, t) of i].
  std::vector<double> Dinv, Kinv;
  // B-row functionals of this strip's west / east element rows (n values).
  std::vector<double> betaW, betaE;
  // W quarter blocks Wq[r][c] (N x N row-major), r: 0 west row, 1 east row;
  // c: 0 west column, 1 east column.
  std::vector<double> Wq[2][2];
};

// ---- one system: a grid and one wavenumber ---------------------------------
struct System {
  int n = 0, mx = 0, mz = 0, n2 = 0, N = 0, nh = 0, d = 0;
  int zm = 1;   // coarse columns per interface: 1, or m_z (one per element segment)
  int64_t r = 0, kS = 0;
  double kwave = 0.0, tau = 0.0;
  bool singular = false;
  std::vector<double> xb, zb;
  std::vector<double> lo, up;            // [e][c]: z-coupling coefficients
  std::vector<int> strip_class;          // per strip
  std::vector<StripClass> classes;

  // Schur matvec: for output half h, y_h = x_h + W^_h x[win(h) .. win(h)+2N)
  // with W^_h an N x 2N block.  Blocks are deduplicated.
  std::vector<int> w_id, w_win;          // per half
  std::vector<double> Wblk;              // unique blocks, N x 2N row-major
  int nW = 0;
  // Block-Jacobi row chunks: y_h = Mc_h x[m_win(h) .. + m_K(h)).
  std::vector<int> m_id, m_win, m_K;     // per half
  std::vector<double> Mblk;              // unique chunks, N x 4N row-major (zero padded)
  int nM = 0, nMblocks = 0;
  // Fused operator S M^-1 for grids whose strips share blocks (built when
  // some Schur block serves two halves): y_h = Fblk[f_id] x[f_win N .. + f_K),
  // an N x f_K block (f_K <= 8N, zero padded to 8N) over the one or two
  // block-Jacobi blocks that half h and its window touch.
  std::vector<int> f_id, f_win, f_K;
  std::vector<double> Fblk;              // unique blocks, N x 8N row-major
  int nF = 0;
  // Deflation: S Z restricted per half to the coarse columns of the two
  // interfaces its window touches (2 zm columns).
  std::vector<int> sz_col;               // per half: [2 zm] coarse columns (-1 if none)
  std::vector<double> SZh;               // per half: [2 zm][N]
  std::vector<double> C;                 // d x d row-major
  std::vector<double> Gc;                // coarse operator C^dagger (I - u_C u_C^T), d x d row-major
  // Null vectors (k = 0 only).
  std::vector<double> uS, uL, uC;
  // Setup steps that ran on the device back end: 1 the u_S elimination,
  // 2 the block-Jacobi inverses, 4 the coarse inverse.
  int dev_steps = 0;
  // Offsets into batched arrays.
  int64_t f_off = 0, g_off = 0, x_off = 0;
};

// Optional device back end of the heavy dense setup steps; an empty member
// means the host code runs that step.
struct DenseBackend {
  // Take the device path for every step below whatever its size (else from
  // 2e10 flops of work per host thread on, where it pays for the transfers
  // and the library start-up).
  bool always = false;
  // In-place inverses of `count` n x n row-major matrices; throws
  // std::domain_error if one is singular.
  std::function<void(int n, int count, double *const *mats)> invert;
  // Block-tridiagonal T over d interfaces (blocks M = 2N square, row-major):
  // diagonal blocks Td[i] (M x M), sub-diagonal Lo[i] (i >= 1: the N x N block
  // at rows 0..N of i, columns 0..N of i - 1), super-diagonal Up[i]
  // (i + 1 < d: the N x N block at rows N..2N of i, columns N..2N of i + 1).
  // tri_factor eliminates it and returns an opaque factorization (throws
  // std::runtime_error on a singular block); tri_solve overwrites v (d M)
  // with T^-1 v; tri_free releases the factorization.
  std::function<void *(int d, int N, const double *Td, const double *Lo, const double *Up)> tri_factor;
  std::function<void(void *fact, double *v)> tri_solve;
  std::function<void(void *fact)> tri_free;
  // Schur quarter blocks of ncl strip classes (the multi-right-hand-side strip
  // solve with the 2N boundary injections): from each class's block-Thomas
  // factors G[c] (m_z blocks n2 x n2, row-major, as StripClass::G), the shared
  // z couplings lo, up (m_z x n) and the class's B-row functionals betaW[c],
  // betaE[c] (n each), writes Wq[4 c + 2 r + col] (N x N row-major, as
  // StripClass::Wq[r][col]).
  std::function<void(int ncl, int n, int mz, const double *const *G, const double *lo, const double *up,
                     const double *const *betaW, const double *const *betaE, double *const *Wq)>
      strip_schur;
  // Starts the back end's stream and library handles and loads the library
  // kernels the steps above use (the strip solves of strips of m_z elements
  // of order n - 1, if n > 0; inverses of inv_n x inv_n matrices, if
  // inv_n > 0; the block-tridiagonal elimination with N-row halves, if
  // tri_N > 0), so that the first step does not pay for them; meant for a
  // worker thread while the host steps run.  Never throws.
  std::function<void(int n, int mz, int inv_n, int tri_N)> warm;
};

struct SetupOptions {
  double tau = 0.0;
  int threads = 0;
  int zlabel = 0;   // deflation space: 0 one column per interface, 1 per element segment
  const DenseBackend *dense = nullptr;
  // A second back end for the u_S elimination, which runs beside the other
  // setup steps (its own stream and library handle); nullptr: `dense`.
  const DenseBackend *dense_null = nullptr;
};

// Build every host table of one system.  Throws std::runtime_error with a
// message on invalid input or singular factorizations.
void build_system(System &s, int mx, int mz, int order, const double *xb, const double *zb,
                  double kwave, const SetupOptions &opt);

// Host references used by export and by the setup itself.
void strip_solve(const System &s, const StripClass &c, double *X, int nrhs);    // A_j^-1 X (in place)
void strip_solve_woodbury(const System &s, const StripClass &c, double *x);     // A_j^-1 x (one rhs)
void strip_solve_t(const System &s, const StripClass &c, double *X, int nrhs);  // A_j^-T X (in place)
void schur_apply_host(const System &s, const double *x, double *y);             // y = S x
// B A_j^-1 of a strip class: [side][row][node], 2 x N x (m_z n^2) row-major.
void class_rhs_blocks(const System &s, const StripClass &cl, std::vector<double> &out);

}  // namespace smpm
