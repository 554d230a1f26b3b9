// Device-side descriptors of the SMPM Schur solver (shared by the kernels
// and the host orchestration in smpm.hip).
#pragma once
#include <cstdint>

namespace smpm {

constexpr int kBlock = 256;
constexpr int kMaxNodes = 22;   // GLL points per direction (polynomial order <= 21)         // threads per workgroup (4 wave64)
constexpr int kChunk = 512;         // interface/node elements per workgroup in vector kernels
constexpr int kMaxN = 544;          // largest n * m_z supported (half-interface length)
constexpr int kMaxRowsPerLane = (kMaxN + 63) / 64;

// Per-system tables on the device.  Block layouts are column-major inside a
// block ([col][row]) so that a wavefront reads consecutive rows of one column.
struct SysDev {
  int n, mx, mz, n2, N, nh, d, singular;
  int Np;                // rows of the stored Schur / block-Jacobi blocks (N rounded up to 8)
  int zm;                // coarse columns per interface: 1, or m_z (one per element segment)
  const int *sz_col;     // per half: [2 zm] coarse columns of its S Z rows (-1: none)
  const double *SZh;     // per half: [2 zm][N]
  int64_t kS, r;
  double tau;
  const double *W64;     // unique Schur half blocks: [blk][2N][N]
  const float *W32;
  const int *w_id, *w_win;
  const double *M64;     // unique block-Jacobi row chunks: [chunk][4N][N]
  const float *M32;
  // FP16 copies (SMPM_FP16S_IR handles only): each row segment of n rows
  // (one element) of a block stored divided by its largest magnitude;
  // scales [blk][m_z].
  const _Float16 *W16, *M16;
  const float *W16s, *M16s;
  // S M^-1 per half (grids whose strips share blocks): [blk][8N][Np] in each
  // precision, FP16 scales [blk][m_z]
  const double *F64;
  const float *F32;
  const _Float16 *F16;
  const float *F16s;
  const int *m_id, *m_win, *m_K;
  const double *Gc;      // coarse operator, column-major d x d
  const double *GcR;     // the same row-major (one coarse column per interface only)
  const double *uS, *uL; // null vectors (k = 0), else nullptr
  const double *Dinv;    // element inverses: [class][e][col n2][row n2]
  const double *Kinv;    // z-interface capacitance inverses: [class][col nq][row nq]
  int nq;                // 2 n (m_z - 1)
  const double *lo, *up; // [e][n]
  const double *beta;    // [class][2][n]: west row, east row
  const int *strip_class;
};

// Per-instance (system, rhs) offsets into the batched work arrays.
struct InstDev {
  int sys, rhs;
  int nchunk_x;          // chunks of the interface vector
  int nchunk_r;          // chunks of the node vector
  int64_t f_off;         // node-space offset (f, u, F, v)
  int64_t g_off;         // Neumann-data offset
  int64_t x_off;         // interface-space offset
  int64_t v_off;         // Krylov basis offset
  int64_t part_off;      // partial-sum offset: [maxit + 1][nchunk_x]
  int64_t pr_off;        // node-space partials: [nchunk_r] x 2
  int64_t hs_off;        // half sums: [nh]
  int64_t c_off;         // coarse vectors: [d]
  int64_t st_off;        // GMRES scalars: [maxit + 1]
  int64_t rr_off;        // R factor: [maxit][maxit]
  int64_t lam_off;       // z-interface functionals: [m_x][nq]
  // Krylov segment: instances seg_first .. seg_first + seg_count - 1 share one
  // GMRES (one Krylov space over all of them, Sec. 5.2); every member then
  // has the leader's st_off and rr_off.  A plain instance is its own segment.
  int seg_first, seg_count;
};

// Work item of the half-interface GEMV: up to kGroup halves of one instance
// that share the same operator block.
constexpr int kGroup = 4;
struct HWork {
  int inst, cnt;
  int h[kGroup];
};

// Work item of the shared-block GEMM: one stored block (N x K, column-major
// with leading dimension Np, in both precisions) applied to `vcount`
// (instance, half) windows listed from `vstart` in the window table.
constexpr int kGemmVecs = 32;   // windows per workgroup
struct GWork {
  const double *blk64;
  const float *blk32;
  const _Float16 *blk16;   // FP16 copy (or nullptr) and its row-segment scales [m_z]
  const float *sc16;
  int N, Np, K, vstart, vcount, ident;   // ident: add the identity (S = I + W)
  int n, pad;                            // n: rows per scale segment (one element)
  int64_t kS;
};
// One window of a GEMM item, with every offset resolved at setup.
struct GVec {
  int64_t x0;     // input vector of the instance (offset of its interface vector)
  int64_t xv;     // Krylov basis of the instance (slot 0)
  int64_t win;    // window start inside the instance's interface vector (may be < 0)
  int64_t xh;     // own half inside the instance's interface vector (identity term)
  int64_t y;      // output offset
  int inst;       // instance (GMRES state, scale)
  int hs;         // Z^T partial sums: slot 0 of this half (slot q at hs + q hn)
  int st_off;     // scale vector of the instance
  int hn;         // stride between the 16-row slots of the partial sums (halves)
  int pad[2];
};

// Column-gather GEMM item (element-interior elimination): Y[:, c] (+)= A X[:, c]
// for the `ccount` columns listed from `cstart`.  A is R x K column-major with
// leading dimension lda; columns k >= ksplit of the product read A's column
// k + agap and the second source segment of the column (x2 + k - ksplit).
constexpr int kColVecs = 64;    // columns per workgroup
struct CGItem {
  const double *A;
  int R, K, lda, ksplit, agap, cstart, ccount, pad;
};
// Offsets (elements) of one column: first and second source segment (-1:
// zeros) and the output.
struct CGCol {
  int64_t x1, x2, y;
};

struct GState {
  int iter;    // columns of the Hessenberg matrix built so far
  int active;  // 1 while iterating
  int status;  // 0 ok, 1 converged, 2 max_iter, 3 non-finite, 4 breakdown
  int pad;
  double r0;   // initial residual norm
  double res;  // |g_{iter}| (recursive residual)
  double ref;  // reference norm of the stopping test |g| <= tol * ref
};

}  // namespace smpm
