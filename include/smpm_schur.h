/*
 * smpm_schur.h -- C ABI of the MI355X (gfx950) Schur-complement solver for the
 * spectral multidomain penalty (SMPM) discretization of the 2-D Poisson- and
 * Helmholtz-Neumann problem, preconditioned by block-Jacobi and deflation.
 *
 * Method: Joshi, Thomsen & Diamessis, "Deflation-accelerated preconditioning
 * of the Poisson-Neumann Schur problem on long domains with a high-order
 * discontinuous element-based collocation method", arXiv:1512.01756.
 *   - discretization: Sec. 2.2, Eq. (smpm_poisson);
 *   - strip split L = A + E B and S = I + B A^-1 E: Sec. 2.3, Eq. (operator_decomp);
 *   - null-space projections: Sec. 2.4, Eqs. (regularize_poisson), (regularize_schur);
 *   - GMRES, block-Jacobi M, deflation P, Q: Sec. 3, Eq. (deflated_schur),
 *     Algorithm 2;
 *   - Fourier modes in y, one Helmholtz Schur problem per wavenumber: Sec. 5,
 *     Eq. (transverse_schur).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * n = order + 1 GLL points per direction; r = n^2 m_x m_z nodes;
 * k_S = 2 n m_z (m_x - 1) interface unknowns; d = m_x - 1 coarse unknowns.
 *
 * Node layout of f and u (FP64):
 *     node(j, e, b, a) = ((j * m_z + e) * n + b) * n + a
 *   j strip (x), e element in the strip (z, bottom first), b GLL index in z,
 *   a GLL index in x (fastest).
 * Neumann data g of one right-hand side (FP64), four sides back to back:
 *     south[m_x][n] (strip, a), north[m_x][n], west[m_z][n] (element, b),
 *     east[m_z][n]                      -> 2 n (m_x + m_z) values.
 * Interface (Schur) vectors: half-interface h = 2i is the east edge of strip
 *   i, h = 2i + 1 the west edge of strip i + 1 (i = 0 .. m_x - 2); inside a
 *   half the order is (e, b); index h * n m_z + e * n + b.
 *
 * A handle holds one or more "systems": a (grid, wavenumber k) pair with its
 * own operators S(k), M(k), C(k).  Each system solves `nrhs` right-hand sides
 * (e.g. the real and imaginary parts of a Fourier mode).  An "instance" is a
 * (system, rhs) pair.  Batched device arrays are the concatenation over
 * systems in setup order, and inside a system over rhs.
 *
 * Memory: pointers named *_dev are device pointers (hipMalloc'ed, or torch
 * CUDA tensors); every other pointer is host memory.  The caller owns all
 * buffers it passes; the handle owns every operator table and workspace,
 * allocated in setup, which also captures and instantiates every HIP graph
 * a solve launches (they hold only the handle's own buffers).  smpm_solve,
 * smpm_solve_fourier and smpm_apply allocate nothing, whatever buffers the
 * caller passes; smpm_apply_noalloc below also uses no handle workspace.
 *
 * Streams: every device call enqueues on the caller's hipStream_t (NULL = the
 * default stream).  Calls that fill host-side results synchronize that
 * stream before returning.
 *
 * Errors: every call returns smpm_status; nothing throws across the ABI.
 * smpm_last_error() returns a thread-local message for the last non-OK
 * status.  A handle is not thread-safe; distinct handles are independent.
 */
#ifndef SMPM_SCHUR_H
#define SMPM_SCHUR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SMPM_OK = 0,
  SMPM_EINVAL = -1,      /* bad argument or shape */
  SMPM_ENOMEM = -2,      /* host or device allocation failed */
  SMPM_EHIP = -3,        /* HIP runtime error */
  SMPM_ESINGULAR = -4,   /* k = 0 with m_x < 4, or a factorization failed */
  SMPM_ENOTCONV = -5,    /* max_iter / sweeps reached, or a refinement sweep failed
                            to cut the residual by 10%, or the rate of the last
                            sweep would need more sweeps than are left; u holds
                            the last iterate */
  SMPM_ENONFINITE = -6,  /* NaN or Inf in the inputs or the iterates */
  SMPM_EUNSUPPORTED = -7 /* the call needs a GPU but the handle is host-only */
} smpm_status;

typedef enum {
  SMPM_FP64 = 0,     /* every step in FP64 */
  SMPM_FP32_IR = 1,  /* FP32 inner DBJ-GMRES (operators, Krylov basis) inside
                        FP64 iterative refinement: outer residual, projections,
                        coarse solve and least squares stay FP64 */
  SMPM_FP16S_IR = 2  /* as FP32_IR, with the Schur and block-Jacobi operators of
                        the inner solve stored in FP16, each element's row
                        segment of a block scaled by its largest magnitude
                        (FP32 scales, FP32 arithmetic) */
} smpm_precision;

typedef enum {
  SMPM_METHOD_DBJ = 0,   /* GMRES(P S M^-1, P b~): Algorithm 2 (default)  */
  SMPM_METHOD_BJ = 1,    /* GMRES(S M^-1, b~), Table 1 "BJ-Schur"          */
  SMPM_METHOD_SCHUR = 2, /* GMRES(S, b~), Table 1 "Schur"                  */
  SMPM_METHOD_2LAS = 3   /* GMRES(S (M^-1 + Z C\(I - u_C u_C^T) Z^T), b~)  */
} smpm_method;

#define SMPM_FLAG_HOST_ONLY 1  /* build the host tables only; no GPU is touched */
#define SMPM_FLAG_NO_TUNE 2    /* skip the setup-time GEMM schedule tuning; pick
                                  schedules by launch size (reproducible across
                                  handles) */
#define SMPM_FLAG_ONE_KRYLOV 4 /* one DBJ-GMRES over every instance of the handle:
                                  the block-diagonal operator of Sec. 5.2 / Alg. 3,
                                  stopping on the norm of the stacked residual;
                                  DBJ only (else EINVAL) */
#define SMPM_FLAG_HOST_SETUP 8 /* run every setup step on the host threads, also
                                  on a GPU handle (by default the large dense
                                  steps of Sec. 2.4 / 3.2 -- the u_S elimination,
                                  block-Jacobi and coarse inverses -- run on the
                                  device through rocSOLVER / rocBLAS) */
#define SMPM_FLAG_DEVICE_SETUP 16 /* take the device path for those steps whatever
                                  their size (default: from 2e10 flops of work per
                                  host thread on: the sequential u_S elimination
                                  of large grids, a large coarse inverse);
                                  ignored with HOST_ONLY or HOST_SETUP */

typedef struct {
  int32_t mx, mz;      /* elements in x (>= 2) and z (>= 1) */
  int32_t order;       /* polynomial degree (>= 1); n = order + 1 */
  const double *xb;    /* host, mx + 1 strictly increasing x breakpoints */
  const double *zb;    /* host, mz + 1 strictly increasing z breakpoints */
} smpm_grid;

typedef struct {
  double tau;          /* penalty; 0 selects -n(n-1)/h_min (one global value) */
  double tol;          /* relative Schur residual target; 0 selects 1e-10 */
  int32_t max_iter;    /* GMRES iterations (no restart); 0 selects 300 */
  int32_t nrhs;        /* right-hand sides per system; 0 selects 1 */
  int32_t precision;   /* smpm_precision */
  int32_t method;      /* smpm_method */
  double inner_tol;    /* FP32_IR: each sweep's inner GMRES stops at
                          max(inner_tol * ||r||, 0.5 * tol * ||b~||), r the sweep's
                          FP64 residual; 0 selects 1e-4 (one sweep gains about
                          1e-4 to 1e-5 with FP32 operators) */
  int32_t max_sweeps;  /* refinement sweeps; 0 selects 12 (FP32_IR) or 40 (FP16S_IR) */
  int32_t flags;       /* SMPM_FLAG_* */
  int32_t zlabel;      /* deflation space Z (Sec. 3.3): 0 one column per interface
                          (the paper's, d = m_x - 1), 1 one column per element
                          segment of an interface (d = (m_x - 1) m_z <= 4096) */
} smpm_opts;

typedef struct {
  int32_t instances;       /* systems * nrhs */
  int32_t converged;       /* instances that reached tol */
  int32_t iters_total;     /* GMRES iterations summed over instances (all sweeps) */
  int32_t iters_max;       /* largest per-instance GMRES iteration count */
  int32_t sweeps_max;      /* refinement sweeps (1 for FP64) */
  int32_t schur_matvecs;   /* S applications in the solve, summed over instances */
  double rel_residual_max; /* max over instances of ||P_u (S x_S - b~)|| / ||b~|| (FP64),
                              P_u = I - u_S u_S^T at k = 0 (the identity at k > 0): the
                              residual of the regularized system within range(S) */
  double compat_defect_max;/* max over k = 0 instances of |u_L^T F| / ||F|| */
  double solve_ms;         /* wall time of the solve (host clock, synchronized) */
  double null_residual_max;/* max over k = 0 instances of |u_S^T (S x_S - b~)| / ||b~||:
                              the residual's component along u_S, which no x_S reduces
                              (the rounding of u_S and of S x_S); 0 at k > 0 */
} smpm_stats;

typedef struct {
  int32_t n, mx, mz;
  int32_t nrhs;
  int64_t r;               /* nodes */
  int64_t kS;              /* interface unknowns */
  int32_t d;               /* coarse unknowns */
  double kwave;            /* wavenumber k of this system */
  double tau;              /* penalty in use */
  int64_t f_offset;        /* element offset of this system in batched f/u */
  int64_t g_offset;        /* element offset in batched g */
  int64_t x_offset;        /* element offset in batched interface vectors */
  int32_t unique_W;        /* distinct Schur strip blocks stored */
  int32_t unique_M;        /* distinct block-Jacobi blocks stored */
  int64_t bytes_W64;       /* algorithmic bytes of one FP64 Schur matvec's operator */
  int64_t bytes_M64;       /* same for one block-Jacobi apply */
  int32_t gemm_sched[4];   /* handle-wide GEMM schedules of the batched shared-block
                              matvecs: S FP64, S FP32, M^-1 FP64, M^-1 FP32
                              (0 split-K 16 waves, 1 split-K 8 waves, 2 LDS-staged
                              XCD-ordered, 3 LDS-staged plain, 4 / 5 the same two
                              staging 64 K-values per chunk, 6 / 7 split-K 8 / 16
                              waves with a wave's K range in flight at once, for
                              lists of at most 16 windows per item, 8 LDS-staged
                              128-row tiles, 9 / 10 64- / 128-row tiles whose 16
                              waves also split K, 11 LDS-staged 128-row tiles in
                              a cost-ordered XCD-aware order, 12 the same with
                              64 K-values per chunk; -1 no shared blocks).
                              SMPM_GEMM_SCHED = 0..12 in the environment,
                              read at setup and load, pins them all (tests,
                              experiments) */
  int32_t elem_sched[6];   /* same for the element-interior GEMM lists
                              (D^-1, K^-1, correction) x (<= 16, <= 64 columns),
                              with two more: 4 LDS-staged 32-row tiles, 5 16-row
                              tiles, their waves splitting K.  The environment
                              variable SMPM_ELEM_SCHED = 1..5, read at setup and
                              load, pins all six (tests, experiments) */
  int32_t fused_op[3];     /* 1 if the GMRES iteration applies S M^-1 as one stored
                              block per half (FP64, FP32, FP16 storage): chosen at
                              setup when faster than M^-1 then S; grids whose strips
                              share blocks only */
  int32_t setup_device;    /* setup steps of this system that ran on the device
                              (rocSOLVER / rocBLAS): 1 the u_S elimination, 2 the
                              block-Jacobi inverses, 4 the coarse inverse, 8 the
                              strip solves behind the Schur blocks W, 16 the
                              element and z-capacitance inverses of the
                              interior elimination */
  /* Algorithmic operator sizes (nonzero entries; "unique" counts each
     distinct stored block once, "total" sums over the halves of one
     instance): the Schur blocks W (Sec. 3.1), the block-Jacobi inverses
     (Sec. 3.2), the stored S M^-1 blocks (0 when the grid has none), the
     strip classes and the distinct element inverses of the interior
     elimination (Sec. 2.3). */
  int64_t nnz_W_unique, nnz_W_total;
  int64_t nnz_M_unique, nnz_M_total;
  int64_t nnz_F_unique, nnz_F_total;
  int32_t strip_classes, elem_unique;
  int32_t fused_sched[3];  /* schedule of the S M^-1 GEMM list (FP64, FP32, FP16
                              storage; -1 none), numbered as gemm_sched */
  int32_t rhs_gemm[2];     /* the Schur right-hand side b_S = (B A^-1) F~ as one
                              GEMM over the strips (grids whose strips share
                              classes): its schedule, numbered as gemm_sched, and
                              the windows per item of the list it runs on (32, or
                              16 for the narrow schedules); -1 -1 when b_S comes
                              from element solves.  SMPM_RHS_GEMM = "s,l" in the
                              environment (s = 0..12; l = 0 for the 32-window
                              list, 1 for the 16-window one, which exists only
                              when some item has more than 16 windows), read at
                              setup and load, pins both (tests, experiments) */
  int32_t gemm_list[4];    /* windows per item (32, or 16 for the narrow
                              schedules) of the list each gemm_sched entry runs
                              on: every S and M^-1 list with an item of more
                              than 16 windows is also built in items of at most
                              16, and the tuner times every schedule on both (-1
                              no shared blocks).  SMPM_GEMM_LIST = 1 in the
                              environment, read at setup and load, pins the
                              16-window lists where they exist (tests,
                              experiments); SMPM_GEMM_SCHED pins the 32-window
                              ones unless SMPM_GEMM_LIST = 1 is set too */
  int32_t elem_alt[3];     /* per element-interior product (D^-1, K^-1,
                              correction): the schedule, numbered as elem_sched,
                              of the whole product as one launch over items of
                              at most 16 columns, where the tuner found that
                              faster than the two width lists (products with an
                              item wider than 16 only); -1 the width lists run.
                              SMPM_ELEM_ALT = 1 with SMPM_ELEM_SCHED pins it
                              (tests, experiments) */
} smpm_info;

typedef struct smpm_handle smpm_handle;

/* One grid, nk wavenumbers (k >= 0; host array).  Each wavenumber is one
 * system with S(k) = I + B (A - k^2 I)^-1 E (Sec. 5).  k = 0 systems get the
 * null-space projections of Sec. 2.4 and need m_x >= 4 (else ESINGULAR).
 * hip_stream: hipStream_t used for the uploads (ignored when host-only). */
smpm_status smpm_setup(const smpm_grid *grid, const double *k, int32_t nk,
                       const smpm_opts *opts, void *hip_stream, smpm_handle **out);

/* nprob independent problems, each with its own grid and one wavenumber
 * k[p] (host arrays), solved as one batch.  Each problem is the 2-D system
 * of Sec. 2.2 (k = 0) or one Helmholtz mode of Sec. 5 (k > 0); batching
 * unrelated problems is not in the paper, whose modes share one grid. */
smpm_status smpm_setup_batch(const smpm_grid *grids, const double *k, int32_t nprob,
                             const smpm_opts *opts, void *hip_stream, smpm_handle **out);

/* The 3-D problem, periodic in y (Sec. 5, Alg. 3): m_y equispaced planes
 * y_j = j l_y / m_y.  One system per Fourier mode m = 0 .. m_y/2 with
 * k_m = 2 pi m / l_y, and two real right-hand sides (Re, Im) per mode (the
 * operator is real), so opts->nrhs must be 0 or 2.  m_y >= 2, l_y > 0. */
smpm_status smpm_setup_fourier(const smpm_grid *grid, int32_t my, double ly, const smpm_opts *opts,
                               void *hip_stream, smpm_handle **out);

/* Physical-space solve on a handle from smpm_setup_fourier.  f_dev: FP64
 * [m_y][r], plane j in the node layout; g_dev: FP64 [m_y][2 n (m_x + m_z)],
 * plane j in the side layout (S | N | W | E), or NULL; u_dev: FP64 [m_y][r].
 * The coefficients f_m = (1/m_y) sum_j f_j exp(-2 pi i m j / m_y) are solved
 * mode by mode with smpm_solve's Algorithm 2 (batched), and u_j is the real
 * Fourier series at y_j.  The k = 0 mode carries the zero-mean gauge.
 * Statuses and stats as for smpm_solve (counted over the 2 (m_y/2 + 1) real
 * instances); EINVAL on a handle not made by smpm_setup_fourier. */
smpm_status smpm_solve_fourier(smpm_handle *h, const double *f_dev, const double *g_dev, double *u_dev,
                               void *hip_stream, smpm_stats *stats);

/* The transform in y of Sec. 5 (Alg. 3) alone, on a handle from
 * smpm_setup_fourier: forward (inverse = 0) in_dev [m_y][r] planes ->
 * out_dev [m_y/2 + 1][2][r], the Re and Im parts of (1/m_y) sum_j f_j
 * exp(-2 pi i m j / m_y); inverse (inverse != 0) the other way, u_j = the
 * real Fourier series at y_j.  A radix-2 FFT when m_y is a power of two, else
 * a dense real DFT product.  Enqueued on hip_stream; in_dev and out_dev must
 * not overlap. */
smpm_status smpm_transform_y(smpm_handle *h, int32_t inverse, const double *in_dev, double *out_dev,
                             void *hip_stream);

/* Save every host table of a handle (its systems' operators, factors, coarse
 * operators and null vectors) to `path`, so that smpm_load can rebuild the
 * handle without the setup.  Works on host-only handles too.  EINVAL when
 * the file cannot be written. */
smpm_status smpm_save(const smpm_handle *h, const char *path);

/* Rebuild a handle from a file written by smpm_save: upload, schedule tuning
 * and the Fourier tables as in setup, no factorization.  opts NULL takes the
 * defaults with the saved deflation space; opts->zlabel must match the saved
 * one.  EINVAL for a missing, foreign or truncated file. */
smpm_status smpm_load(const char *path, const smpm_opts *opts, void *hip_stream, smpm_handle **out);

/* Algorithm 2 for every instance: f_dev (FP64, batched node layout), g_dev
 * (FP64, batched side layout, or NULL for g = 0) -> u_dev (FP64, batched node
 * layout, zero nodal mean for k = 0).  stats (host, nullable) is filled after
 * a stream synchronization.  ENOTCONV leaves the last iterate in u_dev. */
smpm_status smpm_solve(smpm_handle *h, const double *f_dev, const double *g_dev,
                       double *u_dev, void *hip_stream, smpm_stats *stats);

typedef enum {
  SMPM_OP_SCHUR = 0,    /* y = S x                    (k_S -> k_S), Sec. 2.3 */
  SMPM_OP_BJINV = 1,    /* y = M^-1 x                 (k_S -> k_S), Sec. 3.2 */
  SMPM_OP_DEFLATE_P = 2,/* y = P x                    (k_S -> k_S), Sec. 3.3 */
  SMPM_OP_DEFLATE_Q = 3,/* y = Q x                    (k_S -> k_S), Sec. 3.3 */
  SMPM_OP_AINV = 4,     /* y = A(k)^-1 x              (r -> r),     Sec. 2.3 */
  SMPM_OP_B = 5,        /* y = B x                    (r -> k_S),   Sec. 2.3 */
  SMPM_OP_SCHUR_RHS = 6,/* y = b~ from F (the projected Schur right-hand side of Algorithm 2; r -> k_S) */
  SMPM_OP_SCHUR_BJINV = 7 /* y = S M^-1 x (k_S -> k_S), the right-preconditioned
                           operator of Eq. (deflated_schur) without P;
                           smpm_apply_all only */
} smpm_op;

/* Apply one operator of system `sys` to one vector.  x_dev, y_dev: device
 * arrays of the sizes noted above, in the layouts of this header.
 * precision selects the FP64 or FP32 operator tables; x_dev and y_dev are
 * double for SMPM_FP64 and float for SMPM_FP32_IR (SCHUR and BJINV only). */
smpm_status smpm_apply(smpm_handle *h, smpm_op op, int32_t sys, const void *x_dev,
                       void *y_dev, int32_t precision, void *hip_stream);

/* Batched Schur matvec over every instance (Sec. 3.1: S applied as a sum of
 * per-strip block products): x_dev, y_dev hold the interface vectors of all
 * instances back to back (smpm_info.x_offset * nrhs layout), double for
 * SMPM_FP64, float for SMPM_FP32_IR and SMPM_FP16S_IR (the FP16 tables of an
 * FP16S_IR handle).  Enqueued on hip_stream without a synchronization.  This
 * is the kernel the matvec rate is measured on. */
smpm_status smpm_schur_apply_all(smpm_handle *h, const void *x_dev, void *y_dev,
                                 int32_t precision, void *hip_stream);

/* One operator over every instance at once, with the kernels and schedules
 * the solve uses, enqueued on hip_stream without a synchronization (for
 * timing a kernel of the solve on its own):
 *   SMPM_OP_SCHUR        y = S x             (Sec. 3.1),  as smpm_schur_apply_all;
 *   SMPM_OP_BJINV        y = M^-1 x          (Sec. 3.2);
 *   SMPM_OP_SCHUR_BJINV  y = S M^-1 x        (Eq. deflated_schur without P): one
 *                        GEMM over the stored S M^-1 blocks where the setup
 *                        chose them (smpm_info.fused_op), else M^-1 then S
 *                        through the handle's workspace;
 *   SMPM_OP_AINV         y = A(k)^-1 x       (Sec. 2.3; FP64, node layout, all
 *                        instances back to back).
 * Interface vectors as for smpm_schur_apply_all.  x_dev and y_dev must not
 * overlap (EINVAL when they are the same array).  EINVAL for other ops, an
 * unknown precision, FP16 on a handle without FP16 tables, or AINV in a
 * reduced precision. */
smpm_status smpm_apply_all(smpm_handle *h, smpm_op op, const void *x_dev, void *y_dev,
                           int32_t precision, void *hip_stream);

/* smpm_apply without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Ops SCHUR and BJINV (FP64, or FP32 with float x, y) and
 * DEFLATE_P, DEFLATE_Q (FP64) of system `sys`, with the same kernels, work
 * lists and results as smpm_apply; x_dev is read and y_dev written in place
 * (k_S values each; they must not overlap, EINVAL when equal).  The
 * intermediates (S x for Q, the Z^T partial sums, the coarse vector) go to
 * one fixed 16 MiB device array per GPU, held until the process ends;
 * systems needing more (k_S + the partial sums + d above 2^21 doubles)
 * return EINVAL.  Nothing in it has to start at zero: every call writes the
 * parts it reads.  Calls that overlap in time on one GPU share the array and
 * race.  Enqueued on hip_stream with no synchronization and no host copy.
 * The first call on a device looks the array's address up (a host-side
 * query, no allocation). */
smpm_status smpm_apply_noalloc(smpm_handle *h, smpm_op op, int32_t sys, const void *x_dev,
                               void *y_dev, int32_t precision, void *hip_stream);

/* Sizes, offsets, table counts and the schedules picked at setup of system
 * `sys` (host struct).  Not a computation of the paper: bookkeeping for
 * callers that lay out batched vectors (offsets) and for measurement. */
smpm_status smpm_query(const smpm_handle *h, int32_t sys, smpm_info *info);
/* Systems of a handle (0 for NULL). */
int32_t smpm_num_systems(const smpm_handle *h);

typedef enum {
  SMPM_TABLE_SCHUR_DENSE = 0, /* k_S x k_S row-major dense S (small grids only) */
  SMPM_TABLE_BJINV_DENSE = 1, /* k_S x k_S row-major dense M^-1 */
  SMPM_TABLE_COARSE_C = 2,    /* d x d row-major C = Z^T S Z */
  SMPM_TABLE_U_S = 3,         /* k_S, left null vector of S (k = 0) */
  SMPM_TABLE_U_L = 4,         /* r, left null vector of L (k = 0) */
  SMPM_TABLE_U_C = 5,         /* d, left null vector of C (k = 0) */
  SMPM_TABLE_SZ = 6,          /* k_S x d row-major S Z */
  SMPM_TABLE_SMINV_DENSE = 7  /* k_S x k_S row-major S M^-1 from the fused blocks
                                 (EUNSUPPORTED for grids without shared blocks) */
} smpm_table;

/* Copy a host-side operator table of system `sys` into host_out (count
 * doubles, must equal the table size).  Works on host-only handles; this is
 * how the setup is checked without a GPU. */
smpm_status smpm_export(const smpm_handle *h, smpm_table what, int32_t sys,
                        double *host_out, int64_t count);

void smpm_destroy(smpm_handle *h);
const char *smpm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SMPM_SCHUR_H */
