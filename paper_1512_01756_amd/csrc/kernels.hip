// HIP kernels of the SMPM Schur solver for gfx950 (wave64).
//
// Every kernel is batched over instances (system, right-hand side) through a
// work list; an instance whose GMRES has stopped exits at once.  Reductions
// are two-stage with a fixed order (per-workgroup partials, then a fixed
// tree), so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace smpm {

template <typename T> struct Tab;
template <> struct Tab<double> {
  __device__ static const double *W(const SysDev &s) { return s.W64; }
  __device__ static const double *M(const SysDev &s) { return s.M64; }
};
template <> struct Tab<float> {
  __device__ static const float *W(const SysDev &s) { return s.W32; }
  __device__ static const float *M(const SysDev &s) { return s.M32; }
};

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum over the workgroup; the result is valid in thread 0.
__device__ inline double block_sum(double v, double *lds4) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) lds4[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = (lds4[0] + lds4[1]) + (lds4[2] + lds4[3]);
  return s;
}

// ---------------------------------------------------------------------------
// Half-interface block GEMV (Sec. 3.1 Schur matvec, Sec. 3.2 block-Jacobi):
//   op 0:  y_h = x_h + W^_h x[w_win(h) N .. + 2N)      (S = I + sum_j W_j)
//   op 1:  y_h = Mc_h x[m_win(h) N .. + m_K(h))         (M^-1 row chunk)
// One workgroup per (instance, half).  The window is staged in LDS; each
// wave takes a quarter of the columns and each lane rows lane + 64 q, so a
// column of the column-major block is one coalesced read.
// x_vslot: read x from Krylov slot `iter` of the instance, scaled by
// scale[iter].  hsum: write the sum of y_h (for Z^T y).
template <typename TO, typename TX, typename TY>
__global__ __launch_bounds__(kBlock) void k_half_gemv(
    const SysDev *__restrict__ sys, const InstDev *__restrict__ ins, const int2 *__restrict__ work,
    int op, const TX *__restrict__ xbase, int x_vslot, const double *__restrict__ scale,
    TY *__restrict__ ybase, double *__restrict__ hsum, const GState *__restrict__ gs) {
  __shared__ double xw[4 * kMaxN];
  __shared__ double red[4 * kMaxN];
  __shared__ double lds4[4];
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, h = wk.y;
  if (gs && !gs[i].active) return;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int N = S.N;
  const int64_t kS = S.kS;
  int K;
  int64_t win;
  const TO *blk;
  if (op == 0) {
    K = 2 * N;
    win = (int64_t)S.w_win[h] * N;
    blk = Tab<TO>::W(S) + (size_t)S.w_id[h] * 2 * N * N;
  } else {
    K = S.m_K[h];
    win = (int64_t)S.m_win[h] * N;
    blk = Tab<TO>::M(S) + (size_t)S.m_id[h] * 4 * N * N;
  }
  const int it = gs ? gs[i].iter : 0;
  const TX *x = xbase + (x_vslot ? I.v_off + (int64_t)it * kS : I.x_off);
  const double xs = scale ? scale[I.st_off + it] : 1.0;
  for (int c = threadIdx.x; c < K; c += kBlock) {
    const int64_t idx = win + c;
    xw[c] = (idx >= 0 && idx < kS) ? (double)x[idx] * xs : 0.0;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c0 = (K * wave) >> 2, c1 = (K * (wave + 1)) >> 2;
  TO acc[kMaxRowsPerLane];
#pragma unroll
  for (int q = 0; q < kMaxRowsPerLane; ++q) acc[q] = (TO)0;
  for (int c = c0; c < c1; ++c) {
    const TO xv = (TO)xw[c];
    const TO *col = blk + (size_t)c * N;
#pragma unroll
    for (int q = 0; q < kMaxRowsPerLane; ++q) {
      const int row = lane + 64 * q;
      if (row < N) acc[q] += col[row] * xv;
    }
  }
#pragma unroll
  for (int q = 0; q < kMaxRowsPerLane; ++q) {
    const int row = lane + 64 * q;
    if (row < N) red[wave * N + row] = (double)acc[q];
  }
  __syncthreads();
  TY *y = ybase + I.x_off + (int64_t)h * N;
  double lsum = 0.0;
  for (int row = threadIdx.x; row < N; row += kBlock) {
    TO v = ((TO)red[row] + (TO)red[N + row]) + ((TO)red[2 * N + row] + (TO)red[3 * N + row]);
    double vd = (double)v;
    if (op == 0) vd += (double)x[(int64_t)h * N + row] * xs;
    const TY out = (TY)vd;
    y[row] = out;
    lsum += (double)out;
  }
  if (hsum) {
    const double s = block_sum(lsum, lds4);
    if (threadIdx.x == 0) hsum[I.hs_off + h] = s;
  }
}

// Coarse solve of the deflation (Sec. 3.3): t_c = sum of the two halves of
// interface c (= Z^T y), optionally t = tsub - t; c = G t with G the
// precomputed C^dagger (I - u_C u_C^T) (C^-1 for k > 0).  One workgroup per
// instance.
__global__ __launch_bounds__(kBlock) void k_coarse(const SysDev *__restrict__ sys,
                                                   const InstDev *__restrict__ ins,
                                                   const double *__restrict__ hsum,
                                                   const double *__restrict__ tsub,
                                                   double *__restrict__ tout,
                                                   double *__restrict__ cout,
                                                   const GState *__restrict__ gs) {
  __shared__ double t[1024];
  const int i = blockIdx.x;
  if (gs && !gs[i].active) return;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int d = S.d;
  for (int c = threadIdx.x; c < d; c += kBlock) {
    double v = hsum[I.hs_off + 2 * c] + hsum[I.hs_off + 2 * c + 1];
    if (tsub) v = tsub[I.c_off + c] - v;
    t[c] = v;
    if (tout) tout[I.c_off + c] = v;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < d; r += kBlock) {
    double acc = 0.0;
    for (int l = 0; l < d; ++l) acc += S.Gc[(size_t)l * d + r] * t[l];
    cout[I.c_off + r] = acc;
  }
}

// Arnoldi step, part 1: w = y - (S Z) c (the deflation P, Sec. 3.3; c = null
// skips it), stored in Krylov slot iter + 1; partial dots V_t . w, t <= iter.
template <typename TV, typename TY>
__global__ __launch_bounds__(kBlock) void k_pcorr_dot(
    const SysDev *__restrict__ sys, const InstDev *__restrict__ ins, const int2 *__restrict__ work,
    const TY *__restrict__ ybase, const double *__restrict__ cvec, TV *__restrict__ V,
    double *__restrict__ part, const GState *__restrict__ gs, int maxit) {
  extern __shared__ double red[];   // (maxit + 1) * 4
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  if (!gs[i].active) return;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int N = S.N;
  const int64_t kS = S.kS;
  const int j = gs[i].iter;
  const int64_t e0 = (int64_t)ch * kChunk;
  double wv[kChunk / kBlock];
#pragma unroll
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = e0 + threadIdx.x + q * kBlock;
    double w = 0.0;
    if (e < kS) {
      w = (double)ybase[I.x_off + e];
      if (cvec) {
        const int h = (int)(e / N), row = (int)(e - (int64_t)h * N);
        const int ca = S.sz_col[2 * h], cb = S.sz_col[2 * h + 1];
        if (ca >= 0) w -= S.SZh[((size_t)2 * h) * N + row] * cvec[I.c_off + ca];
        if (cb >= 0) w -= S.SZh[((size_t)2 * h + 1) * N + row] * cvec[I.c_off + cb];
      }
      const TV wt = (TV)w;
      V[I.v_off + (int64_t)(j + 1) * kS + e] = wt;
      w = (double)wt;
    }
    wv[q] = w;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int t = 0; t <= j; ++t) {
    const TV *Vt = V + I.v_off + (int64_t)t * kS;
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < kChunk / kBlock; ++q) {
      const int64_t e = e0 + threadIdx.x + q * kBlock;
      if (e < kS) a += (double)Vt[e] * wv[q];
    }
    a = wave_sum(a);
    if (lane == 0) red[t * 4 + wave] = a;
  }
  __syncthreads();
  for (int t = threadIdx.x; t <= j; t += kBlock)
    part[I.part_off + (int64_t)t * I.nchunk_x + ch] = (red[t * 4] + red[t * 4 + 1]) + (red[t * 4 + 2] + red[t * 4 + 3]);
}

// Reduce the chunk partials of pass `part` into coef[t] = s_t^2 sum(...)
// (the coefficient of V_t in w -= sum_t h_t v_t, v_t = s_t V_t).
__device__ inline void reduce_coef(const InstDev &I, const double *__restrict__ part,
                                   const double *__restrict__ scale, int j, double *coef) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int t = wave; t <= j; t += 4) {
    const double *p = part + I.part_off + (int64_t)t * I.nchunk_x;
    double a = 0.0;
    for (int c = lane; c < I.nchunk_x; c += 64) a += p[c];
    a = wave_sum(a);
    if (lane == 0) {
      const double s = scale[I.st_off + t];
      coef[t] = s * s * a;
    }
  }
  __syncthreads();
}

// Classical Gram-Schmidt pass: w -= sum_t coef_t V_t (coef from the partials
// of the previous pass); then either the next pass's partial dots
// (part_out) or the partial squared norm (partn).
template <typename TV>
__global__ __launch_bounds__(kBlock) void k_axpy_dot(
    const SysDev *__restrict__ sys, const InstDev *__restrict__ ins, const int2 *__restrict__ work,
    TV *__restrict__ V, const double *__restrict__ part_in, double *__restrict__ part_out,
    double *__restrict__ partn, const double *__restrict__ scale, const GState *__restrict__ gs) {
  extern __shared__ double sh[];   // coef[maxit + 1] then red[(maxit + 1) * 4]
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  if (!gs[i].active) return;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int64_t kS = S.kS;
  const int j = gs[i].iter;
  double *coef = sh;
  double *red = sh + (j + 1);
  reduce_coef(I, part_in, scale, j, coef);
  const int64_t e0 = (int64_t)ch * kChunk;
  TV *w = V + I.v_off + (int64_t)(j + 1) * kS;
  double wv[kChunk / kBlock];
#pragma unroll
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = e0 + threadIdx.x + q * kBlock;
    double a = 0.0;
    if (e < kS) {
      a = (double)w[e];
      for (int t = 0; t <= j; ++t) a -= coef[t] * (double)V[I.v_off + (int64_t)t * kS + e];
      const TV at = (TV)a;
      w[e] = at;
      a = (double)at;
    }
    wv[q] = a;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (part_out) {
    for (int t = 0; t <= j; ++t) {
      const TV *Vt = V + I.v_off + (int64_t)t * kS;
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < kChunk / kBlock; ++q) {
        const int64_t e = e0 + threadIdx.x + q * kBlock;
        if (e < kS) a += (double)Vt[e] * wv[q];
      }
      a = wave_sum(a);
      if (lane == 0) red[t * 4 + wave] = a;
    }
    __syncthreads();
    for (int t = threadIdx.x; t <= j; t += kBlock)
      part_out[I.part_off + (int64_t)t * I.nchunk_x + ch] =
          (red[t * 4] + red[t * 4 + 1]) + (red[t * 4 + 2] + red[t * 4 + 3]);
  } else {
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < kChunk / kBlock; ++q) a += wv[q] * wv[q];
    a = wave_sum(a);
    if (lane == 0) red[wave] = a;
    __syncthreads();
    if (threadIdx.x == 0) partn[I.part_off + ch] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// Hessenberg column, Givens rotations and the residual estimate (one
// workgroup per instance).  h_t = s_t (sum part1 + sum part2), h_{j+1} = ||w||.
__global__ __launch_bounds__(kBlock) void k_givens(
    const InstDev *__restrict__ ins, const double *__restrict__ part1, const double *__restrict__ part2,
    const double *__restrict__ partn, double *__restrict__ scale, double *__restrict__ R,
    double *__restrict__ cs, double *__restrict__ sn, double *__restrict__ g, GState *__restrict__ gs,
    int maxit, double tol) {
  extern __shared__ double h[];   // maxit + 2
  __shared__ double lds4[4];
  const int i = blockIdx.x;
  if (!gs[i].active) return;
  const InstDev I = ins[i];
  const int j = gs[i].iter;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int t = wave; t <= j; t += 4) {
    const double *p1 = part1 + I.part_off + (int64_t)t * I.nchunk_x;
    const double *p2 = part2 + I.part_off + (int64_t)t * I.nchunk_x;
    double a = 0.0, b = 0.0;
    for (int c = lane; c < I.nchunk_x; c += 64) { a += p1[c]; b += p2[c]; }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) h[t] = scale[I.st_off + t] * (a + b);
  }
  double nn = 0.0;
  for (int c = threadIdx.x; c < I.nchunk_x; c += kBlock) nn += partn[I.part_off + c];
  nn = block_sum(nn, lds4);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double beta = sqrt(nn);
    h[j + 1] = beta;
    double *csI = cs + I.st_off, *snI = sn + I.st_off, *gI = g + I.st_off;
    for (int t = 0; t < j; ++t) {
      const double a = csI[t] * h[t] + snI[t] * h[t + 1];
      h[t + 1] = -snI[t] * h[t] + csI[t] * h[t + 1];
      h[t] = a;
    }
    const double den = hypot(h[j], h[j + 1]);
    const double c = den != 0.0 ? h[j] / den : 1.0;
    const double s = den != 0.0 ? h[j + 1] / den : 0.0;
    csI[j] = c;
    snI[j] = s;
    h[j] = den;
    gI[j + 1] = -s * gI[j];
    gI[j] = c * gI[j];
    double *Rc = R + I.rr_off + (int64_t)j * maxit;
    for (int t = 0; t <= j; ++t) Rc[t] = h[t];
    const double res = fabs(gI[j + 1]);
    GState st = gs[i];
    st.iter = j + 1;
    st.res = res;
    if (!isfinite(res) || !isfinite(den)) {
      st.active = 0; st.status = 3;
    } else if (res <= tol * st.ref || beta == 0.0) {
      st.active = 0; st.status = 1;
    } else if (j + 1 >= maxit) {
      st.active = 0; st.status = 2;
    } else {
      scale[I.st_off + j + 1] = 1.0 / beta;
    }
    gs[i] = st;
  }
}

// Least squares R y = g (upper triangular, m = iter columns); writes
// ycoef[t] = y_t s_t for the basis combination.
__global__ __launch_bounds__(kBlock) void k_backsolve(const InstDev *__restrict__ ins,
                                                      const double *__restrict__ R,
                                                      const double *__restrict__ g,
                                                      const double *__restrict__ scale,
                                                      double *__restrict__ ycoef,
                                                      const GState *__restrict__ gs, int maxit) {
  extern __shared__ double rhs[];
  const int i = blockIdx.x;
  const InstDev I = ins[i];
  const int m = gs[i].iter;
  for (int t = threadIdx.x; t < m; t += kBlock) rhs[t] = g[I.st_off + t];
  __syncthreads();
  for (int c = m - 1; c >= 0; --c) {
    const double *Rc = R + I.rr_off + (int64_t)c * maxit;
    const double yc = rhs[c] / Rc[c];
    __syncthreads();
    for (int t = threadIdx.x; t < c; t += kBlock) rhs[t] -= Rc[t] * yc;
    if (threadIdx.x == 0) rhs[c] = yc;
    __syncthreads();
  }
  for (int t = threadIdx.x; t < m; t += kBlock) ycoef[I.st_off + t] = rhs[t] * scale[I.st_off + t];
}

// x = sum_{t < m} ycoef_t V_t  (interface space, per instance).
template <typename TV, typename TY>
__global__ __launch_bounds__(kBlock) void k_combine(const SysDev *__restrict__ sys,
                                                    const InstDev *__restrict__ ins,
                                                    const int2 *__restrict__ work,
                                                    const TV *__restrict__ V,
                                                    const double *__restrict__ ycoef,
                                                    TY *__restrict__ out, const GState *__restrict__ gs) {
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];
  const int64_t kS = sys[I.sys].kS;
  const int m = gs[i].iter;
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = (int64_t)ch * kChunk + threadIdx.x + q * kBlock;
    if (e >= kS) continue;
    double a = 0.0;
    for (int t = 0; t < m; ++t) a += ycoef[I.st_off + t] * (double)V[I.v_off + (int64_t)t * kS + e];
    out[I.x_off + e] = (TY)a;
  }
}

// ---------------------------------------------------------------------------
// Element-interior elimination (Sec. 2.3): A(k)^-1 per strip by block
// elimination over the m_z elements with the precomputed inverse Schur
// blocks G_e.  One workgroup per (instance, strip).
__global__ __launch_bounds__(kBlock) void k_strip_solve(const SysDev *__restrict__ sys,
                                                        const InstDev *__restrict__ ins,
                                                        const int2 *__restrict__ work,
                                                        const double *__restrict__ src,
                                                        double *__restrict__ dst) {
  __shared__ double rl[512];
  __shared__ double qv[32];
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, j = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int n = S.n, n2 = S.n2, mz = S.mz;
  const double *Gcl = S.Gs + (size_t)S.strip_class[j] * mz * n2 * n2;
  const double *in = src + I.f_off + (int64_t)j * mz * n2;
  double *out = dst + I.f_off + (int64_t)j * mz * n2;
  for (int e = 0; e < mz; ++e) {
    for (int l = threadIdx.x; l < n2; l += kBlock) rl[l] = in[(int64_t)e * n2 + l];
    __syncthreads();
    if (e > 0 && threadIdx.x < n) {
      const int t = threadIdx.x;
      const double *prev = out + (int64_t)(e - 1) * n2;
      double a = 0.0;
      for (int c = 0; c < n; ++c) a += S.lo[e * n + c] * prev[c * n + t];
      rl[t] -= a;   // row (0, t)
    }
    __syncthreads();
    const double *Ge = Gcl + (size_t)e * n2 * n2;
    for (int row = threadIdx.x; row < n2; row += kBlock) {
      double a = 0.0;
      for (int l = 0; l < n2; ++l) a += Ge[(size_t)l * n2 + row] * rl[l];
      out[(int64_t)e * n2 + row] = a;
    }
    __syncthreads();
  }
  for (int e = mz - 2; e >= 0; --e) {
    if (threadIdx.x < n) {
      const int t = threadIdx.x;
      const double *nx = out + (int64_t)(e + 1) * n2;
      double a = 0.0;
      for (int c = 0; c < n; ++c) a += S.up[e * n + c] * nx[c * n + t];
      qv[t] = a;
    }
    __syncthreads();
    const double *Ge = Gcl + (size_t)e * n2 * n2;
    for (int row = threadIdx.x; row < n2; row += kBlock) {
      double a = out[(int64_t)e * n2 + row];
      for (int t = 0; t < n; ++t) a -= Ge[(size_t)((n - 1) * n + t) * n2 + row] * qv[t];
      out[(int64_t)e * n2 + row] = a;
    }
    __syncthreads();
  }
}

// RHS of Eq. (smpm_poisson): F = f + tau g on the physical edges (corners get
// both sides); partials of u_L . F and ||F||^2 for the Sec. 2.4 projection.
__global__ __launch_bounds__(kBlock) void k_rhs(const SysDev *__restrict__ sys,
                                                const InstDev *__restrict__ ins,
                                                const int2 *__restrict__ work,
                                                const double *__restrict__ f,
                                                const double *__restrict__ g,
                                                double *__restrict__ F, double *__restrict__ pr) {
  __shared__ double lds4[4];
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int n = S.n, mz = S.mz, mx = S.mx;
  double pd = 0.0, pn = 0.0;
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = (int64_t)ch * kChunk + threadIdx.x + q * kBlock;
    if (e >= S.r) continue;
    int64_t rem = e;
    const int a = (int)(rem % n); rem /= n;
    const int b = (int)(rem % n); rem /= n;
    const int el = (int)(rem % mz);
    const int j = (int)(rem / mz);
    double v = f[I.f_off + e];
    if (g) {
      const double *gg = g + I.g_off;
      const double *gS = gg, *gN = gg + (size_t)mx * n, *gW = gg + (size_t)2 * mx * n, *gE = gW + (size_t)mz * n;
      double add = 0.0;
      if (el == 0 && b == 0) add += gS[j * n + a];
      if (el == mz - 1 && b == n - 1) add += gN[j * n + a];
      if (j == 0 && a == 0) add += gW[el * n + b];
      if (j == mx - 1 && a == n - 1) add += gE[el * n + b];
      v += S.tau * add;
    }
    F[I.f_off + e] = v;
    if (S.singular) pd += S.uL[e] * v;
    pn += v * v;
  }
  pd = block_sum(pd, lds4);
  __syncthreads();
  pn = block_sum(pn, lds4);
  if (threadIdx.x == 0) {
    pr[I.pr_off + 2 * ch] = pd;
    pr[I.pr_off + 2 * ch + 1] = pn;
  }
}

// F~ = F - u_L (u_L^T F) (Eq. regularize_poisson); every workgroup reduces
// the partials in the same order; the first one records the defect.
__global__ __launch_bounds__(kBlock) void k_proj_r(const SysDev *__restrict__ sys,
                                                   const InstDev *__restrict__ ins,
                                                   const int2 *__restrict__ work,
                                                   double *__restrict__ F,
                                                   const double *__restrict__ pr,
                                                   double *__restrict__ defect) {
  __shared__ double lds4[4];
  __shared__ double alpha_s;
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  if (!S.singular) return;
  double a = 0.0, b = 0.0;
  for (int c = threadIdx.x; c < I.nchunk_r; c += kBlock) { a += pr[I.pr_off + 2 * c]; b += pr[I.pr_off + 2 * c + 1]; }
  a = block_sum(a, lds4);
  __syncthreads();
  b = block_sum(b, lds4);
  if (threadIdx.x == 0) {
    alpha_s = a;
    if (ch == 0) defect[i] = b > 0.0 ? fabs(a) / sqrt(b) : 0.0;
  }
  __syncthreads();
  const double alpha = alpha_s;
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = (int64_t)ch * kChunk + threadIdx.x + q * kBlock;
    if (e < S.r) F[I.f_off + e] -= alpha * S.uL[e];
  }
}

// b_S = B v (Sec. 2.3): the row of a node of half h reads the facing strip's
// edge element row: -tau (v + n . grad v).  One workgroup per (instance, h);
// writes the partial of u_S . b_S into hs.
__global__ __launch_bounds__(kBlock) void k_bS(const SysDev *__restrict__ sys,
                                               const InstDev *__restrict__ ins,
                                               const int2 *__restrict__ work,
                                               const double *__restrict__ v,
                                               double *__restrict__ bS, double *__restrict__ hs) {
  __shared__ double lds4[4];
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, h = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int n = S.n, n2 = S.n2, mz = S.mz, N = S.N;
  const int iface = h >> 1;
  const bool even = (h & 1) == 0;
  const int strip = even ? iface + 1 : iface;
  const double *beta = S.beta + (size_t)S.strip_class[strip] * 2 * n + (even ? 0 : n);
  double pd = 0.0;
  for (int row = threadIdx.x; row < N; row += kBlock) {
    const int e = row / n, b = row - e * n;
    const double *vr = v + I.f_off + ((int64_t)strip * mz + e) * n2 + (int64_t)b * n;
    double a = 0.0;
    for (int c = 0; c < n; ++c) a += beta[c] * vr[c];
    bS[I.x_off + (int64_t)h * N + row] = a;
    if (S.singular) pd += S.uS[(int64_t)h * N + row] * a;
  }
  pd = block_sum(pd, lds4);
  if (threadIdx.x == 0) hs[I.hs_off + h] = pd;
}

// b~ = b_S - u_S (u_S^T b_S) (Eq. regularize_schur), partials per half in hs.
__global__ __launch_bounds__(kBlock) void k_proj_x(const SysDev *__restrict__ sys,
                                                   const InstDev *__restrict__ ins,
                                                   const int2 *__restrict__ work,
                                                   double *__restrict__ x,
                                                   const double *__restrict__ hs) {
  __shared__ double lds4[4];
  __shared__ double alpha_s;
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  if (!S.singular) return;
  double a = 0.0;
  for (int c = threadIdx.x; c < S.nh; c += kBlock) a += hs[I.hs_off + c];
  a = block_sum(a, lds4);
  if (threadIdx.x == 0) alpha_s = a;
  __syncthreads();
  const double alpha = alpha_s;
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = (int64_t)ch * kChunk + threadIdx.x + q * kBlock;
    if (e < S.kS) x[I.x_off + e] -= alpha * S.uS[e];
  }
}

// Sum of each half of an interface vector (Z^T x, two halves per
// interface), and optionally the partial of u_S . x.
__global__ __launch_bounds__(kBlock) void k_halfsum(const SysDev *__restrict__ sys,
                                                    const InstDev *__restrict__ ins,
                                                    const int2 *__restrict__ work,
                                                    const double *__restrict__ x,
                                                    double *__restrict__ hs,
                                                    double *__restrict__ hdot) {
  __shared__ double lds4[4];
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, h = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int N = S.N;
  double a = 0.0, b = 0.0;
  for (int row = threadIdx.x; row < N; row += kBlock) {
    const double v = x[I.x_off + (int64_t)h * N + row];
    a += v;
    if (hdot && S.singular) b += S.uS[(int64_t)h * N + row] * v;
  }
  a = block_sum(a, lds4);
  __syncthreads();
  if (hdot) b = block_sum(b, lds4);
  if (threadIdx.x == 0) {
    hs[I.hs_off + h] = a;
    if (hdot) hdot[I.hs_off + h] = b;
  }
}

// r0 = P b~ = b~ - (S Z) c into Krylov slot 0 (or b~ itself without
// deflation); partial ||r0||^2.
template <typename TV>
__global__ __launch_bounds__(kBlock) void k_init_basis(const SysDev *__restrict__ sys,
                                                       const InstDev *__restrict__ ins,
                                                       const int2 *__restrict__ work,
                                                       const double *__restrict__ b,
                                                       const double *__restrict__ cvec,
                                                       TV *__restrict__ V, double *__restrict__ partn) {
  __shared__ double lds4[4];
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int N = S.N;
  double nn = 0.0;
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = (int64_t)ch * kChunk + threadIdx.x + q * kBlock;
    if (e >= S.kS) continue;
    double w = b[I.x_off + e];
    if (cvec) {
      const int h = (int)(e / N), row = (int)(e - (int64_t)h * N);
      const int ca = S.sz_col[2 * h], cb = S.sz_col[2 * h + 1];
      if (ca >= 0) w -= S.SZh[((size_t)2 * h) * N + row] * cvec[I.c_off + ca];
      if (cb >= 0) w -= S.SZh[((size_t)2 * h + 1) * N + row] * cvec[I.c_off + cb];
    }
    const TV wt = (TV)w;
    V[I.v_off + e] = wt;
    nn += (double)wt * (double)wt;
  }
  nn = block_sum(nn, lds4);
  if (threadIdx.x == 0) partn[I.part_off + ch] = nn;
}

// GMRES start: r0 = sqrt(sum partn), g_0 = r0, s_0 = 1/r0.  The stopping
// test is |g| <= tol * ref with ref = sqrt(pairs[2 i]) (the norm of the
// Schur right-hand side, the quantity of the acceptance test) or r0.
__global__ __launch_bounds__(kBlock) void k_gmres_start(const InstDev *__restrict__ ins,
                                                        const double *__restrict__ partn,
                                                        const double *__restrict__ pairs,
                                                        double *__restrict__ scale,
                                                        double *__restrict__ g, GState *__restrict__ gs,
                                                        int enable) {
  __shared__ double lds4[4];
  const int i = blockIdx.x;
  const InstDev I = ins[i];
  double nn = 0.0;
  for (int c = threadIdx.x; c < I.nchunk_x; c += kBlock) nn += partn[I.part_off + c];
  nn = block_sum(nn, lds4);
  if (threadIdx.x == 0) {
    const double r0 = sqrt(nn);
    GState st;
    st.iter = 0;
    st.r0 = r0;
    st.res = r0;
    st.pad = 0;
    st.ref = pairs ? sqrt(pairs[2 * i]) : r0;
    if (!isfinite(r0)) { st.active = 0; st.status = 3; }
    else if (r0 == 0.0 || !enable) { st.active = 0; st.status = 1; }
    else { st.active = 1; st.status = 0; }
    gs[i] = st;
    scale[I.st_off] = r0 > 0.0 ? 1.0 / r0 : 0.0;
    g[I.st_off] = r0;
  }
}

// Elementwise interface-space helpers.
// mode 0: out = a + Z c          (x_S = z + Z c')
// mode 1: out = out + a + Z c    (refinement update)
// mode 2: out = a - out          (residual r = b - S x), partials ||r||^2 and u_S . r
template <typename TA>
__global__ __launch_bounds__(kBlock) void k_xupdate(const SysDev *__restrict__ sys,
                                                    const InstDev *__restrict__ ins,
                                                    const int2 *__restrict__ work, int mode,
                                                    const TA *__restrict__ a,
                                                    const double *__restrict__ cvec,
                                                    double *__restrict__ out,
                                                    double *__restrict__ partn) {
  __shared__ double lds4[4];
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int N = S.N;
  double nn = 0.0, ud = 0.0;
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = (int64_t)ch * kChunk + threadIdx.x + q * kBlock;
    if (e >= S.kS) continue;
    const int iface = (int)(e / N) >> 1;
    double v = a ? (double)a[I.x_off + e] : 0.0;
    if (mode == 2) {
      v = out[I.x_off + e] - v;   // out holds b
      out[I.x_off + e] = v;
      nn += v * v;
      if (S.singular) ud += S.uS[e] * v;
      continue;
    }
    if (cvec) v += cvec[I.c_off + iface];
    if (mode == 1) v += out[I.x_off + e];
    out[I.x_off + e] = v;
  }
  if (mode == 2) {
    nn = block_sum(nn, lds4);
    __syncthreads();
    ud = block_sum(ud, lds4);
    if (threadIdx.x == 0) {
      partn[I.part_off + 2 * ch] = nn;
      partn[I.part_off + 2 * ch + 1] = ud;
    }
  }
}

// Recovery right-hand side (Algorithm 2, step 9): R = F~ - E x_S.
__global__ __launch_bounds__(kBlock) void k_recover_rhs(const SysDev *__restrict__ sys,
                                                        const InstDev *__restrict__ ins,
                                                        const int2 *__restrict__ work,
                                                        const double *__restrict__ F,
                                                        const double *__restrict__ xS,
                                                        double *__restrict__ R) {
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int n = S.n, mz = S.mz, mx = S.mx, N = S.N;
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = (int64_t)ch * kChunk + threadIdx.x + q * kBlock;
    if (e >= S.r) continue;
    int64_t rem = e;
    const int a = (int)(rem % n); rem /= n;
    const int b = (int)(rem % n); rem /= n;
    const int el = (int)(rem % mz);
    const int j = (int)(rem / mz);
    double v = F[I.f_off + e];
    const int row = el * n + b;
    if (a == n - 1 && j <= mx - 2) v -= xS[I.x_off + (int64_t)(2 * j) * N + row];
    if (a == 0 && j >= 1) v -= xS[I.x_off + (int64_t)(2 * j - 1) * N + row];
    R[I.f_off + e] = v;
  }
}

// Gauge fix for k = 0: subtract the nodal mean (two kernels: partials, apply).
__global__ __launch_bounds__(kBlock) void k_sum_r(const SysDev *__restrict__ sys,
                                                  const InstDev *__restrict__ ins,
                                                  const int2 *__restrict__ work,
                                                  const double *__restrict__ u, double *__restrict__ pr) {
  __shared__ double lds4[4];
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  double a = 0.0;
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = (int64_t)ch * kChunk + threadIdx.x + q * kBlock;
    if (e < S.r) a += u[I.f_off + e];
  }
  a = block_sum(a, lds4);
  if (threadIdx.x == 0) pr[I.pr_off + 2 * ch] = a;
}

__global__ __launch_bounds__(kBlock) void k_sub_mean(const SysDev *__restrict__ sys,
                                                     const InstDev *__restrict__ ins,
                                                     const int2 *__restrict__ work,
                                                     double *__restrict__ u, const double *__restrict__ pr) {
  __shared__ double lds4[4];
  __shared__ double mean_s;
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  if (!S.singular) return;
  double a = 0.0;
  for (int c = threadIdx.x; c < I.nchunk_r; c += kBlock) a += pr[I.pr_off + 2 * c];
  a = block_sum(a, lds4);
  if (threadIdx.x == 0) mean_s = a / (double)S.r;
  __syncthreads();
  const double mean = mean_s;
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = (int64_t)ch * kChunk + threadIdx.x + q * kBlock;
    if (e < S.r) u[I.f_off + e] -= mean;
  }
}

// Reduce interface-space partial pairs (||r||^2, u_S . r) to one instance
// scalar pair: out[2 i], out[2 i + 1].
__global__ __launch_bounds__(kBlock) void k_reduce_pairs(const InstDev *__restrict__ ins,
                                                         const double *__restrict__ partn,
                                                         double *__restrict__ out) {
  __shared__ double lds4[4];
  const int i = blockIdx.x;
  const InstDev I = ins[i];
  double a = 0.0, b = 0.0;
  for (int c = threadIdx.x; c < I.nchunk_x; c += kBlock) { a += partn[I.part_off + 2 * c]; b += partn[I.part_off + 2 * c + 1]; }
  a = block_sum(a, lds4);
  __syncthreads();
  b = block_sum(b, lds4);
  if (threadIdx.x == 0) { out[2 * i] = a; out[2 * i + 1] = b; }
}

// r <- r - u_S (u_S . r) using a reduced scalar (refinement residual).
__global__ __launch_bounds__(kBlock) void k_proj_x_scalar(const SysDev *__restrict__ sys,
                                                          const InstDev *__restrict__ ins,
                                                          const int2 *__restrict__ work,
                                                          double *__restrict__ x,
                                                          const double *__restrict__ pairs) {
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  if (!S.singular) return;
  const double alpha = pairs[2 * i + 1];
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = (int64_t)ch * kChunk + threadIdx.x + q * kBlock;
    if (e < S.kS) x[I.x_off + e] -= alpha * S.uS[e];
  }
}

// Precision conversion of an interface vector (double -> float etc.).
template <typename TA, typename TB>
__global__ __launch_bounds__(kBlock) void k_convert(const SysDev *__restrict__ sys,
                                                    const InstDev *__restrict__ ins,
                                                    const int2 *__restrict__ work,
                                                    const TA *__restrict__ a, TB *__restrict__ b) {
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = (int64_t)ch * kChunk + threadIdx.x + q * kBlock;
    if (e < S.kS) b[I.x_off + e] = (TB)a[I.x_off + e];
  }
}

}  // namespace smpm
