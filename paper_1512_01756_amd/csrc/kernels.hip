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
// Operator tables by storage type.  FP16 rows carry a per-(block, element
// segment) scale, applied to the product row in the epilogue.
template <> struct Tab<double> {
  __device__ static const double *W(const SysDev &s) { return s.W64; }
  __device__ static const double *M(const SysDev &s) { return s.M64; }
  __device__ static const double *blk(const GWork &w) { return w.blk64; }
  __device__ static float rs(const GWork &, int) { return 1.0f; }
  __device__ static float rs(const SysDev &, int, int, int) { return 1.0f; }
};
template <> struct Tab<float> {
  __device__ static const float *W(const SysDev &s) { return s.W32; }
  __device__ static const float *M(const SysDev &s) { return s.M32; }
  __device__ static const float *blk(const GWork &w) { return w.blk32; }
  __device__ static float rs(const GWork &, int) { return 1.0f; }
  __device__ static float rs(const SysDev &, int, int, int) { return 1.0f; }
};
template <> struct Tab<_Float16> {
  __device__ static const _Float16 *W(const SysDev &s) { return s.W16; }
  __device__ static const _Float16 *M(const SysDev &s) { return s.M16; }
  __device__ static const _Float16 *blk(const GWork &w) { return w.blk16; }
  __device__ static float rs(const GWork &w, int row) { return w.sc16[row / w.n]; }
  __device__ static float rs(const SysDev &s, int op, int id, int row) {
    return (op == 0 ? s.W16s : s.M16s)[(size_t)id * s.mz + row / s.n];
  }
};

// Deflation space Z (Sec. 3.3): coarse column of interface row `row` of half
// h (one column per interface, or one per element segment of n rows), and
// (S Z c) at that row from the half's 2 zm columns of S Z; c is indexed from
// coarse column `c0`.
__device__ inline int z_col(const SysDev &S, int h, int row) {
  return (h >> 1) * S.zm + (S.zm > 1 ? row / S.n : 0);
}
__device__ inline double sz_c(const SysDev &S, int h, int row, const double *__restrict__ c, int c0) {
  const int m = 2 * S.zm;
  double a = 0.0;
  for (int p = 0; p < m; ++p) {
    const int col = S.sz_col[(size_t)h * m + p];
    if (col >= 0) a += S.SZh[((size_t)h * m + p) * S.N + row] * c[col - c0];
  }
  return a;
}
// Z^T partial sums.  With zm = 1 the array holds per-(16-row slot, half)
// sums, slot-major: [slot q][half h] (the GEMM epilogues write them; a
// half's sum is the sum over its slots, and the halves 2c, 2c + 1 of
// interface c sit side by side, so a thread per interface reads 16 bytes per
// slot and neighbouring threads read neighbouring bytes).  Else [half][e],
// one sum per element segment.
__device__ inline int hs_slots(const SysDev &S) {
  const int tiles = (S.N + 15) >> 4;
  return S.zm > 1 ? S.zm : tiles;
}

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
// Column-split GEMV core: lane `lane` owns row `row` (< R) of a column-major
// block with leading dimension ld and accumulates columns [c0, c1) for G
// right-hand sides held in LDS (xw[g * xs + c]).  Loads are issued UNROLL
// columns at a time.
template <typename TO, int G, int UNROLL>
__device__ inline void colsplit(const TO *__restrict__ blk, int R, int row, int c0, int c1,
                                const double *xw, int xs, TO (&acc)[G], int ld = -1) {
  if (ld < 0) ld = R;
  const int Rl = ld;
  const bool live = row < R;
  const TO *col = blk + row;
  int c = c0;
  for (; c + UNROLL <= c1; c += UNROLL) {
    TO v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) v[u] = live ? col[(size_t)(c + u) * Rl] : (TO)0;
#pragma unroll
    for (int u = 0; u < UNROLL; ++u)
#pragma unroll
      for (int g = 0; g < G; ++g) acc[g] += v[u] * (TO)xw[g * xs + c + u];
  }
  for (; c < c1; ++c) {
    const TO v = live ? col[(size_t)c * Rl] : (TO)0;
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] += v * (TO)xw[g * xs + c];
  }
}

// ---------------------------------------------------------------------------
// Half-interface block GEMV (Sec. 3.1 Schur matvec, Sec. 3.2 block-Jacobi):
//   op 0:  y_h = x_h + W^_h x[w_win(h) N .. + 2N)      (S = I + sum_j W_j)
//   op 1:  y_h = Mc_h x[m_win(h) N .. + m_K(h))         (M^-1 row chunk)
// Two kernels cover the halves: a streaming GEMV for blocks used by one half
// (distinct strips, HBM bound) and an MFMA GEMM for blocks shared by many
// halves (uniform strips).  x_vslot: read x from Krylov slot `iter` of the
// instance, scaled by scale[iter].  hsum: per-(16-row slot, half) partial sums
// of y, hsum[hs_off + slot * nh + h] (for Z^T y).
//
// Streaming variant for halves whose block is not shared (distinct strips):
// one half per workgroup row tile, vector loads of VR consecutive rows per
// lane along each column of the padded column-major block, NW waves splitting
// the columns.  Same operation and outputs as the MFMA GEMM with one half per
// item.
// Vector load of VR = 4 consecutive rows of one column: 32 bytes (two 16-byte
// loads) in FP64, 16 in FP32, 8 in FP16, so a tile is 256 rows in every
// precision and one tile covers a half of up to 256 rows: the workgroup then
// reads each column's rows as one contiguous run.
struct alignas(8) half4 {
  _Float16 v[4];
};
struct alignas(32) dbl4 {
  double v[4];
};
template <typename TS> struct Vec16;
template <> struct Vec16<double> { using T = dbl4; static constexpr int R = 4; };
template <> struct Vec16<float> { using T = float4; static constexpr int R = 4; };
template <> struct Vec16<_Float16> { using T = half4; static constexpr int R = 4; };

// TS: storage type of the operator tables; TO: arithmetic type.
template <typename TS, typename TO, typename TX, typename TY, int NW>
__global__ __launch_bounds__(64 * NW) void k_half_gemv_stream(
    const SysDev *__restrict__ sys, const InstDev *__restrict__ ins, const HWork *__restrict__ work,
    int op, const TX *__restrict__ xbase, int x_vslot, const double *__restrict__ scale,
    TY *__restrict__ ybase, double *__restrict__ hsum, const GState *__restrict__ gs) {
  using V = typename Vec16<TS>::T;
  constexpr int VR = Vec16<TS>::R;
  constexpr int TR = 64 * VR;
  extern __shared__ double sm[];
  const int i = work[blockIdx.x].inst;
  if (gs && !gs[i].active) return;
  const int h = work[blockIdx.x].h[0];
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int N = S.N, Np = S.Np;
  const int tiles = (N + TR - 1) / TR;
  const int tile = blockIdx.y;
  if (tile >= tiles) return;
  const int64_t kS = S.kS;
  int K, bid;
  const TS *blk;
  int64_t win;
  if (op == 0) {
    K = 2 * N;
    bid = S.w_id[h];
    blk = Tab<TS>::W(S) + (size_t)bid * 2 * N * Np;
    win = (int64_t)S.w_win[h] * N;
  } else {
    K = S.m_K[h];
    bid = S.m_id[h];
    blk = Tab<TS>::M(S) + (size_t)bid * 4 * N * Np;
    win = (int64_t)S.m_win[h] * N;
  }
  const int it = gs ? gs[i].iter : 0;
  const TX *x = xbase + (x_vslot ? I.v_off + (int64_t)it * kS : I.x_off);
  const double xs = scale ? scale[I.st_off + it] : 1.0;
  double *xw = sm;                  // [K]
  double *red = sm + K;             // [NW][TR]
  for (int c = threadIdx.x; c < K; c += 64 * NW) {
    const int64_t idx = win + c;
    xw[c] = (idx >= 0 && idx < kS) ? (double)x[idx] * xs : 0.0;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row0 = tile * TR + lane * VR;
  const bool live = row0 < Np;
  const int c0 = (K * wave) / NW, c1 = (K * (wave + 1)) / NW;
  TO acc[VR];
#pragma unroll
  for (int r = 0; r < VR; ++r) acc[r] = (TO)0;
  const V *colv = reinterpret_cast<const V *>(blk + row0);
  const size_t stride = (size_t)Np / VR;
  constexpr int U = sizeof(V) > 16 ? 4 : 8;   // columns in flight per lane
  int c = c0;
  for (; c + U <= c1; c += U) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = live ? colv[(size_t)(c + u) * stride] : V{};
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const TO xv = (TO)xw[c + u];
      const TS *pv = reinterpret_cast<const TS *>(&v[u]);
#pragma unroll
      for (int r = 0; r < VR; ++r) acc[r] += (TO)pv[r] * xv;
    }
  }
  for (; c < c1; ++c) {
    const V v = live ? colv[(size_t)c * stride] : V{};
    const TO xv = (TO)xw[c];
    const TS *pv = reinterpret_cast<const TS *>(&v);
#pragma unroll
    for (int r = 0; r < VR; ++r) acc[r] += (TO)pv[r] * xv;
  }
#pragma unroll
  for (int r = 0; r < VR; ++r) red[wave * TR + lane * VR + r] = (double)acc[r];
  __syncthreads();
  double out_d = 0.0;
  for (int rr = threadIdx.x; rr < TR; rr += 64 * NW) {
    const int row = tile * TR + rr;
    if (row >= N) continue;
    TO v = (TO)0;
#pragma unroll
    for (int w = 0; w < NW; ++w) v += (TO)red[w * TR + rr];
    double vd = (double)(v * (TO)Tab<TS>::rs(S, op, bid, row));
    if (op == 0) vd += (double)x[(int64_t)h * N + row] * xs;
    const TY out = (TY)vd;
    ybase[I.x_off + (int64_t)h * N + row] = out;
    out_d += (double)out;
  }
  if (hsum) {
    __shared__ double lds4b[NW];
    double sv = wave_sum(out_d);
    if (lane == 0) lds4b[wave] = sv;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < NW; ++w) t += lds4b[w];
      // the tile's sum goes to its first 16-row slot, its other slots are zeroed
      const int slots = (N + 15) >> 4;
      const int q0 = tile * (TR / 16);
      const int q1 = (tile + 1) * (TR / 16) < slots ? (tile + 1) * (TR / 16) : slots;
      hsum[I.hs_off + (int64_t)q0 * S.nh + h] = t;
      for (int q = q0 + 1; q < q1; ++q) hsum[I.hs_off + (int64_t)q * S.nh + h] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// Shared-block GEMM on the matrix cores (Sec. 3.1 Schur matvec, Sec. 3.2
// block-Jacobi, for grids where strips share their operator): one stored
// N x K block (column-major, Np rows) applied to up to kGemmVecs windows at
// once, Y = Blk X (+ the identity for S), with 16x16x4 MFMAs on two 16-window
// column tiles.
// MFMA lane layouts (gfx950): A: lane l holds A[l % 16][l / 16];
// B: lane l holds B[l / 16][l % 16]; D (4 values per lane):
// FP64: D[l / 16 + 4 j][l % 16];  FP32: D[4 (l / 16) + j][l % 16].
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

template <typename TO> struct Mfma;
template <> struct Mfma<double> {
  using Acc = mf_d4;
  __device__ static Acc mac(double a, double b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int j) { return (lane >> 4) + 4 * j; }
};
template <> struct Mfma<float> {
  using Acc = mf_f4;
  __device__ static Acc mac(float a, float b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lane, int j) { return 4 * (lane >> 4) + j; }
};

// Per-window state shared by both GEMM schedules: resolved offsets, whether
// the instance is still iterating, and the basis scale (applied to the
// product in the epilogue, so the operand loads never wait for it).
struct WinInfo {
  int64_t xoff, win, y, xh;
  int64_t sidx;   // entry of the scale vector applied to the output (-1: none)
  int live, hs, hn;
};

template <int VT>
__device__ inline void load_windows(const GWork &wk, const GVec *__restrict__ gvec, int x_vslot,
                                    const double *__restrict__ scale, const GState *__restrict__ gs,
                                    WinInfo *wi) {
  if (threadIdx.x < VT) {
    const int v = threadIdx.x;
    WinInfo w{};
    w.sidx = -1;   // no scale for the unused slots past vcount
    if (v < wk.vcount) {
      const GVec e = gvec[wk.vstart + v];
      int it = 0;
      w.live = 1;
      if (gs) {
        const GState g = gs[e.inst];
        w.live = g.active;
        it = g.iter;
      }
      w.xoff = x_vslot ? e.xv + (int64_t)it * wk.kS : e.x0;
      w.win = e.win;
      w.y = e.y;
      w.xh = e.xh;
      w.hs = e.hs;
      w.hn = e.hn;
      w.sidx = scale ? (int64_t)e.st_off + it : -1;
    }
    wi[v] = w;
  }
}

// Two consecutive vector entries x[i0], x[i0 + 1] (each only if wanted, else
// 0) with one 2-wide load when both are wanted and the pair is aligned to its
// width; else two scalar loads.
template <typename TX> struct Vec2;
template <> struct Vec2<double> { using T = double2; };
template <> struct Vec2<float> { using T = float2; };
template <typename TX, typename TO>
__device__ inline void load_pair(const TX *__restrict__ x, int64_t i0, bool in0, bool in1, TO &v0, TO &v1) {
  using V2 = typename Vec2<TX>::T;
  if (in0 && in1 && ((uintptr_t)(x + i0) & (sizeof(V2) - 1)) == 0) {
    const V2 p = *reinterpret_cast<const V2 *>(x + i0);
    v0 = (TO)p.x;
    v1 = (TO)p.y;
  } else {
    v0 = in0 ? (TO)x[i0] : (TO)0;
    v1 = in1 ? (TO)x[i0 + 1] : (TO)0;
  }
}

// Split-K schedule (few items): grid (item, 16-row tile), KP waves split K;
// U K-steps of operand loads in flight per wave; partial tiles summed in LDS
// in a fixed order.  K-steps go in pairs: in steps 2p and 2p + 1, lane group
// q (lanes 16q .. 16q + 15) takes k = 8p + 2q and 8p + 2q + 1, so each lane
// reads its two window values of a pair with one 2-wide load (the windows are
// contiguous in k; the block rows are read per k as before).  TWO: items may
// hold more than 16 windows (a second 16-window operand); without it the
// registers of that operand are free for a deeper U, which on short launches
// puts a wave's whole K range in flight at once (one wait on memory).
template <typename TS, typename TO, typename TX, typename TY, int KP, int U = (KP >= 16 ? 6 : 8), bool TWO = true>
__global__ __launch_bounds__(64 * KP) void k_half_gemm(
    const GWork *__restrict__ work, const GVec *__restrict__ gvec, const TX *__restrict__ xbase, int x_vslot,
    const double *__restrict__ scale, TY *__restrict__ ybase, double *__restrict__ hsum,
    const GState *__restrict__ gs) {
  constexpr int VT = kGemmVecs;
  __shared__ double red[KP * 16 * VT];
  __shared__ WinInfo wi[VT];
  const GWork wk = work[blockIdx.x];
  const int N = wk.N, Np = wk.Np, K = wk.K;
  const int64_t kS = wk.kS;
  const int rt = blockIdx.y;
  if (rt * 16 >= Np) return;
  const TS *blk = Tab<TS>::blk(wk);
  const int kp = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int arow = rt * 16 + (lane & 15);
  const bool alive = arow < Np;
  const int kq = lane >> 4;
  static_assert(U % 2 == 0, "K-steps go in pairs");
  const int npairs = (((K + 3) >> 2) + 1) >> 1;
  const int s0 = 2 * ((npairs * kp) / KP), s1 = 2 * ((npairs * (kp + 1)) / KP);
  auto kof = [&](int t) { return 8 * (t >> 1) + 2 * kq + (t & 1); };
  // The first block values do not depend on the windows: in flight while
  // the window table is read.
  TO a[U];
  auto load_a = [&](int st) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = kof(st + u);
      a[u] = (alive && st + u < s1 && k < K) ? (TO)blk[(size_t)k * Np + arow] : (TO)0;
    }
  };
  load_a(s0);
  load_windows<VT>(wk, gvec, x_vslot, scale, gs, wi);
  __syncthreads();
  int anylive = 0;
  for (int v = 0; v < wk.vcount; ++v) anylive |= wi[v].live;
  if (!anylive) return;
  const bool two = TWO && wk.vcount > 16;   // second 16-window operand in use
  // the scale and identity values of this thread's first output slot are
  // in flight during the K loop instead of after it
  double e_sc = 1.0;
  TO e_id = (TO)0;
  if (threadIdx.x < 16 * VT) {
    const int lr = threadIdx.x / VT, v = threadIdx.x - lr * VT, row = rt * 16 + lr;
    if (v < wk.vcount && wi[v].live && row < N) {
      if (wi[v].sidx >= 0) e_sc = scale[wi[v].sidx];
      if (wk.ident) e_id = (TO)xbase[wi[v].xoff + wi[v].xh + row];
    }
  }
  const int va = lane & 15, vb = 16 + (lane & 15);
  const bool la = va < wk.vcount && wi[va].live, lb = vb < wk.vcount && wi[vb].live;
  const int64_t xa = wi[va].xoff, wa = wi[va].win, xb = wi[vb].xoff, wb = wi[vb].win;
  using Acc = typename Mfma<TO>::Acc;
  Acc acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  for (int st = s0; st < s1; st += U) {
    if (st != s0) load_a(st);
    TO b0[U], b1[TWO ? U : 1];
#pragma unroll
    for (int u = 0; u < U; u += 2) {
      const int k = kof(st + u);   // this lane's k in step st + u; k + 1 in the next
      const bool kin0 = st + u < s1 && k < K, kin1 = st + u < s1 && k + 1 < K;
      const int64_t ga = wa + k, gb = wb + k;
      load_pair(xbase, xa + ga, la && kin0 && ga >= 0 && ga < kS, la && kin1 && ga + 1 >= 0 && ga + 1 < kS, b0[u],
                b0[u + 1]);
      if constexpr (TWO)
        load_pair(xbase, xb + gb, two && lb && kin0 && gb >= 0 && gb < kS,
                  two && lb && kin1 && gb + 1 >= 0 && gb + 1 < kS, b1[u], b1[u + 1]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc0 = Mfma<TO>::mac(a[u], b0[u], acc0);
    if constexpr (TWO) {
      if (two) {
#pragma unroll
        for (int u = 0; u < U; ++u) acc1 = Mfma<TO>::mac(a[u], b1[u], acc1);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int lr = Mfma<TO>::row(lane, j);
    red[(kp * 16 + lr) * VT + va] = (double)acc0[j];
    red[(kp * 16 + lr) * VT + vb] = (double)acc1[j];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 16 * VT; idx += 64 * KP) {
    const int lr = idx / VT, v = idx - lr * VT;
    const int row = rt * 16 + lr;
    double outv = 0.0;
    if (v < wk.vcount && wi[v].live && row < N) {
      TO t = (TO)red[idx];
#pragma unroll
      for (int q = 1; q < KP; ++q) t += (TO)red[q * 16 * VT + idx];
      t *= (TO)Tab<TS>::rs(wk, row);
      const bool first = idx == (int)threadIdx.x;
      if (wk.ident) t += first ? e_id : (TO)xbase[wi[v].xoff + wi[v].xh + row];
      const double sc = first ? e_sc : (wi[v].sidx >= 0 ? scale[wi[v].sidx] : 1.0);
      const TY out = (TY)((double)t * sc);
      ybase[wi[v].y + row] = out;
      outv = (double)out;
    }
    red[idx] = outv;   // this thread's own slot of the first partial
  }
  if (hsum) {
    __syncthreads();
    if (threadIdx.x < VT) {
      const int v = threadIdx.x;
      if (v < wk.vcount && wi[v].live && rt * 16 < N) {
        double t = 0.0;
        for (int lr = 0; lr < 16; ++lr) t += red[lr * VT + v];
        hsum[wi[v].hs + (int64_t)rt * wi[v].hn] = t;
      }
    }
  }
}

// Throughput schedule (many items): one workgroup per (item, row tile of
// 16 RW rows), items of up to 16 CT windows (CT = 2, or 1 for items of at
// most 16 windows), RW x KW waves: wave (r, p) takes rows 16 r .. 16 r + 15
// of the tile and every KW-th chunk of K starting at chunk p.  The windows
// are staged through double-buffered LDS, KW chunks of KC K-values at a
// time, with coalesced loads while the next chunks' operands are in flight;
// every wave of the tile reads them from there.  With KW > 1 the K parts
// are summed through LDS in a fixed order before the epilogue.  RW = 4,
// KW = 1 is the 64-row tile whose (item, tile) pairs may come in an
// XCD-aware order (`units`): workgroup L runs on XCD L mod 8, and every
// tile that reads one stored block is placed on the same XCD, so the block
// and the windows are fetched into one L2 instead of eight.
template <typename TO> constexpr bool kNarrowMfma = std::is_same<TO, double>::value;
template <typename TS, typename TO, typename TX, typename TY, int CT, int KC, int RW = 4, int KW = 1>
__global__ __launch_bounds__(64 * RW * KW) void k_half_gemm_t(
    const GWork *__restrict__ work, const int2 *__restrict__ units, const GVec *__restrict__ gvec,
    const TX *__restrict__ xbase, int x_vslot, const double *__restrict__ scale, TY *__restrict__ ybase,
    double *__restrict__ hsum, const GState *__restrict__ gs) {
  // Staging as in k_colgemm_t: the TPC threads of a window read its KW KC
  // values interleaved (thread j takes k = j + TPC p), and the row pitch puts
  // the lanes that the LDS serves together (16 for 8-byte, 32 for 4-byte
  // values) in distinct bank slots for the stores and the MFMA operand reads.
  constexpr int NT = 64 * RW * KW, VT = 16 * CT, PITCH = VT + (sizeof(TO) == 8 ? CT : 2 * CT);
  constexpr int KS = KW * KC;             // K-values staged per step
  constexpr int PV = KS * VT / NT;        // staged values per thread per step
  constexpr int TPC = KS / PV;            // threads per window
  static_assert(PV >= 1 && TPC * PV == KS && NT % VT == 0, "staging shape");
  constexpr int BS = KS * PITCH;          // one staging buffer
  constexpr int RED = (KW > 1 ? (KW - 1) * RW * 64 * CT * 4 : 1);
  static_assert(KW == 1 || RED * sizeof(TO) <= 2 * BS * sizeof(TO), "reduction fits the staging buffers");
  __shared__ TO Bs[2 * BS];
  __shared__ WinInfo wi[VT];
  int item = blockIdx.x, rg = blockIdx.y;
  if (units) {   // XCD-ordered (item, row tile) list; x < 0 pads a bucket
    const int2 u = units[blockIdx.x];
    if (u.x < 0) return;
    item = u.x; rg = u.y;
  }
  const GWork wk = work[item];
  const int N = wk.N, Np = wk.Np, K = wk.K;
  const int64_t kS = wk.kS;
  constexpr int TR = 16 * RW;             // rows per tile
  if (rg * TR >= Np) return;
  const TS *__restrict__ blk = Tab<TS>::blk(wk);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = wave % RW, kp = wave / RW;
  const int arow = rg * TR + wr * 16 + (lane & 15);
  const bool alive = arow < Np, wlive = rg * TR + wr * 16 < N;
  const int kq = lane >> 4, cl = lane & 15;
  TO a[KC / 4], an[KC / 4];
  auto load_a = [&](int st, TO *dst) {   // this wave's chunk of step st
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int k = st * KS + kp * KC + 4 * s + kq;
      dst[s] = (alive && k < K) ? (TO)blk[(size_t)k * Np + arow] : (TO)0;
    }
  };
  load_a(0, a);   // the first block chunk does not depend on the windows
  load_windows<VT>(wk, gvec, x_vslot, scale, gs, wi);
  __syncthreads();
  // 16-window column tiles with a live window; the others take no MFMA
  unsigned tmask = 0;
  for (int v = 0; v < wk.vcount; ++v)
    if (wi[v].live) tmask |= 1u << (v >> 4);
  tmask = __builtin_amdgcn_readfirstlane(tmask);
  if (!tmask) return;
  // FP64 items of at most 4 windows: one 4-block 4 x 4 x 4 MFMA per K-step
  // (blocks = the four 4-row groups of the wave's 16 rows, columns = the
  // windows) instead of a 16-window 16 x 16 x 4 tile of which 12 columns
  // would be zero
  const bool narrow = wk.vcount <= 4;
  const int scol = threadIdx.x / TPC, sj = threadIdx.x % TPC;
  const bool slive = scol < wk.vcount && wi[scol].live;
  const int64_t sx = wi[scol].xoff, sw = wi[scol].win;
  TO pre[PV];
  auto load_b = [&](int st) {   // staging step st: K-values st KS .. st KS + KS
#pragma unroll
    for (int p = 0; p < PV; ++p) {
      const int k = st * KS + sj + TPC * p;
      const int64_t g = sw + k;
      pre[p] = (slive && k < K && g >= 0 && g < kS) ? (TO)xbase[sx + g] : (TO)0;
    }
  };
  auto store_b = [&](int buf) {
#pragma unroll
    for (int p = 0; p < PV; ++p) Bs[buf * BS + (sj + TPC * p) * PITCH + scol] = pre[p];
  };
  using Acc = typename Mfma<TO>::Acc;
  Acc acc[CT];
#pragma unroll
  for (int t = 0; t < CT; ++t) acc[t] = Acc{0, 0, 0, 0};
  const int nsteps = (K + KS - 1) / KS;
  load_b(0);
  store_b(0);
  __syncthreads();
  for (int st = 0; st < nsteps; ++st) {
    const int buf = st & 1;
    const bool more = st + 1 < nsteps;
    if (more) {
      load_b(st + 1);
      load_a(st + 1, an);
    }
    const TO *__restrict__ B = Bs + buf * BS + kp * KC * PITCH;
    if constexpr (kNarrowMfma<TO>) {
      if (wlive && narrow) {
#pragma unroll
        for (int s = 0; s < KC / 4; ++s)
          acc[0][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[s], B[(4 * s + kq) * PITCH + (lane & 3)], acc[0][0], 0, 0, 0);
      }
    }
    if (wlive && !(kNarrowMfma<TO> && narrow)) {   // a wave whose 16 rows all lie past the block stages only
#pragma unroll
      for (int t = 0; t < CT; ++t)
        if ((tmask >> t) & 1u) {
#pragma unroll
          for (int s = 0; s < KC / 4; ++s)
            acc[t] = Mfma<TO>::mac(a[s], B[(4 * s + kq) * PITCH + t * 16 + cl], acc[t]);
        }
    }
    if (more) {
      store_b(buf ^ 1);
#pragma unroll
      for (int s = 0; s < KC / 4; ++s) a[s] = an[s];
    }
    __syncthreads();
  }
  if constexpr (KW > 1) {   // sum the K parts: part p > 0 through LDS, in order p = 1 .. KW - 1
    TO *R = Bs;
    if (kp > 0) {
#pragma unroll
      for (int t = 0; t < CT; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) R[((((kp - 1) * RW + wr) * CT + t) * 4 + j) * 64 + lane] = acc[t][j];
    }
    __syncthreads();
    if (kp > 0) return;
#pragma unroll
    for (int q = 1; q < KW; ++q)
#pragma unroll
      for (int t = 0; t < CT; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[t][j] += R[((((q - 1) * RW + wr) * CT + t) * 4 + j) * 64 + lane];
  }
  const int slot = rg * RW + wr;
  if constexpr (kNarrowMfma<TO>) {
    if (narrow) {
      // lane m holds row 4 ((m >> 2) & 3) + (m >> 4) of the wave's 16 for
      // window m & 3; window c's scale is scv[0] of lane c
      const int c = lane & 3;
      const int row = rg * TR + wr * 16 + 4 * ((lane >> 2) & 3) + (lane >> 4);
      const bool ok = c < wk.vcount && wi[c].live;
      const double sc = (ok && wi[c].sidx >= 0) ? scale[wi[c].sidx] : 1.0;
      double part = 0.0;
      if (ok && row < N) {
        TO val = acc[0][0] * (TO)Tab<TS>::rs(wk, row);
        if (wk.ident) val += (TO)xbase[wi[c].xoff + wi[c].xh + row];
        const TY out = (TY)((double)val * sc);
        ybase[wi[c].y + row] = out;
        part = (double)out;
      }
      // sum the 16 rows of this wave's slot: the lanes with the same c
      part += __shfl_xor(part, 4, 64);
      part += __shfl_xor(part, 8, 64);
      part += __shfl_xor(part, 16, 64);
      part += __shfl_xor(part, 32, 64);
      if (hsum && ok && lane < 4 && slot * 16 < N) hsum[wi[c].hs + (int64_t)slot * wi[c].hn] = part;
      return;
    }
  }
  // epilogue: lane holds rows Mfma::row(lane, j) of windows t * 16 + cl
#pragma unroll
  for (int t = 0; t < CT; ++t) {
    const int v = t * 16 + cl;
    const bool ok = v < wk.vcount && wi[v].live;
    double part = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = rg * TR + wr * 16 + Mfma<TO>::row(lane, j);
      if (ok && row < N) {
        TO val = acc[t][j] * (TO)Tab<TS>::rs(wk, row);
        if (wk.ident) val += (TO)xbase[wi[v].xoff + wi[v].xh + row];
        const TY out = (TY)((double)val * (wi[v].sidx >= 0 ? scale[wi[v].sidx] : 1.0));
        ybase[wi[v].y + row] = out;
        part += (double)out;
      }
    }
    // sum the 16 rows of this wave's slot: lanes cl, cl + 16, cl + 32, cl + 48
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    if (hsum && ok && kq == 0 && slot * 16 < N) hsum[wi[v].hs + (int64_t)slot * wi[v].hn] = part;
  }
}

// Coarse solve of the deflation (Sec. 3.3): t_c = sum of the two halves of
// interface c (= Z^T y), optionally t = tsub - t; c = G t with G the
// precomputed C^dagger (I - u_C u_C^T) (C^-1 for k > 0).  Grid (instance,
// 16-row tile of c): every workgroup forms all of t in LDS and multiplies its
// 16 rows of G, so one apply reads G once, spread over many CUs.  Thread
// (row, g) sums columns g, g + 16, ... of its row (16 rows of a column are
// one 128-byte segment); the 16 partial sums of a row are added in a fixed
// order.
__global__ __launch_bounds__(kBlock) void k_coarse(const SysDev *__restrict__ sys,
                                                   const InstDev *__restrict__ ins,
                                                   const double *__restrict__ hsum,
                                                   const double *__restrict__ tsub,
                                                   double *__restrict__ tout,
                                                   double *__restrict__ cout,
                                                   const GState *__restrict__ gs) {
  extern __shared__ double t[];   // d
  __shared__ double red[16 * 17];
  const int i = blockIdx.x;
  if (gs && !gs[i].active) return;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int d = S.d;
  const int r0 = blockIdx.y * 16;
  if (r0 >= d) return;
  const int sl = hs_slots(S);
  for (int c = threadIdx.x; c < d; c += kBlock) {
    double v = 0.0;
    if (S.zm == 1) {
      for (int q = 0; q < sl; ++q) {
        const double2 p = *reinterpret_cast<const double2 *>(hsum + I.hs_off + (int64_t)q * S.nh + 2 * c);
        v += p.x + p.y;
      }
    } else {
      const int a = c / S.zm, e = c - a * S.zm;
      v = hsum[I.hs_off + (int64_t)(2 * a) * sl + e] + hsum[I.hs_off + (int64_t)(2 * a + 1) * sl + e];
    }
    if (tsub) v = tsub[I.c_off + c] - v;
    t[c] = v;
    if (tout && c >= r0 && c < r0 + 16) tout[I.c_off + c] = v;
  }
  __syncthreads();
  const int row = threadIdx.x & 15, g = threadIdx.x >> 4;
  const double *__restrict__ col = S.Gc + r0 + (r0 + row < d ? row : 0);
  double a0 = 0.0, a1 = 0.0;
  int c = g;
#pragma unroll 4
  for (; c + 16 < d; c += 32) {
    a0 += col[(size_t)c * d] * t[c];
    a1 += col[(size_t)(c + 16) * d] * t[c + 16];
  }
  if (c < d) a0 += col[(size_t)c * d] * t[c];
  red[g * 17 + row] = a0 + a1;
  __syncthreads();
  if (threadIdx.x < 16 && r0 + (int)threadIdx.x < d) {
    double v = 0.0;
    for (int q = 0; q < 16; ++q) v += red[q * 17 + threadIdx.x];
    cout[I.c_off + r0 + threadIdx.x] = v;
  }
}

// Short Krylov bases (j < kBasisRegs) are read into registers before
// anything else a pass waits on: the two elements of a thread (e0 + tid and
// e0 + tid + kBlock) of every basis vector t <= j, in one burst of loads that
// overlaps the reduction of the previous pass's partials.  The dots of the
// pass then come from the registers (one block reduction per vector) instead
// of a second sweep over the basis.  Kernels take it with RB = true, for
// handles whose vector launches are few workgroups (latency bound): the 32
// extra registers halve the occupancy, which costs more than it saves where
// thousands of workgroups stream the basis.
constexpr int kBasisRegs = 16;
template <typename TV>
__device__ inline void prefetch_basis(const TV *__restrict__ Vi, int64_t kS, int64_t ea, bool ina, bool inb, int j,
                                      double (&va)[kBasisRegs], double (&vb)[kBasisRegs]) {
#pragma unroll
  for (int t = 0; t < kBasisRegs; ++t) {
    va[t] = (t <= j && ina) ? (double)Vi[(int64_t)t * kS + ea] : 0.0;
    vb[t] = (t <= j && inb) ? (double)Vi[(int64_t)t * kS + ea + kBlock] : 0.0;
  }
}

// part[t nchunk + ch] = sum over the workgroup of va[t] a0 + vb[t] a1, t <= j
// (wave sums, then the four waves in a fixed order).
__device__ inline void block_dots(const double (&va)[kBasisRegs], const double (&vb)[kBasisRegs], double a0,
                                  double a1, int j, double *red, double *__restrict__ part, int nchunk, int ch) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < kBasisRegs; ++t) {
    if (t <= j) {   // uniform over the workgroup
      const double d = wave_sum(va[t] * a0 + vb[t] * a1);
      if (lane == 0) red[wave * kBasisRegs + t] = d;
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t <= j)
    part[(int64_t)t * nchunk + ch] = (red[t] + red[kBasisRegs + t]) + (red[2 * kBasisRegs + t] + red[3 * kBasisRegs + t]);
}

// Partial dots V_t . w over one chunk, t = 0 .. j, written to
// part[t * nchunk + ch].  The chunk of w is in LDS (ws, zero past k_S); wave
// q takes t = q, q + 4, ... two at a time over all kChunk elements (8
// coalesced loads per lane per t), so a reduction serves two dots and no
// cross-wave step is needed.
template <typename TV>
__device__ inline void chunk_dots(const TV *__restrict__ V, int64_t kS, int64_t e0, int j,
                                  const double *__restrict__ ws, double *__restrict__ part, int nchunk, int ch) {
  constexpr int Q = kChunk / 64;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double wl[Q];
  bool in[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    wl[q] = ws[lane + 64 * q];
    in[q] = e0 + lane + 64 * q < kS;
  }
  for (int t = wave; t <= j; t += 8) {
    const int t2 = t + 4;
    const bool two = t2 <= j;
    const TV *Va = V + (int64_t)t * kS + e0 + lane;
    const TV *Vb = V + (int64_t)(two ? t2 : t) * kS + e0 + lane;
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (in[q]) {
        a += (double)Va[64 * q] * wl[q];
        b += (double)Vb[64 * q] * wl[q];
      }
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
      part[(int64_t)t * nchunk + ch] = a;
      if (two) part[(int64_t)t2 * nchunk + ch] = b;
    }
  }
}

// Arnoldi step, part 1: w = y - (S Z) c with c = G Z^T y (the deflation P,
// Sec. 3.3; useP = 0 skips it), stored in Krylov slot iter + 1; partial dots
// V_t . w for t <= iter.  The coarse solve is fused: every workgroup forms
// t = Z^T y from the per-tile half sums and computes only the coarse values
// its chunk needs, against all d values of t.  With one coarse column per
// interface, the loads that do not depend on t (the chunk's y values, its
// S Z rows, the first 8 G rows it needs, from the row-major copy of G) go
// out before t is formed, so the kernel waits on memory once before its
// dots instead of three times.  With cpre (large d, where the workgroups' G
// rows would add up to several reads of G) it takes the coarse values from
// c = G Z^T y formed beforehand by k_coarse.
template <typename TV, typename TY, bool RB = false>
__global__ __launch_bounds__(kBlock) void k_pcorr_dot(
    const SysDev *__restrict__ sys, const InstDev *__restrict__ ins, const int2 *__restrict__ work,
    const TY *__restrict__ ybase, const double *__restrict__ hsum, int useP, TV *__restrict__ V,
    double *__restrict__ part, const GState *__restrict__ gs, const double *__restrict__ cpre) {
  constexpr int Q = kChunk / kBlock;
  extern __shared__ double t_s[];   // d
  __shared__ double c_s[kChunk / 2 + 8];
  __shared__ double ws[kChunk];
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  if (!gs[i].active) return;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int N = S.N;
  const int64_t kS = S.kS;
  const int j = gs[i].iter;
  const int64_t e0 = (int64_t)ch * kChunk;
  static_assert(Q == 2, "two elements per thread, as the register basis holds them");
  const bool regs = RB && j < kBasisRegs;
  double va[kBasisRegs], vb[kBasisRegs];   // the basis of a short space, loaded with everything else
  if (regs) prefetch_basis(V + I.v_off, kS, e0 + threadIdx.x, e0 + threadIdx.x < kS, e0 + threadIdx.x + kBlock < kS, j, va, vb);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool pre = useP && S.zm == 1 && !cpre;
  int c0 = 0, ncol = 0;
  if (useP) {   // the coarse values this chunk needs: interfaces ilo .. ihi
    const int nif = S.mx - 1;
    const int64_t elast = (e0 + kChunk < kS ? e0 + kChunk : kS) - 1;
    const int hlo = (int)(e0 / N), hhi = (int)(elast / N);
    const int ilo = hlo / 2 - 1 < 0 ? 0 : hlo / 2 - 1;
    const int ihi = hhi / 2 + 1 > nif - 1 ? nif - 1 : hhi / 2 + 1;
    c0 = ilo * S.zm;
    ncol = (ihi - ilo + 1) * S.zm;
  }
  double yv[Q], szv[Q][2], gv[2][4];
  int szc[Q][2];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t e = e0 + threadIdx.x + q * kBlock;
    const bool in = e < kS;
    yv[q] = in ? (double)ybase[I.x_off + e] : 0.0;
    szc[q][0] = szc[q][1] = -1;
    szv[q][0] = szv[q][1] = 0.0;
    if (pre && in) {
      const int h = (int)e / N, row = (int)e - h * N;
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        szc[q][p] = S.sz_col[(size_t)h * 2 + p];
        szv[q][p] = S.SZh[((size_t)h * 2 + p) * N + row];
      }
    }
  }
  if (pre) {
#pragma unroll
    for (int rr = 0; rr < 2; ++rr)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int r = wave + 4 * rr, l = lane + 64 * k;
        gv[rr][k] = r < ncol && l < S.d ? S.GcR[(size_t)(c0 + r) * S.d + l] : 0.0;
      }
  }
  if (useP) {
    const int d = S.d, zm = S.zm;
    const int sl = hs_slots(S);
    if (cpre) {   // c = G Z^T y already formed (large d: G read once)
      for (int r = threadIdx.x; r < ncol; r += kBlock) c_s[r] = cpre[I.c_off + c0 + r];
    } else {
      for (int c = threadIdx.x; c < d; c += kBlock) {
        double v = 0.0;
        if (zm == 1) {
          for (int q = 0; q < sl; ++q) {
            const double2 p = *reinterpret_cast<const double2 *>(hsum + I.hs_off + (int64_t)q * S.nh + 2 * c);
            v += p.x + p.y;
          }
        } else {
          const int a = c / zm, e = c - a * zm;
          v = hsum[I.hs_off + (int64_t)(2 * a) * sl + e] + hsum[I.hs_off + (int64_t)(2 * a + 1) * sl + e];
        }
        t_s[c] = v;
      }
      __syncthreads();
      if (pre) {
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
          const int r = wave + 4 * rr;
          if (r >= ncol) continue;
          double a = 0.0;
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (lane + 64 * k < d) a += gv[rr][k] * t_s[lane + 64 * k];
          for (int l = lane + 256; l < d; l += 64) a += S.GcR[(size_t)(c0 + r) * d + l] * t_s[l];
          a = wave_sum(a);
          if (lane == 0) c_s[r] = a;
        }
        for (int r = wave + 8; r < ncol; r += 4) {
          double a = 0.0;
          for (int l = lane; l < d; l += 64) a += S.GcR[(size_t)(c0 + r) * d + l] * t_s[l];
          a = wave_sum(a);
          if (lane == 0) c_s[r] = a;
        }
      } else {
        for (int r = wave; r < ncol; r += 4) {
          double a = 0.0;
          for (int l = lane; l < d; l += 64) a += S.Gc[(size_t)l * d + c0 + r] * t_s[l];
          a = wave_sum(a);
          if (lane == 0) c_s[r] = a;
        }
      }
    }
    __syncthreads();
  }
  double wq[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t e = e0 + threadIdx.x + q * kBlock;
    double w = 0.0;
    if (e < kS) {
      w = yv[q];
      if (pre) {
        double a = 0.0;
#pragma unroll
        for (int p = 0; p < 2; ++p)
          if (szc[q][p] >= 0) a += szv[q][p] * c_s[szc[q][p] - c0];
        w -= a;
      } else if (useP) {
        const int h = (int)e / N, row = (int)e - h * N;
        w -= sz_c(S, h, row, c_s, c0);
      }
      const TV wt = (TV)w;
      V[I.v_off + (int64_t)(j + 1) * kS + e] = wt;
      w = (double)wt;
    }
    wq[q] = w;
    if (!regs) ws[threadIdx.x + q * kBlock] = w;
  }
  if (regs) {   // ws is free: the scratch of the block sums
    block_dots(va, vb, wq[0], wq[1], j, ws, part + I.part_off, I.nchunk_x, ch);
    return;
  }
  __syncthreads();
  chunk_dots(V + I.v_off, kS, e0, j, ws, part + I.part_off, I.nchunk_x, ch);
}

// Reduce the chunk partials of pass `part` into coef[t] = s_t^2 sum(...)
// (the coefficient of V_t in w -= sum_t h_t v_t, v_t = s_t V_t).
__device__ inline void reduce_coef(const InstDev &I, const double *__restrict__ part,
                                   const double *__restrict__ scale, int j, double *coef) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int t = wave; t <= j; t += 8) {   // two coefficients per reduction pass
    const int t2 = t + 4;
    const bool two = t2 <= j;
    const double *p = part + I.part_off + (int64_t)t * I.nchunk_x;
    const double *p2 = part + I.part_off + (int64_t)(two ? t2 : t) * I.nchunk_x;
    double a = 0.0, b = 0.0;
    for (int c = lane; c < I.nchunk_x; c += 64) {
      a += p[c];
      b += p2[c];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
      const double s = scale[I.st_off + t];
      coef[t] = s * s * a;
      if (two) {
        const double s2 = scale[I.st_off + t2];
        coef[t2] = s2 * s2 * b;
      }
    }
  }
  __syncthreads();
}

// The second pass's coefficients as reduce_coef forms them from part2, and
// with them, from the same loads, what the Givens step of the column needs:
// h[t] = s_t (sum part1_t + sum part2_t), h2sq[t] = (s_t sum part2_t)^2 and
// the first pass's squared norm sum(partn) (returned in thread 0), summed in
// the order givens_step sums them.  Every workgroup of the pass forms them
// while its basis loads are in flight, so the one that arrives last starts
// its Givens step without another round of loads.
__device__ inline double reduce_coef_givens(const InstDev &I, const double *__restrict__ part1,
                                            const double *__restrict__ part2, const double *__restrict__ partn,
                                            const double *__restrict__ scale, int j, double *coef, double *h,
                                            double *h2sq, double *lds4) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double nn = 0.0;
  for (int k = threadIdx.x; k < I.nchunk_x; k += kBlock) nn += partn[I.part_off + k];
  for (int t = wave; t <= j; t += 8) {   // two columns per reduction pass
    const int t2 = t + 4;
    const bool two = t2 <= j;
    const double *p1 = part1 + I.part_off + (int64_t)t * I.nchunk_x;
    const double *p2 = part2 + I.part_off + (int64_t)t * I.nchunk_x;
    const double *q1 = part1 + I.part_off + (int64_t)(two ? t2 : t) * I.nchunk_x;
    const double *q2 = part2 + I.part_off + (int64_t)(two ? t2 : t) * I.nchunk_x;
    double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
    for (int k = lane; k < I.nchunk_x; k += 64) {
      a += p1[k];
      b += p2[k];
      c += q1[k];
      d += q2[k];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    d = wave_sum(d);
    if (lane == 0) {
      const double st = scale[I.st_off + t];
      coef[t] = st * st * b;
      h[t] = st * (a + b);
      h2sq[t] = (st * b) * (st * b);
      if (two) {
        const double st2 = scale[I.st_off + t2];
        coef[t2] = st2 * st2 * d;
        h[t2] = st2 * (c + d);
        h2sq[t2] = (st2 * d) * (st2 * d);
      }
    }
  }
  return block_sum(nn, lds4);   // its barriers publish coef, h and h2sq
}

// The serial part of the Givens step, in thread 0, once h[0 .. j] (and h2sq
// when pyth), the earlier rotations and nn (thread 0's value) are in place:
// layout of sh as in givens_step.  r0 and ref: the instance's GMRES state,
// carried over unchanged.
__device__ inline void givens_rotate(const InstDev &I, int i, int j, double nn, double *scale, double *__restrict__ R,
                                     double *__restrict__ cs, double *__restrict__ sn, double *__restrict__ g,
                                     GState *gs, int maxit, double tol, double *sh, bool pyth, double r0,
                                     double ref) {
  if (threadIdx.x == 0) {
    double *h = sh;
    const double *cl = sh + maxit + 2, *sl = cl + maxit, *h2sq = sl + maxit;
    if (pyth) {
      for (int t = 0; t <= j; ++t) nn -= h2sq[t];
      nn = nn > 0.0 ? nn : 0.0;
    }
    const double beta = sqrt(nn);
    h[j + 1] = beta;
    double *gI = g + I.st_off;
    for (int t = 0; t < j; ++t) {
      const double a = cl[t] * h[t] + sl[t] * h[t + 1];
      h[t + 1] = -sl[t] * h[t] + cl[t] * h[t + 1];
      h[t] = a;
    }
    const double den = hypot(h[j], h[j + 1]);
    const double c = den != 0.0 ? h[j] / den : 1.0;
    const double s = den != 0.0 ? h[j + 1] / den : 0.0;
    cs[I.st_off + j] = c;
    sn[I.st_off + j] = s;
    h[j] = den;
    gI[j + 1] = -s * gI[j];
    gI[j] = c * gI[j];
    double *Rc = R + I.rr_off + (int64_t)j * maxit;
    for (int t = 0; t <= j; ++t) Rc[t] = h[t];
    const double res = fabs(gI[j + 1]);
    int active = 0, status = 0;
    if (!isfinite(res) || !isfinite(den)) {
      status = 3;
    } else if (res <= tol * ref || beta == 0.0) {
      status = 1;
    } else if (j + 1 >= maxit) {
      status = 2;
    } else {
      active = 1;
      scale[I.st_off + j + 1] = 1.0 / beta;
    }
    // field by field: a whole-struct copy is kept in scratch by the compiler
    for (int m = i; m < i + I.seg_count; ++m) {
      gs[m].iter = j + 1;
      gs[m].active = active;
      gs[m].status = status;
      gs[m].r0 = r0;
      gs[m].res = res;
      gs[m].ref = ref;
    }
  }
}

// One Givens step of instance (segment leader) i at Arnoldi column j: the
// Hessenberg column h_t = s_t (sum part1 + sum part2), h_{j+1} = ||w|| from
// the per-chunk partials (or from the segment sums r1, r2, rn), the earlier
// rotations applied to it, a new rotation, the residual estimate |g_{j+1}|,
// the next basis scale and the GMRES state (written to every instance of the
// segment).  Called by a whole workgroup; sh holds 3 maxit + 2 doubles: h,
// then the earlier rotations, read into LDS while the sums are formed.
__device__ inline void givens_step(const InstDev &I, int i, int j, const double *__restrict__ part1,
                                   const double *__restrict__ part2, const double *__restrict__ partn,
                                   const double *__restrict__ r1, const double *__restrict__ r2,
                                   const double *__restrict__ rn, double *scale, double *__restrict__ R,
                                   double *__restrict__ cs, double *__restrict__ sn, double *__restrict__ g,
                                   GState *gs, int maxit, double tol, double *sh, double *lds4,
                                   bool pyth = false) {
  // pyth: partn holds the partial squared norms of w after the first CGS
  // pass; the second pass removes sum_t h2_t^2 (h2_t = s_t sum(part2_t), the
  // second-pass coefficients of the orthonormal v_t), so |w|^2 after it is
  // the difference (sh then holds 4 maxit + 3 doubles: h2_t^2 after the
  // rotations).  The second pass removes only rounding-level components, so
  // the difference loses nothing.
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double *h = sh, *cl = sh + maxit + 2, *sl = cl + maxit, *h2sq = sl + maxit;
  for (int t = threadIdx.x; t < j; t += kBlock) {
    cl[t] = cs[I.st_off + t];
    sl[t] = sn[I.st_off + t];
  }
  double nn = 0.0;
  if (r1) {   // segment sums reduced by k_seg_reduce
    for (int t = threadIdx.x; t <= j; t += kBlock) h[t] = scale[I.st_off + t] * (r1[I.st_off + t] + r2[I.st_off + t]);
    nn = rn[I.st_off];
  } else {
    for (int t = wave; t <= j; t += 8) {   // two columns per reduction pass
      const int t2 = t + 4;
      const bool two = t2 <= j;
      const double *p1 = part1 + I.part_off + (int64_t)t * I.nchunk_x;
      const double *p2 = part2 + I.part_off + (int64_t)t * I.nchunk_x;
      const double *q1 = part1 + I.part_off + (int64_t)(two ? t2 : t) * I.nchunk_x;
      const double *q2 = part2 + I.part_off + (int64_t)(two ? t2 : t) * I.nchunk_x;
      double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
      for (int k = lane; k < I.nchunk_x; k += 64) {
        a += p1[k];
        b += p2[k];
        c += q1[k];
        d += q2[k];
      }
      a = wave_sum(a);
      b = wave_sum(b);
      c = wave_sum(c);
      d = wave_sum(d);
      if (lane == 0) {
        const double st = scale[I.st_off + t];
        h[t] = st * (a + b);
        if (pyth) h2sq[t] = (st * b) * (st * b);
        if (two) {
          const double st2 = scale[I.st_off + t2];
          h[t2] = st2 * (c + d);
          if (pyth) h2sq[t2] = (st2 * d) * (st2 * d);
        }
      }
    }
    for (int k = threadIdx.x; k < I.nchunk_x; k += kBlock) nn += partn[I.part_off + k];
    nn = block_sum(nn, lds4);
  }
  __syncthreads();
  givens_rotate(I, i, j, nn, scale, R, cs, sn, g, gs, maxit, tol, sh, pyth, gs[i].r0, gs[i].ref);
}


// Classical Gram-Schmidt pass: w -= sum_t coef_t V_t (coef from the partials
// of the previous pass); then either the next pass's partial dots
// (part_out) or the partial squared norm (partn).
template <typename TV, bool RB = false>
__global__ __launch_bounds__(kBlock) void k_axpy_dot(
    const SysDev *__restrict__ sys, const InstDev *__restrict__ ins, const int2 *__restrict__ work,
    TV *__restrict__ V, const double *__restrict__ part_in, double *__restrict__ part_out,
    double *__restrict__ partn, const double *__restrict__ scale, const GState *__restrict__ gs,
    const double *__restrict__ coefr) {
  extern __shared__ double coef[];   // maxit + 1
  __shared__ double ws[kChunk];
  __shared__ double red[4];
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];   // loaded with the state, not after its test
  const GState G = gs[i];
  if (!G.active) return;
  const SysDev &S = sys[I.sys];
  const int64_t kS = S.kS;
  const int j = G.iter;
  static_assert(kChunk == 2 * kBlock, "two elements per thread");
  const int64_t e0 = (int64_t)ch * kChunk;
  const int64_t ea = e0 + threadIdx.x, eb = ea + kBlock;
  const bool ina = ea < kS, inb = eb < kS;
  TV *w = V + I.v_off + (int64_t)(j + 1) * kS;
  double a0 = ina ? (double)w[ea] : 0.0, a1 = inb ? (double)w[eb] : 0.0;
  const bool regs = RB && j < kBasisRegs && part_out && !coefr;
  double va[kBasisRegs], vb[kBasisRegs];
  if (regs) prefetch_basis(V + I.v_off, kS, ea, ina, inb, j, va, vb);
  if (coefr) {   // segment sums reduced by k_seg_reduce
    for (int t = threadIdx.x; t <= j; t += kBlock) {
      const double s = scale[I.st_off + t];
      coef[t] = s * s * coefr[I.st_off + t];
    }
    __syncthreads();
  } else {
    reduce_coef(I, part_in, scale, j, coef);
  }
  if (regs) {
#pragma unroll
    for (int t = 0; t < kBasisRegs; ++t) {
      if (t <= j) {
        const double c = coef[t];
        a0 -= c * va[t];
        a1 -= c * vb[t];
      }
    }
    if (ina) {
      const TV at = (TV)a0;
      w[ea] = at;
      a0 = (double)at;
    }
    if (inb) {
      const TV at = (TV)a1;
      w[eb] = at;
      a1 = (double)at;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (partn) {   // |w|^2 after this pass, for the Pythagorean norm of the next
      const double a = wave_sum(a0 * a0 + a1 * a1);
      if (lane == 0) red[wave] = a;
    }
    block_dots(va, vb, a0, a1, j, ws, part_out + I.part_off, I.nchunk_x, ch);   // syncs before the sums
    if (partn && threadIdx.x == 0) partn[I.part_off + ch] = (red[0] + red[1]) + (red[2] + red[3]);
    return;
  }
  const TV *Vt = V + I.v_off + ea;
#pragma unroll 4
  for (int t = 0; t <= j; ++t, Vt += kS) {
    const double c = coef[t];
    if (ina) a0 -= c * (double)Vt[0];
    if (inb) a1 -= c * (double)Vt[kBlock];
  }
  if (ina) {
    const TV at = (TV)a0;
    w[ea] = at;
    a0 = (double)at;
  }
  if (inb) {
    const TV at = (TV)a1;
    w[eb] = at;
    a1 = (double)at;
  }
  const double wv[2] = {a0, a1};
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (part_out) {
    ws[threadIdx.x] = a0;
    ws[threadIdx.x + kBlock] = a1;
    if (partn) {   // |w|^2 after this pass, for the Pythagorean norm of the next
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < 2; ++q) a += wv[q] * wv[q];
      a = wave_sum(a);
      if (lane == 0) red[wave] = a;
    }
    __syncthreads();
    if (partn && threadIdx.x == 0) partn[I.part_off + ch] = (red[0] + red[1]) + (red[2] + red[3]);
    chunk_dots(V + I.v_off, kS, e0, j, ws, part_out + I.part_off, I.nchunk_x, ch);
  } else {
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < 2; ++q) a += wv[q] * wv[q];
    a = wave_sum(a);
    if (lane == 0) red[wave] = a;
    __syncthreads();
    if (threadIdx.x == 0) partn[I.part_off + ch] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// Classical Gram-Schmidt, second pass, with the Givens step: w -= sum_t
// coef_t V_t (coef from the second-pass partials `part2`),
// then the instance's last workgroup to finish (an arrival counter) takes the
// Givens step (givens_step with the Pythagorean norm: the first pass left
// the partial |w|^2 in partn).  The step needs only partials written by the
// kernels before this one, so no workgroup waits for another's stores; and
// every other workgroup has read the GMRES state before it counts itself, so
// the last one may advance it.  Saves the separate Givens launch per
// iteration.  Instances of one Krylov space over several instances (segments)
// keep the separate launch.
template <typename TV, bool RB = false>
__global__ __launch_bounds__(kBlock) void k_axpy_givens(
    const SysDev *__restrict__ sys, const InstDev *__restrict__ ins, const int2 *__restrict__ work,
    TV *__restrict__ V, const double *__restrict__ part1, const double *__restrict__ part2,
    const double *__restrict__ partn, double *scale, double *__restrict__ R, double *__restrict__ cs,
    double *__restrict__ sn, double *__restrict__ g, GState *gs, int *__restrict__ arrive, int maxit, double tol) {
  extern __shared__ double dyn[];   // coef[maxit + 1], then the Givens scratch (4 maxit + 3)
  __shared__ double lds4[4];
  __shared__ int last_s;
  double *coef = dyn, *sh = dyn + maxit + 1;
  double *hcol = sh, *cl = sh + maxit + 2, *sl = cl + maxit, *h2sq = sl + maxit;
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];
  const GState G = gs[i];
  if (!G.active) return;
  const SysDev &S = sys[I.sys];
  const int64_t kS = S.kS;
  const int j = G.iter;
  const int64_t e0 = (int64_t)ch * kChunk;
  const int64_t ea = e0 + threadIdx.x, eb = ea + kBlock;
  const bool ina = ea < kS, inb = eb < kS;
  TV *w = V + I.v_off + (int64_t)(j + 1) * kS;
  double a0 = ina ? (double)w[ea] : 0.0, a1 = inb ? (double)w[eb] : 0.0;
  for (int t = threadIdx.x; t < j; t += kBlock) {   // the earlier rotations, for the Givens step
    cl[t] = cs[I.st_off + t];
    sl[t] = sn[I.st_off + t];
  }
  double nn;
  if (RB && j < kBasisRegs) {   // the basis loads overlap the reduction of the partials
    double va[kBasisRegs], vb[kBasisRegs];
    prefetch_basis(V + I.v_off, kS, ea, ina, inb, j, va, vb);
    nn = reduce_coef_givens(I, part1, part2, partn, scale, j, coef, hcol, h2sq, lds4);
#pragma unroll
    for (int t = 0; t < kBasisRegs; ++t) {
      if (t <= j) {
        const double c = coef[t];
        a0 -= c * va[t];
        a1 -= c * vb[t];
      }
    }
  } else {
    nn = reduce_coef_givens(I, part1, part2, partn, scale, j, coef, hcol, h2sq, lds4);
    const TV *Vt = V + I.v_off + ea;
#pragma unroll 4
    for (int t = 0; t <= j; ++t, Vt += kS) {
      const double c = coef[t];
      if (ina) a0 -= c * (double)Vt[0];
      if (inb) a1 -= c * (double)Vt[kBlock];
    }
  }
  if (ina) w[ea] = (TV)a0;
  if (inb) w[eb] = (TV)a1;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int prev = atomicAdd(&arrive[i], 1);
    last_s = prev == I.nchunk_x - 1;
    if (last_s) arrive[i] = 0;   // ready for the next iteration's launch
  }
  __syncthreads();
  if (!last_s) return;
  givens_rotate(I, i, j, nn, scale, R, cs, sn, g, gs, maxit, tol, sh, true, G.r0, G.ref);
}

// Segment-wide sums of per-chunk partials, for instances that share one
// Krylov space: out[st_off + t] = sum over the segment's instances and
// chunks of part[part_off + t nchunk_x + c], t = 0 .. iter (dots), or of
// part[part_off + c] (norm).  Grid (coefficient, instance); only segment
// leaders work.  Fixed summation order.
__global__ __launch_bounds__(kBlock) void k_seg_reduce(const InstDev *__restrict__ ins,
                                                       const double *__restrict__ part, double *__restrict__ out,
                                                       const GState *__restrict__ gs, int norm) {
  __shared__ double lds4[4];
  const int i = blockIdx.y, t = blockIdx.x;
  const InstDev L = ins[i];
  if (L.seg_first != i || !gs[i].active) return;
  if (norm ? t > 0 : t > gs[i].iter) return;
  double a = 0.0;
  for (int m = i; m < i + L.seg_count; ++m) {
    const InstDev M = ins[m];
    const double *p = part + M.part_off + (norm ? 0 : (int64_t)t * M.nchunk_x);
    for (int c = threadIdx.x; c < M.nchunk_x; c += kBlock) a += p[c];
  }
  a = block_sum(a, lds4);
  if (threadIdx.x == 0) out[L.st_off + t] = a;
}

__global__ __launch_bounds__(kBlock) void k_givens(
    const InstDev *__restrict__ ins, const double *__restrict__ part1, const double *__restrict__ part2,
    const double *__restrict__ partn, double *__restrict__ scale, double *__restrict__ R,
    double *__restrict__ cs, double *__restrict__ sn, double *__restrict__ g, GState *__restrict__ gs,
    int maxit, double tol, const double *__restrict__ r1, const double *__restrict__ r2,
    const double *__restrict__ rn) {
  extern __shared__ double sh[];   // 3 maxit + 2
  __shared__ double lds4[4];
  const int i = blockIdx.x;
  const InstDev I = ins[i];
  const GState G = gs[i];
  if (I.seg_first != i) return;   // a segment's Givens step runs once, on its leader
  if (!G.active) return;
  givens_step(I, i, G.iter, part1, part2, partn, r1, r2, rn, scale, R, cs, sn, g, gs, maxit, tol, sh, lds4);
}

// Least squares R y = g (upper triangular, m = iter columns); writes
// ycoef[t] = y_t s_t for the basis combination.  A triangle of at most
// kTriLds entries is first read into LDS in one parallel pass (column c
// packed at c (c + 1) / 2), so the column sweep waits on no global load.
constexpr int kTriLds = 4096;
__global__ __launch_bounds__(kBlock) void k_backsolve(const InstDev *__restrict__ ins,
                                                      const double *__restrict__ R,
                                                      const double *__restrict__ g,
                                                      const double *__restrict__ scale,
                                                      double *__restrict__ ycoef,
                                                      const GState *__restrict__ gs, int maxit) {
  extern __shared__ double rhs[];   // maxit, then the packed triangle
  double *tri = rhs + maxit;
  const int i = blockIdx.x;
  const InstDev I = ins[i];
  if (I.seg_first != i) return;   // one least-squares solve per segment
  const int m = gs[i].iter;
  const int ntri = m * (m + 1) / 2;
  const bool staged = ntri <= kTriLds;
  for (int t = threadIdx.x; t < m; t += kBlock) rhs[t] = g[I.st_off + t];
  if (staged) {
    for (int q = threadIdx.x; q < ntri; q += kBlock) {
      int c = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
      if (c * (c + 1) / 2 > q) --c;                 // guard the rounding of the root
      if ((c + 1) * (c + 2) / 2 <= q) ++c;
      tri[q] = R[I.rr_off + (int64_t)c * maxit + (q - c * (c + 1) / 2)];
    }
  }
  __syncthreads();
  for (int c = m - 1; c >= 0; --c) {
    const double *Rc = staged ? tri + c * (c + 1) / 2 : R + I.rr_off + (int64_t)c * maxit;
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
// Element-interior elimination (Sec. 2.3): A(k)^-1 per strip.  The strip
// operator is A_j = D + P Lambda, D = blockdiag of the element operators
// (with their own Robin terms), P Lambda the coupling across the z-interfaces
// inside the strip.  By the capacitance (Woodbury) identity
//   A_j^-1 v = w - D^-1 P q,  w = D^-1 v,  q = K^-1 Lambda w,  K = I + Lambda D^-1 P,
// every element is solved independently and only the small z-interface
// system K couples them.  All strips of one class share D^-1 and K^-1, so
// each of the three products is a GEMM whose columns are the (instance,
// strip) vectors: k_colgemm below, on FP64 MFMA.
//
// Two schedules of the same product.  k_colgemm (few items: latency-bound
// launches): grid (item, 16-row tile), 8 waves split K, each multiplies its
// 16 rows by CT tiles of 16 columns with v_mfma_f64_16x16x4f64, U K-steps of
// loads in flight, the K parts summed in LDS in a fixed order.
// k_colgemm_t (LDS-staged): grid (item, 16 RW-row tile), 4 waves; the
// columns are staged through double-buffered LDS in chunks of 32 K-values
// with coalesced loads (each column is contiguous in memory) while the next
// chunk's operands are in flight.  RW = 4: each wave owns 16 rows over all of
// K (many items: throughput-bound launches).  RW = 2 or 1: 4 / RW waves share
// each 16 rows and split every chunk's K-steps between them, their sums added
// in LDS in a fixed order; this shortens each wave's chain of dependent MFMAs
// and spreads one item over more CUs (few items: latency-bound launches).
// MODE 0: Y = A X; MODE 1: Y -= A X.  X and Y must not overlap.
__device__ inline double colval(const double *__restrict__ xb, int64_t x1, int64_t x2, int k, int K, int ks) {
  if (k >= K) return 0.0;
  if (k < ks) return x1 >= 0 ? xb[x1 + k] : 0.0;
  return x2 >= 0 ? xb[x2 + (k - ks)] : 0.0;
}

template <int CT, int MODE>
__global__ __launch_bounds__(512) void k_colgemm(const CGItem *__restrict__ items, const CGCol *__restrict__ cols,
                                                 const double *__restrict__ xb, double *__restrict__ yb) {
  constexpr int VC = 16 * CT;
  constexpr int KP = 8;
  constexpr int U = 4;
  __shared__ double red[KP * 16 * VC];
  const CGItem it = items[blockIdx.x];
  const int rt = blockIdx.y;
  if (rt * 16 >= it.R) return;
  const int kp = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int arow = rt * 16 + (lane & 15);
  const bool alive = arow < it.R;
  const int kq = lane >> 4, cl = lane & 15;
  int64_t x1[CT], x2[CT];
#pragma unroll
  for (int t = 0; t < CT; ++t) {
    const int ci = t * 16 + cl;
    const bool ok = ci < it.ccount;
    x1[t] = ok ? cols[it.cstart + ci].x1 : -1;
    x2[t] = ok ? cols[it.cstart + ci].x2 : -1;
  }
  using Acc = Mfma<double>::Acc;
  Acc acc[CT];
#pragma unroll
  for (int t = 0; t < CT; ++t) acc[t] = Acc{0, 0, 0, 0};
  const int K = it.K, ks = it.ksplit;
  const int nsteps = (K + 3) >> 2;
  const int s0 = (nsteps * kp) / KP, s1 = (nsteps * (kp + 1)) / KP;
  for (int st = s0; st < s1; st += U) {
    double a[U], b[CT][U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = 4 * (st + u) + kq;
      const bool kin = st + u < s1 && k < K;
      const int ka = k < ks ? k : k + it.agap;
      a[u] = (alive && kin) ? it.A[(size_t)ka * it.lda + arow] : 0.0;
#pragma unroll
      for (int t = 0; t < CT; ++t) b[t][u] = kin ? colval(xb, x1[t], x2[t], k, K, ks) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < CT; ++t) acc[t] = Mfma<double>::mac(a[u], b[t][u], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < CT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) red[(kp * 16 + Mfma<double>::row(lane, j)) * VC + t * 16 + cl] = acc[t][j];
  __syncthreads();
  for (int idx = threadIdx.x; idx < 16 * VC; idx += 512) {
    const int lr = idx / VC, ci = idx - lr * VC;
    const int row = rt * 16 + lr;
    if (ci < it.ccount && row < it.R) {
      double v = red[idx];
#pragma unroll
      for (int q = 1; q < KP; ++q) v += red[q * 16 * VC + idx];
      const int64_t yo = cols[it.cstart + ci].y + row;
      if (MODE == 0) yb[yo] = v;
      else yb[yo] -= v;
    }
  }
}

template <int CT, int MODE, int RW>
__global__ __launch_bounds__(256) void k_colgemm_t(const CGItem *__restrict__ items, const int2 *__restrict__ units,
                                                   const CGCol *__restrict__ cols, const double *__restrict__ xb,
                                                   double *__restrict__ yb) {
  // Staging: the TPC = 16 / CT threads of a column read its chunk interleaved
  // (thread j takes k = j + TPC p), so one load instruction covers TPC
  // consecutive values of each column.  The LDS serves 8-byte accesses 16
  // lanes at a time; a row pitch of CT mod 16 doubles puts those 16 lanes in
  // distinct bank slots, for the stores (TPC rows x CT columns) and for the
  // MFMA operand reads (16 columns of one row).
  // chunks of 64 K-values where the waves split K: half as many chunks, each
  // one staged while the last is multiplied
  constexpr int VC = 16 * CT, KC = RW == 4 ? 32 : 64, PITCH = VC + CT;
  constexpr int PV = KC * VC / 256;      // staged values per thread per chunk
  constexpr int TPC = KC / PV;           // threads per column
  constexpr int KW = 4 / RW;             // waves splitting the K-steps of 16 rows
  constexpr int TR = 16 * RW;            // rows per tile
  constexpr int SW = KC / 4 / KW;        // K-steps per wave per chunk
  static_assert(RW == 1 || RW == 2 || RW == 4, "4 waves per workgroup");
  static_assert((KW - 1) * RW * 4 * CT * 64 <= 2 * KC * PITCH, "K-split sums fit in the staging buffers");
  __shared__ double Bs[2][KC * PITCH];
  __shared__ int64_t c1[VC], c2[VC];
  int item = blockIdx.x, rg = blockIdx.y;
  if (units) {   // XCD-ordered (item, 64-row tile) list; x < 0 pads a bucket
    const int2 u = units[blockIdx.x];
    if (u.x < 0) return;
    item = u.x; rg = u.y;
  }
  const CGItem it = items[item];
  if (rg * TR >= it.R) return;
  if (threadIdx.x < VC) {
    const bool ok = (int)threadIdx.x < it.ccount;
    c1[threadIdx.x] = ok ? cols[it.cstart + threadIdx.x].x1 : -1;
    c2[threadIdx.x] = ok ? cols[it.cstart + threadIdx.x].x2 : -1;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rw = wave % RW, kw = wave / RW;
  const int arow = rg * TR + rw * 16 + (lane & 15);
  const bool alive = arow < it.R, wlive = rg * TR + rw * 16 < it.R;
  const int kq = lane >> 4, cl = lane & 15;
  const int ctl = (it.ccount + 15) >> 4;   // column tiles holding columns
  const bool narrow = it.ccount <= 4;
  const int K = it.K, ks = it.ksplit, lda = it.lda, agap = it.agap;
  const double *__restrict__ A = it.A;
  const int scol = threadIdx.x / TPC, sj = threadIdx.x % TPC;
  const int64_t sx1 = c1[scol], sx2 = c2[scol];
  double pre[PV];
  double a[SW], an[SW];
  auto load_b = [&](int kc) {
#pragma unroll
    for (int p = 0; p < PV; ++p) pre[p] = colval(xb, sx1, sx2, kc * KC + sj + TPC * p, K, ks);
  };
  auto load_a = [&](int kc, double *dst) {   // this wave's K-steps s KW + kw
#pragma unroll
    for (int s = 0; s < SW; ++s) {
      const int k = kc * KC + 4 * (s * KW + kw) + kq;
      const int ka = k < ks ? k : k + agap;
      dst[s] = (alive && k < K) ? A[(size_t)ka * lda + arow] : 0.0;
    }
  };
  auto store_b = [&](int buf) {
#pragma unroll
    for (int p = 0; p < PV; ++p) Bs[buf][(sj + TPC * p) * PITCH + scol] = pre[p];
  };
  using Acc = Mfma<double>::Acc;
  Acc acc[CT];
#pragma unroll
  for (int t = 0; t < CT; ++t) acc[t] = Acc{0, 0, 0, 0};
  const int nchunks = (K + KC - 1) / KC;
  load_b(0);
  load_a(0, a);
  store_b(0);
  __syncthreads();
  for (int kc = 0; kc < nchunks; ++kc) {
    const int buf = kc & 1;
    const bool more = kc + 1 < nchunks;
    if (more) {
      load_b(kc + 1);
      load_a(kc + 1, an);
    }
    const double *__restrict__ B = Bs[buf];
    // A wave whose 16 rows all lie past the block stages only; an item of at
    // most 16 columns multiplies one column tile, and one of at most 4 the
    // 4-block 4 x 4 x 4 MFMA (blocks = the wave's four 4-row groups).
    if (wlive && narrow) {
#pragma unroll
      for (int s = 0; s < SW; ++s)
        acc[0][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[s], B[(4 * (s * KW + kw) + kq) * PITCH + (lane & 3)], acc[0][0],
                                                       0, 0, 0);
    } else if (wlive && ctl > 1) {
#pragma unroll
      for (int s = 0; s < SW; ++s)
#pragma unroll
        for (int t = 0; t < CT; ++t)
          acc[t] = Mfma<double>::mac(a[s], B[(4 * (s * KW + kw) + kq) * PITCH + t * 16 + cl], acc[t]);
    } else if (wlive) {
#pragma unroll
      for (int s = 0; s < SW; ++s) acc[0] = Mfma<double>::mac(a[s], B[(4 * (s * KW + kw) + kq) * PITCH + cl], acc[0]);
    }
    if (more) {
      store_b(buf ^ 1);
#pragma unroll
      for (int s = 0; s < SW; ++s) a[s] = an[s];
    }
    __syncthreads();
  }
  if constexpr (KW > 1) {   // add the K parts; the staging buffers are free
    double *red = &Bs[0][0];
    if (kw > 0)
#pragma unroll
      for (int t = 0; t < CT; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) red[((((kw - 1) * RW + rw) * CT + t) * 4 + j) * 64 + lane] = acc[t][j];
    __syncthreads();
    if (kw > 0) return;
#pragma unroll
    for (int q = 1; q < KW; ++q)
#pragma unroll
      for (int t = 0; t < CT; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[t][j] += red[((((q - 1) * RW + rw) * CT + t) * 4 + j) * 64 + lane];
  }
  if (narrow) {   // lane m: row 4 ((m >> 2) & 3) + (m >> 4) of the wave's 16, column m & 3
    const int ci = lane & 3;
    const int row = rg * TR + rw * 16 + 4 * ((lane >> 2) & 3) + (lane >> 4);
    if (ci < it.ccount && row < it.R) {
      const int64_t y0 = cols[it.cstart + ci].y;
      if (MODE == 0) yb[y0 + row] = acc[0][0];
      else yb[y0 + row] -= acc[0][0];
    }
    return;
  }
#pragma unroll
  for (int t = 0; t < CT; ++t) {
    const int ci = t * 16 + cl;
    if (ci >= it.ccount) continue;
    const int64_t y0 = cols[it.cstart + ci].y;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = rg * TR + rw * 16 + Mfma<double>::row(lane, j);
      if (row < it.R) {
        if (MODE == 0) yb[y0 + row] = acc[t][j];
        else yb[y0 + row] -= acc[t][j];
      }
    }
  }
}

// lambda = Lambda w for every (instance, strip): the lo functional of
// z-interface i reads element i, the up functional reads element i+1.
__global__ __launch_bounds__(kBlock) void k_lambda(const SysDev *__restrict__ sys, const InstDev *__restrict__ ins,
                                                   const int2 *__restrict__ work, const double *__restrict__ w,
                                                   double *__restrict__ lam) {
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, j = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int n = S.n, n2 = S.n2, mz = S.mz, nq = S.nq;
  const double *ws = w + I.f_off + (int64_t)j * mz * n2;
  for (int idx = threadIdx.x; idx < nq; idx += kBlock) {
    const int iface = idx / (2 * n), r = idx - iface * 2 * n;
    const int part = r / n, t = r - part * n;
    const double *coef = part == 0 ? S.lo + (iface + 1) * n : S.up + iface * n;
    const double *we = ws + (int64_t)(part == 0 ? iface : iface + 1) * n2 + t;
    // fully unrolled to the largest n so that every load is issued at once
    double cv[kMaxNodes], wv[kMaxNodes];
#pragma unroll
    for (int c = 0; c < kMaxNodes; ++c) {
      cv[c] = c < n ? coef[c] : 0.0;
      wv[c] = c < n ? we[c * n] : 0.0;
    }
    double a = 0.0;
#pragma unroll
    for (int c = 0; c < kMaxNodes; ++c) a += cv[c] * wv[c];
    lam[I.lam_off + (int64_t)j * nq + idx] = a;
  }
}

// RHS of Eq. (smpm_poisson): F = f + tau g on the physical edges (corners get
// both sides); for singular (k = 0) systems, partials of u_L . F and ||F||^2
// for the Sec. 2.4 projection.
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
    double v = f[I.f_off + e];
    if (g) {   // node (a, b) of element el of strip j; instance-local, 32-bit
      int rem = (int)e;
      const int a = rem % n; rem /= n;
      const int b = rem % n; rem /= n;
      const int el = rem % mz;
      const int j = rem / mz;
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
  if (!S.singular) return;   // the sums feed only the k = 0 projection and its defect
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
    double a;
    if (v) {
      const int e = row / n, b = row - e * n;
      const double *vr = v + I.f_off + ((int64_t)strip * mz + e) * n2 + (int64_t)b * n;
      a = 0.0;
      for (int c = 0; c < n; ++c) a += beta[c] * vr[c];
      bS[I.x_off + (int64_t)h * N + row] = a;
    } else {   // b_S formed already (B A^-1 GEMM): the u_S partial sums only
      a = bS[I.x_off + (int64_t)h * N + row];
    }
    if (S.singular) pd += S.uS[(int64_t)h * N + row] * a;
  }
  pd = block_sum(pd, lds4);
  if (threadIdx.x == 0) hs[I.hs_off + h] = pd;
}

// b~ = b_S - u_S (u_S^T b_S) (Eq. regularize_schur), partials per half in hs;
// then the chunk's partials of ||b~||^2 and u_S . b~ into partn (pairs per
// chunk, as k_xupdate's residual mode leaves them), for every system.
__global__ __launch_bounds__(kBlock) void k_proj_x(const SysDev *__restrict__ sys,
                                                   const InstDev *__restrict__ ins,
                                                   const int2 *__restrict__ work,
                                                   double *__restrict__ x,
                                                   const double *__restrict__ hs,
                                                   double *__restrict__ partn) {
  __shared__ double lds4[4];
  __shared__ double alpha_s;
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  double alpha = 0.0;
  if (S.singular) {
    double a = 0.0;
    for (int c = threadIdx.x; c < S.nh; c += kBlock) a += hs[I.hs_off + c];
    a = block_sum(a, lds4);
    if (threadIdx.x == 0) alpha_s = a;
    __syncthreads();
    alpha = alpha_s;
  }
  double nn = 0.0, ud = 0.0;
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = (int64_t)ch * kChunk + threadIdx.x + q * kBlock;
    if (e >= S.kS) continue;
    double v = x[I.x_off + e];
    if (S.singular) {
      v -= alpha * S.uS[e];
      x[I.x_off + e] = v;
      ud += S.uS[e] * v;
    }
    nn += v * v;
  }
  nn = block_sum(nn, lds4);
  __syncthreads();
  ud = block_sum(ud, lds4);
  if (threadIdx.x == 0) {
    partn[I.part_off + 2 * ch] = nn;
    partn[I.part_off + 2 * ch + 1] = ud;
  }
}

// Z^T partial sums of an interface vector in precision T (Sec. 3.3): per
// (instance, half) either the whole half's sum in its first 16-row slot
// (zm = 1, the layout of the GEMM epilogues; other slots zeroed) or one sum
// per element segment (zm = m_z).  Reads Krylov slot `iter` times the basis
// scale when x_vslot is set (the two-level preconditioner).  Stopped
// instances are skipped when gs is given.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_zt(const SysDev *__restrict__ sys, const InstDev *__restrict__ ins,
                                               const int2 *__restrict__ work, const T *__restrict__ x, int x_vslot,
                                               const double *__restrict__ scale, const GState *__restrict__ gs,
                                               double *__restrict__ hs) {
  __shared__ double lds4[4];
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, h = wk.y;
  if (gs && !gs[i].active) return;
  const int it = gs ? gs[i].iter : 0;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int N = S.N;
  const int64_t off = (x_vslot ? I.v_off + (int64_t)it * S.kS : I.x_off) + (int64_t)h * N;
  const double sc = scale ? scale[I.st_off + it] : 1.0;
  const int sl = hs_slots(S);
  if (S.zm == 1) {
    double *out = hs + I.hs_off + h;   // slot q at out[q nh]
    double a = 0.0;
    for (int row = threadIdx.x; row < N; row += kBlock) a += (double)x[off + row];
    a = block_sum(a, lds4);
    if (threadIdx.x == 0) out[0] = a * sc;
    for (int q = 1 + (int)threadIdx.x; q < sl; q += kBlock) out[(int64_t)q * S.nh] = 0.0;
  } else {
    double *out = hs + I.hs_off + (int64_t)h * sl;
    // wave w sums segments w, w + 4, ...: one row per lane (n <= 64)
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int e = wave; e < S.zm; e += 4) {
      double a = lane < S.n ? (double)x[off + (int64_t)e * S.n + lane] : 0.0;
      a = wave_sum(a);
      if (lane == 0) out[e] = a * sc;
    }
  }
}

// z += Z c in precision T (the coarse term of the two-level preconditioner).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_add_zc(const SysDev *__restrict__ sys, const InstDev *__restrict__ ins,
                                                   const int2 *__restrict__ work, T *__restrict__ z,
                                                   const double *__restrict__ cvec, const GState *__restrict__ gs) {
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  if (gs && !gs[i].active) return;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  const int N = S.N;
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = (int64_t)ch * kChunk + threadIdx.x + q * kBlock;
    if (e >= S.kS) continue;
    const int h = (int)e / N;
    z[I.x_off + e] = (T)((double)z[I.x_off + e] + cvec[I.c_off + z_col(S, h, (int)e - h * N)]);
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
      const int h = (int)e / N, row = (int)e - h * N;
      w -= sz_c(S, h, row, cvec + I.c_off, 0);
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
                                                        int enable, const double *__restrict__ nb, double bfrac) {
  __shared__ double lds4[4];
  const int i = blockIdx.x;
  const InstDev I = ins[i];
  if (I.seg_first != i) return;   // a segment starts once, on its leader
  double nn = 0.0, pb = 0.0, nbb = 0.0;
  for (int m = i; m < i + I.seg_count; ++m) {
    const InstDev M = ins[m];
    for (int c = threadIdx.x; c < M.nchunk_x; c += kBlock) nn += partn[M.part_off + c];
    if (pairs) pb += pairs[2 * m];
    if (nb) nbb += nb[2 * m];
  }
  nn = block_sum(nn, lds4);
  if (threadIdx.x == 0) {
    const double r0 = sqrt(nn);
    GState st;
    st.iter = 0;
    st.r0 = r0;
    st.res = r0;
    st.pad = 0;
    // stopping reference: |g| <= tol * ref.  In a refinement sweep the
    // reference is also floored at bfrac * ||b~||, so the sweep stops once
    // the outer tolerance is within reach instead of at a fixed reduction.
    double ref = pairs ? sqrt(pb) : r0;
    if (nb && bfrac > 0.0) ref = fmax(ref, bfrac * sqrt(nbb));
    st.ref = ref;
    if (!isfinite(r0)) { st.active = 0; st.status = 3; }
    else if (r0 == 0.0 || !enable) { st.active = 0; st.status = 1; }
    else { st.active = 1; st.status = 0; }
    for (int m = i; m < i + I.seg_count; ++m) gs[m] = st;
    scale[I.st_off] = r0 > 0.0 ? 1.0 / r0 : 0.0;
    g[I.st_off] = r0;
  }
}

// Elementwise interface-space helpers.
// mode 0: out = a + Z c          (x_S = z + Z c')
// mode 1: out = out + a + Z c    (refinement update)
// mode 2: out = base - a         (residual r = b - S x; base = nullptr: out
//                                holds b), partials ||r||^2 and u_S . r
// mode 3: out = a - (S Z) c      (deflation P)
// mode 4: out = a - Z c          (deflation Q after c = G Z^T S a)
template <typename TA>
__global__ __launch_bounds__(kBlock) void k_xupdate(const SysDev *__restrict__ sys,
                                                    const InstDev *__restrict__ ins,
                                                    const int2 *__restrict__ work, int mode,
                                                    const TA *__restrict__ a,
                                                    const double *__restrict__ cvec,
                                                    double *__restrict__ out,
                                                    double *__restrict__ partn,
                                                    const double *__restrict__ base) {
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
    const int h = (int)e / N;
    const int row = (int)e - h * N;
    const int zc = z_col(S, h, row);
    double v = a ? (double)a[I.x_off + e] : 0.0;
    if (mode == 2) {   // residual: base - a (- (S Z) c when cvec is given)
      if (cvec) v += sz_c(S, h, row, cvec + I.c_off, 0);
      v = (base ? base[I.x_off + e] : out[I.x_off + e]) - v;
      out[I.x_off + e] = v;
      nn += v * v;
      if (S.singular) ud += S.uS[e] * v;
      continue;
    }
    if (mode == 3) {
      v -= sz_c(S, h, row, cvec + I.c_off, 0);
    } else if (mode == 4) {
      v -= cvec[I.c_off + zc];
    } else {
      if (cvec) v += cvec[I.c_off + zc];
      if (mode == 1) v += out[I.x_off + e];
    }
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

// Recovery right-hand side of Algorithm 2: R = F~ - E x_S.
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
    int rem = (int)e;   // instance-local node index: 32-bit arithmetic
    const int a = rem % n; rem /= n;
    const int b = rem % n; rem /= n;
    const int el = rem % mz;
    const int j = rem / mz;
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
  if (!S.singular) return;   // only the k = 0 gauge needs the sum (k_sub_mean reads it only then)
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
                                                     const double *__restrict__ v, double *__restrict__ u,
                                                     const double *__restrict__ pr) {
  __shared__ double lds4[4];
  __shared__ double mean_s;
  const int2 wk = work[blockIdx.x];
  const int i = wk.x, ch = wk.y;
  const InstDev I = ins[i];
  const SysDev &S = sys[I.sys];
  double mean = 0.0;
  if (S.singular) {   // zero nodal mean (the Neumann problem's gauge)
    double a = 0.0;
    for (int c = threadIdx.x; c < I.nchunk_r; c += kBlock) a += pr[I.pr_off + 2 * c];
    a = block_sum(a, lds4);
    if (threadIdx.x == 0) mean_s = a / (double)S.r;
    __syncthreads();
    mean = mean_s;
  }
  for (int q = 0; q < kChunk / kBlock; ++q) {
    const int64_t e = (int64_t)ch * kChunk + threadIdx.x + q * kBlock;
    if (e < S.r) u[I.f_off + e] = v[I.f_off + e] - mean;
  }
}

// Reduce interface-space partial pairs (||r||^2, u_S . r) to one instance
// scalar pair: out[2 i], out[2 i + 1] (and the same into out2 if given).
__global__ __launch_bounds__(kBlock) void k_reduce_pairs(const InstDev *__restrict__ ins,
                                                         const double *__restrict__ partn,
                                                         double *__restrict__ out, double *__restrict__ out2) {
  __shared__ double lds4[4];
  const int i = blockIdx.x;
  const InstDev I = ins[i];
  double a = 0.0, b = 0.0;
  for (int c = threadIdx.x; c < I.nchunk_x; c += kBlock) { a += partn[I.part_off + 2 * c]; b += partn[I.part_off + 2 * c + 1]; }
  a = block_sum(a, lds4);
  __syncthreads();
  b = block_sum(b, lds4);
  if (threadIdx.x == 0) {
    out[2 * i] = a;
    out[2 * i + 1] = b;
    if (out2) {
      out2[2 * i] = a;
      out2[2 * i + 1] = b;
    }
  }
}

// The transform in the periodic y direction of the 3-D problem (Sec. 5) as a
// dense product: C[M x ncol] = A[M x K] B[K x ncol], all row-major FP64.  A is
// the small real DFT (or inverse DFT) matrix, B and C stream one row per y
// plane (or per mode and Re/Im part), so the kernel is bound by HBM.  Grid
// (ceil(ncol / 64), ceil(M / (16 kDftTiles))); wave w owns 16 columns, lane
// layout as for the other MFMA kernels; up to kDftTiles row tiles per wave.
// K runs in chunks of 32: the chunk of A is staged in LDS, and the next
// chunk's B values are loaded into registers while this chunk's MFMAs run.
constexpr int kDftTiles = 10;
__global__ __launch_bounds__(256) void k_dft_gemm(const double *__restrict__ A, int M, int K,
                                                  const double *__restrict__ B, double *__restrict__ C, int64_t ncol) {
  constexpr int KC = 32, PA = KC + 1;
  __shared__ double As[kDftTiles * 16 * PA];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kq = lane >> 4, cl = lane & 15;
  const int64_t col = (int64_t)blockIdx.x * 64 + wave * 16 + cl;
  const bool cin = col < ncol;
  const int t0 = blockIdx.y * kDftTiles;
  const int nt = min(kDftTiles, (M + 15) / 16 - t0);
  if (nt <= 0) return;
  const int row0 = t0 * 16;
  using Acc = Mfma<double>::Acc;
  Acc acc[kDftTiles];
#pragma unroll
  for (int t = 0; t < kDftTiles; ++t) acc[t] = Acc{0, 0, 0, 0};
  double bv[KC / 4], bn[KC / 4];
  auto load_b = [&](int k0, double *dst) {
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int k = k0 + 4 * s + kq;
      dst[s] = (cin && k < K) ? B[(int64_t)k * ncol + col] : 0.0;
    }
  };
  load_b(0, bv);
  for (int k0 = 0; k0 < K; k0 += KC) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < nt * 16 * KC; idx += 256) {
      const int rr = idx / KC, kk = idx - rr * KC;
      const int row = row0 + rr, k = k0 + kk;
      As[rr * PA + kk] = (row < M && k < K) ? A[(int64_t)row * K + k] : 0.0;
    }
    __syncthreads();
    const bool more = k0 + KC < K;
    if (more) load_b(k0 + KC, bn);
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
#pragma unroll
      for (int t = 0; t < kDftTiles; ++t)
        if (t < nt) acc[t] = Mfma<double>::mac(As[(t * 16 + cl) * PA + 4 * s + kq], bv[s], acc[t]);
    }
    if (more) {
#pragma unroll
      for (int s = 0; s < KC / 4; ++s) bv[s] = bn[s];
    }
  }
#pragma unroll
  for (int t = 0; t < kDftTiles; ++t) {
    if (t >= nt) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = (t0 + t) * 16 + Mfma<double>::row(lane, j);
      if (row < M && cin) C[(int64_t)row * ncol + col] = acc[t][j];
    }
  }
}

// p[0, n) = v.
// The transform in y of Sec. 5 (Alg. 3) as a radix-2 FFT, for m_y a power of
// two.  Each workgroup takes CT = kFftSlots / m_y consecutive columns (nodes
// of the 2-D section) with all m_y planes, staged in LDS as complex values in
// bit-reversed plane order, and runs the log2(m_y) butterfly stages there
// (decimation in time); every column is read and written once.
//   forward: out[(2m + q) ncol + c] = (1/m_y) sum_j in[j ncol + c] (cos, -sin)(2 pi m j / m_y),
//            m = 0 .. m_y/2, q = 0 (Re), 1 (Im);
//   inverse: out[j ncol + c] = sum_m w_m (Re_m cos - Im_m sin)(2 pi m j / m_y), w_0 = w_{m_y/2} = 1,
//            else 2: the inverse transform of the Hermitian spectrum X_{m_y - m} = conj(X_m).
// tw[k] = exp(-2 pi i k / m_y), k < m_y / 2 (the inverse uses the conjugates).
constexpr int kFftSlots = 4096;   // complex values staged per workgroup (64 KiB)
template <bool INV>
__global__ __launch_bounds__(256) void k_fft_y(const double *__restrict__ in, double *__restrict__ out, int my,
                                               int logmy, int64_t ncol, const double2 *__restrict__ tw) {
  extern __shared__ double2 fb[];   // [m_y][CT]
  const int CT = kFftSlots / my;
  const int64_t c0 = (int64_t)blockIdx.x * CT;
  const int nc = (int)min<int64_t>(CT, ncol - c0);
  const int nk = my / 2 + 1;
  auto brev = [&](int j) { return (int)(__brev((unsigned)j) >> (32 - logmy)); };
  if (!INV) {
    for (int idx = threadIdx.x; idx < my * CT; idx += blockDim.x) {
      const int j = idx / CT, c = idx - j * CT;
      const double v = c < nc ? in[(int64_t)j * ncol + c0 + c] : 0.0;
      fb[brev(j) * CT + c] = make_double2(v, 0.0);
    }
  } else {
    for (int idx = threadIdx.x; idx < nk * CT; idx += blockDim.x) {
      const int m = idx / CT, c = idx - m * CT;
      double re = 0.0, im = 0.0;
      if (c < nc) {
        re = in[(int64_t)(2 * m) * ncol + c0 + c];
        im = in[(int64_t)(2 * m + 1) * ncol + c0 + c];
      }
      if (m == 0 || m == my / 2) im = 0.0;   // real modes
      fb[brev(m) * CT + c] = make_double2(re, im);
      if (m > 0 && m < my / 2) fb[brev(my - m) * CT + c] = make_double2(re, -im);
    }
  }
  __syncthreads();
  const int nb = (my / 2) * CT;   // butterflies per stage
  for (int s = 0; s < logmy; ++s) {
    const int half = 1 << s, stride = (my / 2) >> s;   // twiddle step for this stage
    for (int idx = threadIdx.x; idx < nb; idx += blockDim.x) {
      const int p = idx / CT, c = idx - p * CT;
      const int k = p & (half - 1);
      const int i0 = ((p >> s) << (s + 1)) + k, i1 = i0 + half;
      double2 w = tw[k * stride];
      if (INV) w.y = -w.y;
      const double2 a = fb[i0 * CT + c], b = fb[i1 * CT + c];
      const double2 t = make_double2(w.x * b.x - w.y * b.y, w.x * b.y + w.y * b.x);
      fb[i0 * CT + c] = make_double2(a.x + t.x, a.y + t.y);
      fb[i1 * CT + c] = make_double2(a.x - t.x, a.y - t.y);
    }
    __syncthreads();
  }
  if (!INV) {
    const double sc = 1.0 / my;
    for (int idx = threadIdx.x; idx < 2 * nk * CT; idx += blockDim.x) {
      const int row = idx / CT, c = idx - row * CT;
      if (c >= nc) continue;
      const double2 v = fb[(row >> 1) * CT + c];
      out[(int64_t)row * ncol + c0 + c] = ((row & 1) ? v.y : v.x) * sc;
    }
  } else {
    for (int idx = threadIdx.x; idx < my * CT; idx += blockDim.x) {
      const int j = idx / CT, c = idx - j * CT;
      if (c < nc) out[(int64_t)j * ncol + c0 + c] = fb[j * CT + c].x;
    }
  }
}

// The same transforms for m_y = 2^LOGMY <= 2048 with every size fixed at
// compile time, two real columns per complex FFT: a workgroup takes 2 CT
// consecutive columns (CT = 2048 / m_y) and stages z = x_c + i x_{c+CT}
// (32 KiB of LDS, so several workgroups share a CU).  All of a thread's
// loads are issued before it writes the staging buffer.  Forward: with Z the
// FFT of z, X_c(m) = (Z_m + conj Z_{m_y-m}) / 2 and X_{c+CT}(m) = (Z_m -
// conj Z_{m_y-m}) / (2 i).  Inverse: Z_m = X_c(m) + i X_{c+CT}(m) over all
// m by the Hermitian symmetry of both spectra; the inverse FFT of Z is then
// x_c + i x_{c+CT}.
constexpr int kFftPackSlots = 2048;
template <int LOGMY, bool INV>
__global__ __launch_bounds__(256) void k_fft_y_pack(const double *__restrict__ in, double *__restrict__ out,
                                                    int64_t ncol, const double2 *__restrict__ tw) {
  constexpr int MY = 1 << LOGMY, CT = kFftPackSlots / MY, CW = 2 * CT, NK = MY / 2 + 1;
  static_assert(CT >= 1, "m_y too large for the packed FFT");
  __shared__ double2 fb[MY * CT];
  __shared__ double2 tws[MY / 2];   // the twiddles, staged once: the stages read them from LDS
  for (int k = threadIdx.x; k < MY / 2; k += 256) {
    double2 w = tw[k];
    if (INV) w.y = -w.y;
    tws[k] = w;
  }
  const int64_t c0 = (int64_t)blockIdx.x * CW;
  const int nc = (int)min<int64_t>(CW, ncol - c0);
  auto brev = [](int j) { return (int)(__brev((unsigned)j) >> (32 - LOGMY)); };
  if (!INV) {
    constexpr int PER = MY * CW / 256;   // values per thread
    double v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = threadIdx.x + 256 * q, j = idx / CW, cc = idx % CW;
      v[q] = cc < nc ? in[(int64_t)j * ncol + c0 + cc] : 0.0;
    }
    double *fd = reinterpret_cast<double *>(fb);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = threadIdx.x + 256 * q, j = idx / CW, cc = idx % CW;
      fd[2 * (brev(j) * CT + cc % CT) + cc / CT] = v[q];
    }
  } else {
    constexpr int ITEMS = NK * CT, PER = (ITEMS + 255) / 256;
    double4 v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = threadIdx.x + 256 * q, m = idx / CT, c = idx % CT;
      v[q] = make_double4(0.0, 0.0, 0.0, 0.0);
      if (idx < ITEMS) {
        const double *r0 = in + (int64_t)(2 * m) * ncol + c0, *r1 = r0 + ncol;
        if (c < nc) { v[q].x = r0[c]; v[q].y = r1[c]; }
        if (c + CT < nc) { v[q].z = r0[c + CT]; v[q].w = r1[c + CT]; }
      }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = threadIdx.x + 256 * q, m = idx / CT, c = idx % CT;
      if (idx >= ITEMS) continue;
      double a = v[q].x, b = v[q].y, e = v[q].z, d = v[q].w;   // X_c = a + i b, X_{c+CT} = e + i d
      if (m == 0 || m == MY / 2) b = d = 0.0;                  // real modes
      fb[brev(m) * CT + c] = make_double2(a - d, b + e);
      if (m > 0 && m < MY / 2) fb[brev(MY - m) * CT + c] = make_double2(a + d, e - b);
    }
  }
  __syncthreads();
  constexpr int NB = (MY / 2) * CT, BPER = (NB + 255) / 256;
#pragma unroll
  for (int s = 0; s < LOGMY; ++s) {
    const int half = 1 << s, stride = (MY / 2) >> s;
#pragma unroll
    for (int q = 0; q < BPER; ++q) {
      const int idx = threadIdx.x + 256 * q;
      if (NB % 256 != 0 && idx >= NB) continue;
      const int p = idx / CT, c = idx % CT;
      const int k = p & (half - 1);
      const int i0 = ((p >> s) << (s + 1)) + k, i1 = i0 + half;
      const double2 w = tws[k * stride];
      const double2 a = fb[i0 * CT + c], b = fb[i1 * CT + c];
      const double2 t = make_double2(w.x * b.x - w.y * b.y, w.x * b.y + w.y * b.x);
      fb[i0 * CT + c] = make_double2(a.x + t.x, a.y + t.y);
      fb[i1 * CT + c] = make_double2(a.x - t.x, a.y - t.y);
    }
    __syncthreads();
  }
  if (!INV) {
    constexpr double sc = 0.5 / MY;
    constexpr int ITEMS = 2 * NK * CW;
    for (int idx = threadIdx.x; idx < ITEMS; idx += 256) {
      const int row = idx / CW, cc = idx % CW;
      if (cc >= nc) continue;
      const int m = row >> 1, c = cc % CT;
      const double2 A = fb[m * CT + c], B = fb[((MY - m) & (MY - 1)) * CT + c];
      double val;
      if (cc < CT)   // (A + conj B) / 2
        val = (row & 1) ? (A.y - B.y) : (A.x + B.x);
      else           // (A - conj B) / (2 i)
        val = (row & 1) ? -(A.x - B.x) : (A.y + B.y);
      out[(int64_t)row * ncol + c0 + cc] = val * sc;
    }
  } else {
    constexpr int ITEMS = MY * CW;
    for (int idx = threadIdx.x; idx < ITEMS; idx += 256) {
      const int j = idx / CW, cc = idx % CW;
      if (cc >= nc) continue;
      const double2 z = fb[j * CT + cc % CT];
      out[(int64_t)j * ncol + c0 + cc] = cc < CT ? z.x : z.y;
    }
  }
}

// W_16^m = exp(-2 pi i m / 16), m < 8, correctly rounded (W_{2h}^k = W_16^{8k/h}):
// the butterflies of a length-R DFT, R <= 16, take their twiddles as
// constants, exact for m = 0 (1) and m = 4 (-i).
__device__ constexpr double w16re(int m) {
  return m == 0 ? 1.0 : m == 1 ? 0.9238795325112867 : m == 2 ? 0.7071067811865476 : m == 3 ? 0.3826834323650898
       : m == 4 ? 0.0 : m == 5 ? -0.3826834323650898 : m == 6 ? -0.7071067811865476 : -0.9238795325112867;
}
__device__ constexpr double w16im(int m) {
  return m == 0 ? 0.0 : m == 1 ? -0.3826834323650898 : m == 2 ? -0.7071067811865476 : m == 3 ? -0.9238795325112867
       : m == 4 ? -1.0 : m == 5 ? -0.9238795325112867 : m == 6 ? -0.7071067811865476 : -0.3826834323650898;
}

// A length-R DFT in registers (R <= 16 a power of two, all indices fixed at
// compile time): `a` holds the inputs in bit-reversed order and ends with the
// outputs in natural order.  Radix-2 decimation in time; the twiddle of span
// 2h is W_{2h}^k = W_16^{8k/h} (conjugated for the inverse).
template <int R, bool INV>
__device__ inline void dft_reg(double2 (&a)[R]) {
  static_assert(R >= 2 && R <= 16 && (R & (R - 1)) == 0, "length 2 .. 16, a power of two");
#pragma unroll
  for (int h = 1; h < R; h *= 2) {
#pragma unroll
    for (int g = 0; g < R; g += 2 * h) {
#pragma unroll
      for (int k = 0; k < h; ++k) {
        const int m = k * (8 / h);
        const double2 b = a[g + k + h];
        double2 t;
        if (m == 0) {
          t = b;
        } else if (m == 4) {   // -i, or i for the inverse
          t = INV ? make_double2(-b.y, b.x) : make_double2(b.y, -b.x);
        } else {
          const double wr = w16re(m), wi = INV ? -w16im(m) : w16im(m);
          t = make_double2(wr * b.x - wi * b.y, wr * b.y + wi * b.x);
        }
        a[g + k + h] = make_double2(a[g + k].x - t.x, a[g + k].y - t.y);
        a[g + k] = make_double2(a[g + k].x + t.x, a[g + k].y + t.y);
      }
    }
  }
}

template <int L>
__device__ constexpr int brev_c(int j) {
  int r = 0;
  for (int b = 0; b < L; ++b) r |= ((j >> b) & 1) << (L - 1 - b);
  return r;
}

// The y transform for m_y = 16 .. 128 as a two-step (four-step) FFT,
// m_y = 8 N2, two real columns per complex FFT as in k_fft_y_pack: with
// j = N2 j1 + j2 and m = k1 + 8 k2, a thread first takes the length-8 DFT over
// j1 of one (column, j2) in registers, multiplies by W^{j2 k1}, and stages
// the result; after one barrier a thread takes the length-N2 DFT over j2 of
// one (column, k1).  Two passes through LDS instead of log2(m_y).
template <int LOGMY, bool INV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(INV ? 3 : 4))) void k_fft_y_4s(
    const double *__restrict__ in, double *__restrict__ out,
                                                  int64_t ncol, const double2 *__restrict__ tw) {
  constexpr int MY = 1 << LOGMY, N1 = 8, N2 = MY / N1, L2 = LOGMY - 3;
  constexpr int CT = kFftPackSlots / MY, CW = 2 * CT, NK = MY / 2 + 1;
  constexpr int I1 = CT * N2, I3 = CT * N1;                 // items of the two steps
  constexpr int P1 = (I1 + 255) / 256, P3 = (I3 + 255) / 256;
  static_assert(N2 >= 2 && N2 <= 16, "m_y from 16 to 128");
  __shared__ double2 fb[MY * CT];
  __shared__ double2 tws[MY / 2];
  for (int k = threadIdx.x; k < MY / 2; k += 256) {
    double2 w = tw[k];
    if (INV) w.y = -w.y;
    tws[k] = w;
  }
  const int64_t c0 = (int64_t)blockIdx.x * CW;
  const int nc = (int)min<int64_t>(CW, ncol - c0);
  auto twid = [&](int idx) {   // W_MY^idx, idx < MY
    const double2 w = tws[idx & (MY / 2 - 1)];
    return idx < MY / 2 ? w : make_double2(-w.x, -w.y);
  };
  double2 a[P1][N1];
  if (!INV) {   // step 1 straight from the planes: z = x_c + i x_{c+CT}
#pragma unroll
    for (int q = 0; q < P1; ++q) {
      const int it = threadIdx.x + 256 * q, c = it % CT, j2 = it / CT;
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) {
        const int64_t row = (int64_t)(N2 * j1 + j2) * ncol + c0;
        const bool ok = it < I1;
        a[q][brev_c<3>(j1)] = make_double2(ok && c < nc ? in[row + c] : 0.0, ok && c + CT < nc ? in[row + c + CT] : 0.0);
      }
    }
    __syncthreads();   // the twiddle table
  } else {   // the full spectrum Z_m = X_c(m) + i X_{c+CT}(m), natural order
    constexpr int PS = (NK * CT + 255) / 256;
    double4 v[PS];   // every load issued before the first store
#pragma unroll
    for (int q = 0; q < PS; ++q) {
      const int it = threadIdx.x + 256 * q, m = it / CT, c = it % CT;
      v[q] = make_double4(0.0, 0.0, 0.0, 0.0);
      if (it < NK * CT) {
        const double *r0 = in + (int64_t)(2 * m) * ncol + c0, *r1 = r0 + ncol;
        if (c < nc) { v[q].x = r0[c]; v[q].y = r1[c]; }
        if (c + CT < nc) { v[q].z = r0[c + CT]; v[q].w = r1[c + CT]; }
      }
    }
#pragma unroll
    for (int q = 0; q < PS; ++q) {
      const int it = threadIdx.x + 256 * q, m = it / CT, c = it % CT;
      if (it >= NK * CT) continue;
      double ar = v[q].x, br = v[q].y, er = v[q].z, dr = v[q].w;   // X_c = a + i b, X_{c+CT} = e + i d
      if (m == 0 || m == MY / 2) br = dr = 0.0;
      fb[m * CT + c] = make_double2(ar - dr, br + er);
      if (m > 0 && m < MY / 2) fb[(MY - m) * CT + c] = make_double2(ar + dr, er - br);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < P1; ++q) {
      const int it = threadIdx.x + 256 * q, c = it % CT, j2 = it / CT;
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1)
        a[q][brev_c<3>(j1)] = it < I1 ? fb[(N2 * j1 + j2) * CT + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();   // every read of the spectrum before step 1 overwrites it
  }
#pragma unroll
  for (int q = 0; q < P1; ++q) {
    const int it = threadIdx.x + 256 * q, c = it % CT, j2 = it / CT;
    dft_reg<N1, INV>(a[q]);
    if (it < I1) {
#pragma unroll
      for (int k1 = 0; k1 < N1; ++k1) {
        const double2 w = twid(j2 * k1), v = a[q][k1];
        fb[(k1 * N2 + j2) * CT + c] = make_double2(w.x * v.x - w.y * v.y, w.x * v.y + w.y * v.x);
      }
    }
  }
  __syncthreads();
  double2 b[P3][N2];
#pragma unroll
  for (int q = 0; q < P3; ++q) {
    const int it = threadIdx.x + 256 * q, c = it % CT, k1 = it / CT;
#pragma unroll
    for (int j2 = 0; j2 < N2; ++j2)
      b[q][brev_c<L2>(j2)] = it < I3 ? fb[(k1 * N2 + j2) * CT + c] : make_double2(0.0, 0.0);
    dft_reg<N2, INV>(b[q]);
  }
  if (INV) {   // z_j at j = k1 + 8 k2: column c in Re, column c + CT in Im
#pragma unroll
    for (int q = 0; q < P3; ++q) {
      const int it = threadIdx.x + 256 * q, c = it % CT, k1 = it / CT;
      if (it >= I3) continue;
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) {
        double *o = out + (int64_t)(k1 + N1 * k2) * ncol + c0;
        if (c < nc) o[c] = b[q][k2].x;
        if (c + CT < nc) o[c + CT] = b[q][k2].y;
      }
    }
    return;
  }
  __syncthreads();   // every read of step 1's output before it is overwritten
#pragma unroll
  for (int q = 0; q < P3; ++q) {
    const int it = threadIdx.x + 256 * q, c = it % CT, k1 = it / CT;
    if (it >= I3) continue;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) fb[(k1 + N1 * k2) * CT + c] = b[q][k2];
  }
  __syncthreads();
  // Each (mode m, packed column c) gives both columns' Re and Im of mode m
  // from the same two spectrum values; the planes are not read again, so the
  // stores bypass the caches.
  constexpr double sc = 0.5 / MY;
  for (int idx = threadIdx.x; idx < NK * CT; idx += 256) {
    const int m = idx / CT, c = idx % CT;
    const double2 A = fb[m * CT + c], B = fb[((MY - m) & (MY - 1)) * CT + c];
    double *o0 = out + (int64_t)(2 * m) * ncol + c0, *o1 = o0 + ncol;
    if (c < nc) {   // column c: (A + conj B) / 2
      __builtin_nontemporal_store((A.x + B.x) * sc, o0 + c);
      __builtin_nontemporal_store((A.y - B.y) * sc, o1 + c);
    }
    if (c + CT < nc) {   // column c + CT: (A - conj B) / (2 i)
      __builtin_nontemporal_store((A.y + B.y) * sc, o0 + c + CT);
      __builtin_nontemporal_store(-(A.x - B.x) * sc, o1 + c + CT);
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_fill(double *__restrict__ p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

// out[0, n) = (float)in[0, n): the FP32 operator tables from the uploaded
// FP64 ones (same padded layout), at setup.
// Column-major copy, rows padded to ld with zeros, of nb row-major rows x cols
// blocks (the setup's tables as the host builds them): 32 x 32 tiles through
// LDS, grid (column tiles, row tiles of ld, blocks), 32 x 8 threads.
__global__ __launch_bounds__(256) void k_colmajor_pad(const double *__restrict__ src, double *__restrict__ dst,
                                                      int nb, int rows, int cols, int ld) {
  __shared__ double tile[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  for (int b = blockIdx.z; b < nb; b += gridDim.z) {
    const double *sb = src + (size_t)b * rows * cols;
    double *db = dst + (size_t)b * ld * cols;
    for (int k = threadIdx.y; k < 32; k += 8) {
      const int r = r0 + k, c = c0 + threadIdx.x;
      tile[k][threadIdx.x] = (r < rows && c < cols) ? sb[(size_t)r * cols + c] : 0.0;
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += 8) {
      const int c = c0 + k, r = r0 + threadIdx.x;
      if (c < cols && r < ld) db[(size_t)c * ld + r] = tile[threadIdx.x][k];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_to_f32(const double *__restrict__ in, float *__restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
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

}  // namespace smpm
