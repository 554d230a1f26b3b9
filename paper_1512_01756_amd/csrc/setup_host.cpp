// Host-side FP64 setup of the SMPM Schur solver.
//
// Discretization (Sec. 2.2, Eq. smpm_poisson): on each axis-aligned element
// the operator is the GLL-collocated Laplacian plus, on each edge node, tau
// times the Robin mismatch (u + n.grad u) - (u_nb + n.grad u_nb) against the
// neighbour, or tau n.grad u on the physical boundary.  One global tau.
//
// Strip split (Sec. 2.3): a strip (m_z elements stacked in z) couples to its
// neighbours only through B; its local operator A_j(k) = A_j - k^2 I is
// block tridiagonal over the elements, factored here by block elimination
// in z (block Thomas).  The Schur blocks W_j = B_rows A_j^-1 E_cols come from
// a multi-right-hand-side solve with those factors.
//
// Block-Jacobi (Sec. 3.2), deflation C = Z^T S Z, S Z (Sec. 3.3) and the null
// vectors (Sec. 2.4: shifted inverse iteration on S^T - sigma I, then
// Claim 1 for u_L) follow.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <future>
#include <map>
#include <stdexcept>
#include <tuple>

#include "host.hpp"

namespace smpm {

// ---------------------------------------------------------------------------
// GLL nodes (Newton on the Legendre recurrence), weights, and the
// differentiation matrix in barycentric form with a negative-sum diagonal.
static void legendre_pair(int N, double x, double &pN, double &pNm1) {
  double p0 = 1.0, p1 = x;
  if (N == 0) { pN = 1.0; pNm1 = 0.0; return; }
  for (int k = 1; k < N; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1; p1 = p2;
  }
  pN = p1; pNm1 = p0;
}

GLL make_gll(int n) {
  if (n < 2) throw std::runtime_error("GLL needs n >= 2");
  GLL g;
  g.n = n;
  g.x.resize(n); g.w.resize(n); g.D.assign((size_t)n * n, 0.0);
  const int N = n - 1;
  g.x[0] = -1.0; g.x[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    double x = -std::cos(M_PI * i / N);
    for (int it = 0; it < 100; ++it) {
      // (1 - x^2) P'_N = N (P_{N-1} - x P_N); roots via q = P_{N+1} - P_{N-1},
      // q' = (2N + 1) P_N.
      double pN, pNm1, pN1, dummy;
      legendre_pair(N, x, pN, pNm1);
      legendre_pair(N + 1, x, pN1, dummy);
      const double dx = (pN1 - pNm1) / ((2.0 * N + 1.0) * pN);
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    g.x[i] = x;
  }
  std::sort(g.x.begin(), g.x.end());
  for (int i = 0; i < n; ++i) {
    double pN, pNm1;
    legendre_pair(N, g.x[i], pN, pNm1);
    g.w[i] = 2.0 / (N * (N + 1.0) * pN * pN);
  }
  std::vector<double> lam(n, 1.0);   // barycentric weights
  for (int j = 0; j < n; ++j) {
    double p = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != j) p *= (g.x[j] - g.x[k]);
    lam[j] = 1.0 / p;
  }
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j)
      if (j != i) {
        const double v = (lam[j] / lam[i]) / (g.x[i] - g.x[j]);
        g.D[(size_t)i * n + j] = v;
        s += v;
      }
    g.D[(size_t)i * n + i] = -s;
  }
  return g;
}

// ---------------------------------------------------------------------------
// Strip operator pieces.  Local node index l = b * n + a.
static void element_diag_block(const System &s, const GLL &g, double hx, double hz,
                               bool w_if, bool e_if, bool s_if, bool n_if,
                               std::vector<double> &Dg) {
  const int n = s.n, n2 = s.n2;
  const double *D = g.D.data();
  std::vector<double> D2((size_t)n * n, 0.0);
  gemm(n, n, n, 1.0, D, n, D, n, 0.0, D2.data(), n);
  Dg.assign((size_t)n2 * n2, 0.0);
  auto at = [&](int b, int a, int bb, int aa) -> double & {
    return Dg[(size_t)(b * n + a) * n2 + (bb * n + aa)];
  };
  const double cx = (2.0 / hx), cz = (2.0 / hz);
  const double tau = s.tau;
  for (int b = 0; b < n; ++b)
    for (int a = 0; a < n; ++a)
      for (int c = 0; c < n; ++c) {
        at(b, a, b, c) += cx * cx * D2[(size_t)a * n + c];
        at(b, a, c, a) += cz * cz * D2[(size_t)b * n + c];
      }
  for (int t = 0; t < n; ++t) {
    // west side a = 0, outward normal -x
    for (int c = 0; c < n; ++c) at(t, 0, t, c) += tau * (-cx * D[c]);
    if (w_if) at(t, 0, t, 0) += tau;
    // east side a = n - 1, outward normal +x
    for (int c = 0; c < n; ++c) at(t, n - 1, t, c) += tau * (cx * D[(size_t)(n - 1) * n + c]);
    if (e_if) at(t, n - 1, t, n - 1) += tau;
    // south side b = 0, outward normal -z
    for (int c = 0; c < n; ++c) at(0, t, c, t) += tau * (-cz * D[c]);
    if (s_if) at(0, t, 0, t) += tau;
    // north side b = n - 1, outward normal +z
    for (int c = 0; c < n; ++c) at(n - 1, t, c, t) += tau * (cz * D[(size_t)(n - 1) * n + c]);
    if (n_if) at(n - 1, t, n - 1, t) += tau;
  }
  const double k2 = s.kwave * s.kwave;
  if (k2 != 0.0)
    for (int l = 0; l < n2; ++l) Dg[(size_t)l * n2 + l] -= k2;
}

// Factor one strip class: G[e] = (D~_e)^-1 with
// D~_0 = Dg_0, D~_e = Dg_e - Lo_e G_{e-1} Up_{e-1}.  Lo_e acts on element
// e-1's column t (coefficients lo[e][c] on (c, t)) into row (0, t) of e; Up_e
// acts on element e+1's column t into row (n-1, t) of e.
static void factor_class(const System &s, const GLL &g, StripClass &cl) {
  const int n = s.n, n2 = s.n2, mz = s.mz;
  cl.G.assign((size_t)mz * n2 * n2, 0.0);
  std::vector<double> Dg;
  for (int e = 0; e < mz; ++e) {
    const double hz = s.zb[e + 1] - s.zb[e];
    element_diag_block(s, g, cl.hx, hz, cl.west_if, cl.east_if, e > 0, e < mz - 1, Dg);
    if (e > 0) {
      const double *Gp = &cl.G[(size_t)(e - 1) * n2 * n2];
      const double *lo = &s.lo[(size_t)e * n];
      const double *upp = &s.up[(size_t)(e - 1) * n];
      for (int t = 0; t < n; ++t)
        for (int tp = 0; tp < n; ++tp) {
          double gam = 0.0;   // sum_c lo[c] G_{e-1}[(c,t)][(n-1,tp)]
          for (int c = 0; c < n; ++c) gam += lo[c] * Gp[(size_t)(c * n + t) * n2 + ((n - 1) * n + tp)];
          if (gam == 0.0) continue;
          for (int cp = 0; cp < n; ++cp) Dg[(size_t)(0 * n + t) * n2 + (cp * n + tp)] -= gam * upp[cp];
        }
    }
    if (!invert(n2, Dg.data(), n2))
      throw std::runtime_error("singular element block in the strip factorization");
    std::memcpy(&cl.G[(size_t)e * n2 * n2], Dg.data(), sizeof(double) * n2 * n2);
  }
}

// Element inverses and the z-interface capacitance matrices of every class:
// A_j^-1 = D^-1 - D^-1 P K^-1 Lambda D^-1, K = I + Lambda D^-1 P.  The
// element operators are assembled on the host threads and inverted as one
// batch, then the capacitance matrices (which need D^-1) likewise; each batch
// goes to the device back end when it is large (invert_many).
static bool invert_many(const SetupOptions &opt, int n, const std::vector<double *> &mats);

// Returns the setup_device bit of the inverses that ran on the device back end
// (16) or 0; writes only the classes' Dinv and Kinv.
static int element_woodbury_all(System &s, const GLL &g, const SetupOptions &opt) {
  int dev = 0;
  const int n = s.n, n2 = s.n2, mz = s.mz;
  const int nq = 2 * n * (mz - 1);
  const int ncl = (int)s.classes.size();
  std::vector<double *> mats((size_t)ncl * mz);
  for (int c = 0; c < ncl; ++c) {
    s.classes[c].Dinv.assign((size_t)mz * n2 * n2, 0.0);
    for (int e = 0; e < mz; ++e) mats[(size_t)c * mz + e] = &s.classes[c].Dinv[(size_t)e * n2 * n2];
  }
  parallel_for(ncl * mz, opt.threads, [&](int q) {
    const int c = q / mz, e = q % mz;
    const StripClass &cl = s.classes[c];
    std::vector<double> Dg;
    element_diag_block(s, g, cl.hx, s.zb[e + 1] - s.zb[e], cl.west_if, cl.east_if, e > 0, e < mz - 1, Dg);
    std::memcpy(mats[q], Dg.data(), sizeof(double) * n2 * n2);
  });
  if (invert_many(opt, n2, mats)) dev = 16;
  for (StripClass &cl : s.classes) cl.Kinv.assign((size_t)nq * nq, 0.0);
  if (nq == 0) return dev;
  // column (interface i, part p, t): P puts a unit at element e_c, local l_c
  parallel_for(ncl, opt.threads, [&](int c) {
    StripClass &cl = s.classes[c];
    std::vector<double> &K = cl.Kinv;
    for (int a = 0; a < nq; ++a) K[(size_t)a * nq + a] = 1.0;
    for (int i = 0; i + 1 < mz; ++i)
      for (int p = 0; p < 2; ++p)
        for (int t = 0; t < n; ++t) {
          const int col = (2 * i + p) * n + t;
          const int ec = p == 0 ? i + 1 : i;
          const int lc = p == 0 ? t : (n - 1) * n + t;
          const double *Di = &cl.Dinv[(size_t)ec * n2 * n2];
          // rows reading element ec: lo of interface ec (reads element ec, i.e.
          // lo_{ec+1}) and up of interface ec-1 (reads element ec, up_{ec-1}).
          if (ec + 1 < mz) {
            const double *lo = &s.lo[(size_t)(ec + 1) * n];
            for (int tr = 0; tr < n; ++tr) {
              double acc = 0.0;
              for (int cc = 0; cc < n; ++cc) acc += lo[cc] * Di[(size_t)(cc * n + tr) * n2 + lc];
              K[(size_t)((2 * ec + 0) * n + tr) * nq + col] += acc;
            }
          }
          if (ec >= 1) {
            const double *up = &s.up[(size_t)(ec - 1) * n];
            for (int tr = 0; tr < n; ++tr) {
              double acc = 0.0;
              for (int cc = 0; cc < n; ++cc) acc += up[cc] * Di[(size_t)(cc * n + tr) * n2 + lc];
              K[(size_t)((2 * (ec - 1) + 1) * n + tr) * nq + col] += acc;
            }
          }
        }
  });
  std::vector<double *> kmats(ncl);
  for (int c = 0; c < ncl; ++c) kmats[c] = s.classes[c].Kinv.data();
  if (invert_many(opt, nq, kmats)) dev = 16;
  return dev;
}

void strip_solve_woodbury(const System &s, const StripClass &cl, double *x) {
  const int n = s.n, n2 = s.n2, mz = s.mz;
  const int nq = 2 * n * (mz - 1);
  std::vector<double> w((size_t)mz * n2, 0.0), lam(nq, 0.0), q(nq, 0.0);
  for (int e = 0; e < mz; ++e) {
    const double *Di = &cl.Dinv[(size_t)e * n2 * n2];
    for (int r = 0; r < n2; ++r) {
      double a = 0.0;
      for (int l = 0; l < n2; ++l) a += Di[(size_t)r * n2 + l] * x[(size_t)e * n2 + l];
      w[(size_t)e * n2 + r] = a;
    }
    for (int t = 0; t < n; ++t) {
      if (e + 1 < mz) {
        double a = 0.0;
        for (int c = 0; c < n; ++c) a += s.lo[(size_t)(e + 1) * n + c] * w[(size_t)e * n2 + c * n + t];
        lam[(size_t)(2 * e) * n + t] = a;
      }
      if (e >= 1) {
        double a = 0.0;
        for (int c = 0; c < n; ++c) a += s.up[(size_t)(e - 1) * n + c] * w[(size_t)e * n2 + c * n + t];
        lam[(size_t)(2 * (e - 1) + 1) * n + t] = a;
      }
    }
  }
  for (int a = 0; a < nq; ++a) {
    double acc = 0.0;
    for (int b = 0; b < nq; ++b) acc += cl.Kinv[(size_t)a * nq + b] * lam[b];
    q[a] = acc;
  }
  for (int e = 0; e < mz; ++e) {
    const double *Di = &cl.Dinv[(size_t)e * n2 * n2];
    for (int r = 0; r < n2; ++r) {
      double a = w[(size_t)e * n2 + r];
      for (int t = 0; t < n; ++t) {
        if (e >= 1) a -= Di[(size_t)r * n2 + t] * q[(size_t)(2 * (e - 1)) * n + t];
        if (e + 1 < mz) a -= Di[(size_t)r * n2 + (n - 1) * n + t] * q[(size_t)(2 * e + 1) * n + t];
      }
      x[(size_t)e * n2 + r] = a;
    }
  }
}

void strip_solve(const System &s, const StripClass &cl, double *X, int nrhs) {
  const int n = s.n, n2 = s.n2, mz = s.mz;
  std::vector<double> R((size_t)n2 * nrhs), q((size_t)n * nrhs);
  for (int e = 0; e < mz; ++e) {
    double *Xe = X + (size_t)e * n2 * nrhs;
    std::memcpy(R.data(), Xe, sizeof(double) * n2 * nrhs);
    if (e > 0) {
      const double *Wp = X + (size_t)(e - 1) * n2 * nrhs;   // w_{e-1}
      const double *lo = &s.lo[(size_t)e * n];
      for (int t = 0; t < n; ++t)
        for (int c = 0; c < n; ++c) {
          const double cf = lo[c];
          if (cf == 0.0) continue;
          const double *src = Wp + (size_t)(c * n + t) * nrhs;
          double *dst = &R[(size_t)(0 * n + t) * nrhs];
          for (int j = 0; j < nrhs; ++j) dst[j] -= cf * src[j];
        }
    }
    gemm(n2, nrhs, n2, 1.0, &cl.G[(size_t)e * n2 * n2], n2, R.data(), nrhs, 0.0, Xe, nrhs);
  }
  for (int e = mz - 2; e >= 0; --e) {
    const double *Xn = X + (size_t)(e + 1) * n2 * nrhs;
    const double *up = &s.up[(size_t)e * n];
    std::fill(q.begin(), q.end(), 0.0);
    for (int t = 0; t < n; ++t)
      for (int c = 0; c < n; ++c) {
        const double cf = up[c];
        if (cf == 0.0) continue;
        const double *src = Xn + (size_t)(c * n + t) * nrhs;
        for (int j = 0; j < nrhs; ++j) q[(size_t)t * nrhs + j] += cf * src[j];
      }
    // X_e -= G_e[:, (n-1, t)] q[t]
    const double *Ge = &cl.G[(size_t)e * n2 * n2];
    double *Xe = X + (size_t)e * n2 * nrhs;
    for (int row = 0; row < n2; ++row) {
      double *dst = Xe + (size_t)row * nrhs;
      for (int t = 0; t < n; ++t) {
        const double gv = Ge[(size_t)row * n2 + (n - 1) * n + t];
        if (gv == 0.0) continue;
        const double *src = &q[(size_t)t * nrhs];
        for (int j = 0; j < nrhs; ++j) dst[j] -= gv * src[j];
      }
    }
  }
}

void strip_solve_t(const System &s, const StripClass &cl, double *X, int nrhs) {
  // A = L D~ U with L_{e,e-1} = Lo_e G_{e-1}, U_{e,e+1} = G_e Up_e.
  // A^T x = v: U^T p = v, q = G^T p, L^T x = q.
  const int n = s.n, n2 = s.n2, mz = s.mz;
  std::vector<double> y((size_t)n2 * nrhs), P((size_t)mz * n2 * nrhs);
  for (int e = 0; e < mz; ++e) {
    double *Pe = &P[(size_t)e * n2 * nrhs];
    std::memcpy(Pe, X + (size_t)e * n2 * nrhs, sizeof(double) * n2 * nrhs);
    if (e > 0) {
      // y = G_{e-1}^T p_{e-1}; only rows (n-1, t) of y are needed.
      const double *Gp = &cl.G[(size_t)(e - 1) * n2 * n2];
      const double *Pp = &P[(size_t)(e - 1) * n2 * nrhs];
      const double *upp = &s.up[(size_t)(e - 1) * n];
      for (int t = 0; t < n; ++t) {
        const int rowy = (n - 1) * n + t;
        std::vector<double> acc(nrhs, 0.0);
        for (int l = 0; l < n2; ++l) {
          const double gv = Gp[(size_t)l * n2 + rowy];
          if (gv == 0.0) continue;
          for (int j = 0; j < nrhs; ++j) acc[j] += gv * Pp[(size_t)l * nrhs + j];
        }
        // (Up_{e-1}^T y)[(c, t)] = up_{e-1}[c] y[(n-1, t)]
        for (int c = 0; c < n; ++c)
          for (int j = 0; j < nrhs; ++j) Pe[(size_t)(c * n + t) * nrhs + j] -= upp[c] * acc[j];
      }
    }
  }
  // q_e = G_e^T p_e; then backward L^T.
  for (int e = mz - 1; e >= 0; --e) {
    const double *Ge = &cl.G[(size_t)e * n2 * n2];
    double *Pe = &P[(size_t)e * n2 * nrhs];
    if (e < mz - 1) {
      // p_e -= (Lo_{e+1}^T x_{e+1}) BEFORE applying G_e^T: x_e = G_e^T (p_e - Lo_{e+1}^T x_{e+1})
      // is equivalent to q_e - G_e^T Lo_{e+1}^T x_{e+1}.
      const double *Xn = X + (size_t)(e + 1) * n2 * nrhs;
      const double *lo = &s.lo[(size_t)(e + 1) * n];
      for (int t = 0; t < n; ++t)
        for (int c = 0; c < n; ++c)
          for (int j = 0; j < nrhs; ++j)
            Pe[(size_t)(c * n + t) * nrhs + j] -= lo[c] * Xn[(size_t)(0 * n + t) * nrhs + j];
    }
    // X_e = G_e^T Pe
    double *Xe = X + (size_t)e * n2 * nrhs;
    std::fill(y.begin(), y.end(), 0.0);
    for (int l = 0; l < n2; ++l) {
      const double *gl = Ge + (size_t)l * n2;
      const double *pl = Pe + (size_t)l * nrhs;
      for (int row = 0; row < n2; ++row) {
        const double gv = gl[row];
        if (gv == 0.0) continue;
        double *dst = &y[(size_t)row * nrhs];
        for (int j = 0; j < nrhs; ++j) dst[j] += gv * pl[j];
      }
    }
    std::memcpy(Xe, y.data(), sizeof(double) * n2 * nrhs);
  }
}

// W quarter blocks of one class from a 2N-right-hand-side strip solve.
static void class_schur_blocks(const System &s, StripClass &cl) {
  const int n = s.n, n2 = s.n2, mz = s.mz, N = s.N;
  const int nr = 2 * N;
  std::vector<double> X((size_t)mz * n2 * nr, 0.0);
  for (int e = 0; e < mz; ++e)
    for (int b = 0; b < n; ++b) {
      const int col = e * n + b;
      X[((size_t)e * n2 + b * n + 0) * nr + col] = 1.0;          // west injection
      X[((size_t)e * n2 + b * n + (n - 1)) * nr + N + col] = 1.0; // east injection
    }
  strip_solve(s, cl, X.data(), nr);
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) {
      const std::vector<double> &beta = r == 0 ? cl.betaW : cl.betaE;
      std::vector<double> &Wq = cl.Wq[r][c];
      Wq.assign((size_t)N * N, 0.0);
      for (int e = 0; e < mz; ++e)
        for (int b = 0; b < n; ++b) {
          double *dst = &Wq[(size_t)(e * n + b) * N];
          for (int a = 0; a < n; ++a) {
            const double *src = &X[((size_t)e * n2 + b * n + a) * nr + c * N];
            const double bv = beta[a];
            for (int q = 0; q < N; ++q) dst[q] += bv * src[q];
          }
        }
    }
}

// The Schur right-hand side operator of one strip class, B A_j^-1 (Sec. 2.3:
// b_S = B A^-1 F~, and B reads a strip only through the functionals of its
// west and east edge rows): the functionals' rows through A_j^-T, i.e.
// out[side][row][node] = (B A_j^-1)[row of that side][node], side 0 the
// west rows (read by the half west of the strip), 1 the east rows; row =
// e n + b, node the strip's local node index; 2 x N x (m_z n^2) row-major.
void class_rhs_blocks(const System &s, const StripClass &cl, std::vector<double> &out) {
  const int n = s.n, n2 = s.n2, mz = s.mz, N = s.N, K = mz * n2, nr = 2 * N;
  std::vector<double> X((size_t)K * nr, 0.0);
  for (int e = 0; e < mz; ++e)
    for (int b = 0; b < n; ++b)
      for (int c = 0; c < n; ++c) {
        const size_t node = (size_t)e * n2 + b * n + c;
        X[node * nr + e * n + b] = cl.betaW[c];
        X[node * nr + N + e * n + b] = cl.betaE[c];
      }
  strip_solve_t(s, cl, X.data(), nr);
  out.assign((size_t)2 * N * K, 0.0);
  for (size_t node = 0; node < (size_t)K; ++node)
    for (int q = 0; q < nr; ++q) out[(size_t)q * K + node] = X[node * nr + q];
}

// ---------------------------------------------------------------------------
void schur_apply_host(const System &s, const double *x, double *y) {
  const int N = s.N;
  for (int h = 0; h < s.nh; ++h) {
    const double *W = &s.Wblk[(size_t)s.w_id[h] * N * 2 * N];
    for (int i = 0; i < N; ++i) {
      double acc = x[(size_t)h * N + i];
      for (int c = 0; c < 2 * N; ++c) {
        const int64_t idx = (int64_t)s.w_win[h] * N + c;
        if (idx < 0 || idx >= s.kS) continue;
        acc += W[(size_t)i * 2 * N + c] * x[idx];
      }
      y[(size_t)h * N + i] = acc;
    }
  }
}

static double norm2(const std::vector<double> &v) {
  double s = 0.0;
  for (double a : v) s += a * a;
  return std::sqrt(s);
}

// Work per host thread from which the device back end is used: below it the
// transfers and the library start-up cost more than the host threads take
// (measured on the c2 and c3 grids).
constexpr double kDeviceWork = 2e10;
// Batches of inverses: from 5e9 flops per host thread on (the c3 block-Jacobi
// blocks, 128 of 832 x 832, take 0.30 s there against 0.60 s on 16 threads).
constexpr double kDeviceInvertWork = 5e9;
// Interfaces from which the u_S elimination goes to the device back end (its
// cyclic reduction is log2(d) levels of batched calls).
constexpr int kDeviceInterfaces = 16;

// In-place inverses of row-major n x n matrices: through the device back end
// when one is given and the work per host thread is large (2 n^3 per matrix;
// the host inverts matrices on separate threads), else on the host threads.
// Returns true when the device ran them.
static bool invert_many(const SetupOptions &opt, int n, const std::vector<double *> &mats) {
  if (mats.empty()) return false;
  const int threads = std::max(1, std::min<int>((int)mats.size(), opt.threads > 0 ? opt.threads : default_threads()));
  const double per_thread = 2.0 * (double)n * n * n * (double)mats.size() / threads;
  if (opt.dense && opt.dense->invert && (per_thread >= kDeviceInvertWork || opt.dense->always)) {
    opt.dense->invert(n, (int)mats.size(), mats.data());
    return true;
  }
  parallel_for((int)mats.size(), opt.threads, [&](int q) {
    if (!invert(n, mats[q], n)) throw std::domain_error("singular matrix in the setup");
  });
  return false;
}

// Left null vector of S (k = 0) by shifted inverse iteration on S^T - sigma I
// (Sec. 2.4).  S is block tridiagonal over interfaces (2N x 2N blocks); the
// shifted transpose T is factored by block elimination, the diagonal blocks
// with partial pivoting, on the host or through opt.dense.
// Returns 1 when the elimination ran on the device back end, else 0.
static int left_null_schur(const System &s, const SetupOptions &opt, std::vector<double> &uS) {
  const DenseBackend *be = opt.dense_null ? opt.dense_null : opt.dense;
  int dev = 0;
  const int N = s.N, M = 2 * N, d = s.mx - 1;   // d: interfaces
  // Interface blocks of S: Sd[i] (M x M), Su[i] = S[i][i+1] (upper-left N x N
  // of rows of half 2i, cols of half 2i+2), Sl[i] = S[i][i-1] (rows of half
  // 2i+1, cols of half 2i-1).
  auto Wpart = [&](int h, int p, int i, int c) -> double {
    return s.Wblk[(size_t)s.w_id[h] * N * 2 * N + (size_t)i * 2 * N + p * N + c];
  };
  double snorm = 0.0;
  for (int h = 0; h < s.nh; ++h)
    for (int i = 0; i < N; ++i) {
      double rs = 1.0;
      for (int c = 0; c < 2 * N; ++c) rs += std::fabs(Wpart(h, 0, i, c));
      snorm = std::max(snorm, rs);
    }
  const double sigma = 1e-10 * snorm;
  // T = S^T - sigma I; blocks: Td[i] = Sd[i]^T - sigma, T[i][i+1] = Sl[i+1]^T
  // (nonzero at rows N..2N, cols N..2N: Up[i]), T[i][i-1] = Su[i-1]^T (rows
  // 0..N, cols 0..N: Lo[i]).
  std::vector<double> Td((size_t)d * M * M, 0.0), Lo((size_t)d * N * N, 0.0), Up((size_t)d * N * N, 0.0);
  for (int i = 0; i < d; ++i) {
    double *T = &Td[(size_t)i * M * M];
    // Sd[i] rows 0..N (half 2i): cols N..2N (half 2i+1) = W^_{2i} part 0.
    // rows N..2N (half 2i+1): cols 0..N (half 2i) = W^_{2i+1} part 1.
    for (int a = 0; a < M; ++a) T[(size_t)a * M + a] = 1.0 - sigma;
    for (int r = 0; r < N; ++r)
      for (int c = 0; c < N; ++c) {
        // T = Sd^T: T[col][row] = Sd[row][col]
        T[(size_t)(N + c) * M + r] += Wpart(2 * i, 0, r, c);
        T[(size_t)c * M + (N + r)] += Wpart(2 * i + 1, 1, r, c);
      }
    // Su[i-1] has rows of half 2i-2 and cols of half 2i = W^_{2i-2} part 1.
    if (i > 0)
      for (int r = 0; r < N; ++r)
        for (int c = 0; c < N; ++c) Lo[(size_t)i * N * N + (size_t)c * N + r] = Wpart(2 * i - 2, 1, r, c);
    // Sl[i+1] rows of half 2i+3, cols of half 2i+1 = W^_{2i+3} part 0.
    if (i + 1 < d)
      for (int r = 0; r < N; ++r)
        for (int c = 0; c < N; ++c) Up[(size_t)i * N * N + (size_t)c * N + r] = Wpart(2 * i + 3, 0, r, c);
  }
  std::function<void(std::vector<double> &)> solve;
  void *dev_fact = nullptr;
  std::vector<int> piv;
  std::vector<double> X;
  // On the host the elimination is sequential over the interfaces (one
  // thread); the device back end reduces the interfaces cyclically, log2(d)
  // levels of batched calls, and takes every system of 16 interfaces or more.
  if (be && be->tri_factor && (d >= kDeviceInterfaces || be->always)) {
    dev_fact = be->tri_factor(d, N, Td.data(), Lo.data(), Up.data());
    dev = 1;
    solve = [&](std::vector<double> &v) { be->tri_solve(dev_fact, v.data()); };
  } else {
    // Block elimination: T~_i = Td[i] - T[i][i-1] X_{i-1}, X_i = T~_i^-1 T[i][i+1]
    // (X_i: the M x N nonzero columns N..2N).
    piv.assign((size_t)d * M, 0);
    X.assign((size_t)d * M * N, 0.0);
    for (int i = 0; i < d; ++i) {
      double *T = &Td[(size_t)i * M * M];
      if (i > 0)   // T~[0..N][N..2N] -= Lo[i] X_{i-1}[0..N][0..N]
        gemm(N, N, N, -1.0, &Lo[(size_t)i * N * N], N, &X[(size_t)(i - 1) * M * N], N, 1.0, T + N, M);
      if (!getrf(M, T, M, &piv[(size_t)i * M]))
        throw std::runtime_error("singular block in the inverse iteration for u_S");
      if (i + 1 < d) {
        double *B = &X[(size_t)i * M * N];
        for (int r = 0; r < N; ++r)
          std::memcpy(B + (size_t)(N + r) * N, &Up[(size_t)i * N * N + (size_t)r * N], sizeof(double) * N);
        getrs(M, N, T, M, &piv[(size_t)i * M], B, N);
      }
    }
    solve = [&](std::vector<double> &v) {
      // forward: y_i = v_i - T[i][i-1] T~_{i-1}^-1 y_{i-1}
      std::vector<double> tmp(M);
      for (int i = 1; i < d; ++i) {
        std::memcpy(tmp.data(), &v[(size_t)(i - 1) * M], sizeof(double) * M);
        getrs(M, 1, &Td[(size_t)(i - 1) * M * M], M, &piv[(size_t)(i - 1) * M], tmp.data(), 1);
        const double *L = &Lo[(size_t)i * N * N];
        for (int r = 0; r < N; ++r) {
          double acc = 0.0;
          for (int c = 0; c < N; ++c) acc += L[(size_t)r * N + c] * tmp[c];
          v[(size_t)i * M + r] -= acc;
        }
      }
      // backward: x_i = T~_i^-1 y_i - X_i x_{i+1}[N..2N]
      for (int i = d - 1; i >= 0; --i) {
        double *vi = &v[(size_t)i * M];
        getrs(M, 1, &Td[(size_t)i * M * M], M, &piv[(size_t)i * M], vi, 1);
        if (i + 1 < d) {
          const double *xn = &v[(size_t)(i + 1) * M + N];
          const double *Xi = &X[(size_t)i * M * N];
          for (int r = 0; r < M; ++r) {
            double acc = 0.0;
            for (int c = 0; c < N; ++c) acc += Xi[(size_t)r * N + c] * xn[c];
            vi[r] -= acc;
          }
        }
      }
    };
  }
  std::vector<double> u(s.kS, 1.0 / std::sqrt((double)s.kS));
  std::vector<double> Stu(s.kS);
  try {
    for (int it = 0; it < 6; ++it) {
      solve(u);
      const double nu = norm2(u);
      if (!(nu > 0.0) || !std::isfinite(nu)) throw std::runtime_error("inverse iteration for u_S failed");
      for (auto &a : u) a /= nu;
      // residual ||S^T u|| / ||S||
      std::fill(Stu.begin(), Stu.end(), 0.0);
      for (int h = 0; h < s.nh; ++h)
        for (int i = 0; i < N; ++i) {
          const double ui = u[(size_t)h * N + i];
          Stu[(size_t)h * N + i] += ui;
          for (int c = 0; c < 2 * N; ++c) {
            const int64_t idx = (int64_t)s.w_win[h] * N + c;
            if (idx < 0 || idx >= s.kS) continue;
            Stu[idx] += Wpart(h, 0, i, c) * ui;
          }
        }
      if (norm2(Stu) <= 1e-13 * snorm && it >= 1) break;
    }
  } catch (...) {
    if (dev_fact) be->tri_free(dev_fact);
    throw;
  }
  if (dev_fact) be->tri_free(dev_fact);
  double sum = 0.0;
  for (double a : u) sum += a;
  if (sum < 0) for (auto &a : u) a = -a;
  uS = std::move(u);
  return dev;
}

// S M^-1 per half (shared-block grids): F_h = E_h M^-1 + W_h [M^-1 rows of the
// window halves w, w + 1], over the contiguous column range of the block-Jacobi
// blocks of h, w and w + 1.  Identical (W, M, offsets) combinations share one
// stored block.
static void build_fused(System &s, const SetupOptions &opt) {
  s.f_id.assign(s.nh, -1); s.f_win.assign(s.nh, 0); s.f_K.assign(s.nh, 0);
  s.Fblk.clear(); s.nF = 0;
  if (s.nW >= s.nh) return;   // no shared blocks: the two-step apply streams W and M
  const int N = s.N, nh = s.nh, F8 = 8 * N;
  std::map<std::vector<int>, int> fmap;
  std::vector<int> first;
  for (int h = 0; h < nh; ++h) {
    const int w0 = s.w_win[h];
    int blo = h / 4, bhi = h / 4;
    for (int p = 0; p < 2; ++p) {
      const int wh = w0 + p;
      if (wh < 0 || wh >= nh) continue;
      blo = std::min(blo, wh / 4); bhi = std::max(bhi, wh / 4);
    }
    const int start = 4 * blo, end = std::min(nh, 4 * (bhi + 1));
    s.f_win[h] = start;
    s.f_K[h] = (end - start) * N;
    std::vector<int> key = {s.f_K[h], s.w_id[h], s.m_id[h], s.m_win[h] - start};
    for (int p = 0; p < 2; ++p) {
      const int wh = w0 + p;
      if (wh < 0 || wh >= nh) { key.push_back(-1); key.push_back(0); continue; }
      key.push_back(s.m_id[wh]); key.push_back(s.m_win[wh] - start);
    }
    auto it = fmap.find(key);
    if (it == fmap.end()) { it = fmap.emplace(key, (int)first.size()).first; first.push_back(h); }
    s.f_id[h] = it->second;
  }
  s.nF = (int)first.size();
  s.Fblk.assign((size_t)s.nF * N * F8, 0.0);
  parallel_for(s.nF, opt.threads, [&](int u) {
    const int h = first[u], start = s.f_win[h];
    double *F = &s.Fblk[(size_t)u * N * F8];
    // E_h M^-1: the half's own row chunk of M^-1
    const double *Mh = &s.Mblk[(size_t)s.m_id[h] * N * 4 * N];
    const int oh = (s.m_win[h] - start) * N;
    for (int i = 0; i < N; ++i)
      for (int c = 0; c < s.m_K[h]; ++c) F[(size_t)i * F8 + oh + c] += Mh[(size_t)i * 4 * N + c];
    // W_h [M^-1 rows of the window halves]
    const double *W = &s.Wblk[(size_t)s.w_id[h] * N * 2 * N];
    for (int p = 0; p < 2; ++p) {
      const int wh = s.w_win[h] + p;
      if (wh < 0 || wh >= s.nh) continue;
      const double *Mw = &s.Mblk[(size_t)s.m_id[wh] * N * 4 * N];
      const int ow = (s.m_win[wh] - start) * N;
      gemm(N, s.m_K[wh], N, 1.0, W + p * N, 2 * N, Mw, 4 * N, 1.0, F + ow, F8);
    }
  });
}

// With SMPM_SETUP_TIMES set in the environment, each step of build_system
// prints its wall time to stderr (for measurement; the tables are the same).
namespace {
struct StepTimer {
  bool on = std::getenv("SMPM_SETUP_TIMES") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void lap(const char *what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "setup %-28s %8.1f ms\n", what, std::chrono::duration<double, std::milli>(now - t).count());
    t = now;
  }
};
}  // namespace

void build_system(System &s, int mx, int mz, int order, const double *xb, const double *zb,
                  double kwave, const SetupOptions &opt) {
  StepTimer timer;
  if (mx < 2 || mz < 1 || order < 1) throw std::invalid_argument("need mx >= 2, mz >= 1, order >= 1");
  if (!(kwave >= 0.0) || !std::isfinite(kwave)) throw std::invalid_argument("wavenumber must be finite and >= 0");
  s.n = order + 1; s.mx = mx; s.mz = mz;
  if (opt.zlabel != 0 && opt.zlabel != 1) throw std::invalid_argument("zlabel must be 0 or 1");
  s.zm = opt.zlabel == 1 ? mz : 1;
  s.n2 = s.n * s.n; s.N = s.n * mz; s.nh = 2 * (mx - 1); s.d = (mx - 1) * s.zm;
  s.r = (int64_t)s.n2 * mx * mz; s.kS = (int64_t)s.N * s.nh;
  s.kwave = kwave; s.singular = (kwave == 0.0);
  s.xb.assign(xb, xb + mx + 1); s.zb.assign(zb, zb + mz + 1);
  double hmin = 1e300;
  for (int j = 0; j < mx; ++j) {
    const double h = s.xb[j + 1] - s.xb[j];
    if (!(h > 0.0) || !std::isfinite(h)) throw std::invalid_argument("x breakpoints must be finite and increasing");
    hmin = std::min(hmin, h);
  }
  for (int e = 0; e < mz; ++e) {
    const double h = s.zb[e + 1] - s.zb[e];
    if (!(h > 0.0) || !std::isfinite(h)) throw std::invalid_argument("z breakpoints must be finite and increasing");
    hmin = std::min(hmin, h);
  }
  if (s.singular && mx < 4)
    throw std::domain_error("k = 0 needs m_x >= 4 (a block-Jacobi block would be all of the singular S)");
  const int n = s.n, N = s.N;
  s.tau = opt.tau != 0.0 ? opt.tau : -(double)n * (n - 1) / hmin;
  const GLL g = make_gll(n);
  const double *D = g.D.data();
  const double tau = s.tau;
  // z couplings inside a strip
  s.lo.assign((size_t)mz * n, 0.0);
  s.up.assign((size_t)mz * n, 0.0);
  for (int e = 0; e < mz; ++e) {
    if (e > 0) {
      const double hzp = s.zb[e] - s.zb[e - 1];
      for (int c = 0; c < n; ++c)
        s.lo[(size_t)e * n + c] = (c == n - 1 ? -tau : 0.0) + tau * (2.0 / hzp) * D[(size_t)(n - 1) * n + c];
    }
    if (e < mz - 1) {
      const double hzn = s.zb[e + 2] - s.zb[e + 1];
      for (int c = 0; c < n; ++c)
        s.up[(size_t)e * n + c] = (c == 0 ? -tau : 0.0) - tau * (2.0 / hzn) * D[c];
    }
  }
  // strip classes: equal width (to 1e-13 relative) and equal boundary type
  s.strip_class.assign(mx, -1);
  for (int j = 0; j < mx; ++j) {
    const double hx = s.xb[j + 1] - s.xb[j];
    const bool wif = j > 0, eif = j < mx - 1;
    int found = -1;
    for (int c = 0; c < (int)s.classes.size(); ++c) {
      const StripClass &cl = s.classes[c];
      if (cl.west_if == wif && cl.east_if == eif && std::fabs(cl.hx - hx) <= 1e-13 * hx) { found = c; break; }
    }
    if (found < 0) {
      StripClass cl;
      cl.hx = hx; cl.west_if = wif; cl.east_if = eif;
      cl.betaW.resize(n); cl.betaE.resize(n);
      for (int c = 0; c < n; ++c) {
        cl.betaW[c] = (c == 0 ? -tau : 0.0) - tau * (2.0 / hx) * D[c];
        cl.betaE[c] = (c == n - 1 ? -tau : 0.0) + tau * (2.0 / hx) * D[(size_t)(n - 1) * n + c];
      }
      s.classes.push_back(cl);
      found = (int)s.classes.size() - 1;
    }
    s.strip_class[j] = found;
  }
  // The W blocks' strip solves (2 n2^2 2N flops per element and class) go
  // to the device back end from a quarter of the usual work per host thread:
  // they are GEMMs with little to transfer back.
  const int ncl = (int)s.classes.size();
  const int wthreads = std::max(1, std::min(ncl, opt.threads > 0 ? opt.threads : default_threads()));
  const double wwork = 4.0 * mz * (double)s.n2 * s.n2 * N * ncl / wthreads;
  const bool dev_w = opt.dense && opt.dense->strip_schur && (opt.dense->always || wwork >= 0.25 * kDeviceWork);
  parallel_for(ncl, opt.threads, [&](int c) {
    factor_class(s, g, s.classes[c]);
    if (!dev_w) class_schur_blocks(s, s.classes[c]);
  });
  timer.lap(dev_w ? "strip factorizations" : "strip factorizations, W");
  // The element and capacitance inverses (Dinv, Kinv) serve the interior
  // elimination of the solve only: with the host threads to itself, the
  // setup runs them on a task of their own beside the W blocks' device
  // solves and the block-Jacobi step, and joins it at the end.  The task
  // writes only the classes' Dinv and Kinv, which nothing below reads.
  std::future<int> elem_task;
  SetupOptions eopt = opt;   // half the host threads: the rest drive the device steps and their copies
  eopt.threads = std::max(1, (opt.threads > 0 ? opt.threads : default_threads()) / 2);
  if (opt.threads != 1) {
    elem_task = std::async(std::launch::async, [&s, &g, &eopt] { return element_woodbury_all(s, g, eopt); });
  } else {
    s.dev_steps |= element_woodbury_all(s, g, opt);
    timer.lap("element inverses");
  }
  if (dev_w) {
    std::vector<const double *> Gp(ncl), bw(ncl), be(ncl);
    std::vector<double *> Wp(4 * ncl);
    for (int c = 0; c < ncl; ++c) {
      StripClass &cl = s.classes[c];
      Gp[c] = cl.G.data(); bw[c] = cl.betaW.data(); be[c] = cl.betaE.data();
      for (int r = 0; r < 2; ++r)
        for (int q = 0; q < 2; ++q) {
          cl.Wq[r][q].assign((size_t)N * N, 0.0);
          Wp[4 * c + 2 * r + q] = cl.Wq[r][q].data();
        }
    }
    opt.dense->strip_schur(ncl, n, mz, Gp.data(), s.lo.data(), s.up.data(), bw.data(), be.data(), Wp.data());
    s.dev_steps |= 8;
    timer.lap("W strip solves (device)");
  }
  // Schur blocks per output half, deduplicated by (strip class, row side).
  s.w_id.assign(s.nh, -1); s.w_win.assign(s.nh, 0);
  std::map<std::pair<int, int>, int> wmap;
  std::vector<std::pair<int, int>> wkeys;
  for (int h = 0; h < s.nh; ++h) {
    const int i = h / 2;
    const bool even = (h % 2 == 0);
    const int strip = even ? i + 1 : i;
    const int rside = even ? 0 : 1;
    s.w_win[h] = even ? h + 1 : h - 2;
    const auto key = std::make_pair(s.strip_class[strip], rside);
    auto it = wmap.find(key);
    if (it == wmap.end()) {
      it = wmap.emplace(key, (int)wkeys.size()).first;
      wkeys.push_back(key);
    }
    s.w_id[h] = it->second;
  }
  s.nW = (int)wkeys.size();
  s.Wblk.assign((size_t)s.nW * N * 2 * N, 0.0);
  for (int b = 0; b < s.nW; ++b) {
    const StripClass &cl = s.classes[wkeys[b].first];
    const int rs = wkeys[b].second;
    for (int c = 0; c < 2; ++c) {
      const bool exists = (c == 0 ? cl.west_if : cl.east_if) && (rs == 0 ? cl.west_if : cl.east_if);
      if (!exists) continue;
      const std::vector<double> &Wq = cl.Wq[rs][c];
      for (int i = 0; i < N; ++i)
        std::memcpy(&s.Wblk[(size_t)b * N * 2 * N + (size_t)i * 2 * N + c * N], &Wq[(size_t)i * N], sizeof(double) * N);
    }
  }
  // The left null vector of S (k = 0) needs only the Schur blocks, and its
  // elimination is one sequential chain over the interfaces: it runs on a
  // thread of its own (with its own device back end) beside the
  // block-Jacobi, S M^-1 and coarse steps, which read none of its output.
  std::vector<double> uS_out;
  std::future<int> us_task;
  if (s.singular) {
    const System &cs = s;
    us_task = std::async(std::launch::async, [&cs, &opt, &uS_out] { return left_null_schur(cs, opt, uS_out); });
  }
  // Block-Jacobi: blocks over interfaces (2b, 2b+1), deduplicated.
  s.m_id.assign(s.nh, -1); s.m_win.assign(s.nh, 0); s.m_K.assign(s.nh, 0);
  const int nblocks = s.mx / 2;   // pairs of the m_x - 1 interfaces
  s.nMblocks = nblocks;
  std::map<std::vector<int>, int> mmap;
  std::vector<int> mfirst;   // representative block of each unique M
  std::vector<int> mblock_uid(nblocks);
  for (int b = 0; b < nblocks; ++b) {
    const int h0 = 4 * b;
    const int nhb = std::min(4, s.nh - h0);
    std::vector<int> key = {nhb};
    for (int q = 0; q < nhb; ++q) { key.push_back(s.w_id[h0 + q]); key.push_back(s.w_win[h0 + q] - h0); }
    auto it = mmap.find(key);
    if (it == mmap.end()) { it = mmap.emplace(key, (int)mfirst.size()).first; mfirst.push_back(b); }
    mblock_uid[b] = it->second;
  }
  const int nMu = (int)mfirst.size();
  // A full block (4 halves, K = 4N) is assembled and inverted in place in
  // Mblk, whose four N x 4N chunks of unique block u are that block's K x K
  // row-major matrix; a narrower last block goes through a buffer.
  s.nM = nMu * 4;
  s.Mblk.assign((size_t)s.nM * N * 4 * N, 0.0);
  std::vector<std::vector<double>> narrow(nMu);
  std::vector<double *> Mptr(nMu);
  parallel_for(nMu, opt.threads, [&](int u) {   // assemble; inverted below
    const int b = mfirst[u];
    const int h0 = 4 * b;
    const int nhb = std::min(4, s.nh - h0);
    const int K = nhb * N;
    double *Mb = &s.Mblk[(size_t)u * 16 * N * N];
    if (nhb < 4) {
      narrow[u].assign((size_t)K * K, 0.0);
      Mb = narrow[u].data();
    }
    for (int a = 0; a < K; ++a) Mb[(size_t)a * K + a] = 1.0;
    for (int q = 0; q < nhb; ++q) {
      const int h = h0 + q;
      const double *W = &s.Wblk[(size_t)s.w_id[h] * N * 2 * N];
      for (int p = 0; p < 2; ++p) {
        const int wh = s.w_win[h] + p;
        if (wh < h0 || wh >= h0 + nhb) continue;
        const int lc = wh - h0;
        for (int i = 0; i < N; ++i)
          for (int c = 0; c < N; ++c) Mb[(size_t)(q * N + i) * K + lc * N + c] += W[(size_t)i * 2 * N + p * N + c];
      }
    }
    Mptr[u] = Mb;
  });
  {
    std::map<int, std::vector<double *>> byK;   // the last block may be narrower
    for (int u = 0; u < nMu; ++u) {
      const int K = std::min(4, s.nh - 4 * mfirst[u]) * N;
      byK[K].push_back(Mptr[u]);
    }
    try {
      for (auto &kv : byK)
        if (invert_many(opt, kv.first, kv.second)) s.dev_steps |= 2;
    } catch (const std::domain_error &) {
      throw std::domain_error("singular block-Jacobi block");
    }
  }
  for (int u = 0; u < nMu; ++u) {
    if (narrow[u].empty()) continue;
    const int nhb = std::min(4, s.nh - 4 * mfirst[u]);
    const int K = nhb * N;
    for (int q = 0; q < nhb; ++q)
      for (int i = 0; i < N; ++i)
        std::memcpy(&s.Mblk[((size_t)(u * 4 + q) * N + i) * 4 * N], &narrow[u][(size_t)(q * N + i) * K],
                    sizeof(double) * K);
  }
  for (int b = 0; b < nblocks; ++b) {
    const int h0 = 4 * b;
    const int nhb = std::min(4, s.nh - h0);
    for (int q = 0; q < nhb; ++q) {
      s.m_id[h0 + q] = mblock_uid[b] * 4 + q;
      s.m_win[h0 + q] = h0;
      s.m_K[h0 + q] = nhb * N;
    }
  }
  timer.lap("block-Jacobi");
  build_fused(s, opt);
  timer.lap("S M^-1 blocks");
  // Deflation tables: S Z per half (two coarse columns), C = Z^T S Z.
  // Z column (interface a, segment e) is the indicator of rows e*seg .. (e+1)*seg-1
  // of both halves of interface a (seg = N / zm).  Half h's window is halves
  // (w, w+1) of interfaces (ca, cb); its own half belongs to ca (even h) or cb.
  const int zm = s.zm, seg = N / zm, nif = mx - 1;
  s.sz_col.assign((size_t)s.nh * 2 * zm, -1);
  s.SZh.assign((size_t)s.nh * 2 * zm * N, 0.0);
  s.C.assign((size_t)s.d * s.d, 0.0);
  for (int h = 0; h < s.nh; ++h) {
    const int i = h / 2;
    const bool even = (h % 2 == 0);
    const int ca = even ? i : i - 1, cb = even ? i + 1 : i;
    const double *W = &s.Wblk[(size_t)s.w_id[h] * N * 2 * N];
    for (int p = 0; p < 2; ++p) {
      const int iface = p == 0 ? ca : cb;
      if (iface < 0 || iface >= nif) continue;
      const bool own = (p == 0 && even) || (p == 1 && !even);
      for (int e = 0; e < zm; ++e) {
        const int col = iface * zm + e;
        s.sz_col[((size_t)h * 2 + p) * zm + e] = col;
        double *sz = &s.SZh[(((size_t)h * 2 + p) * zm + e) * N];
        for (int r = 0; r < N; ++r) {
          double rs = 0.0;
          for (int c = e * seg; c < (e + 1) * seg; ++c) rs += W[(size_t)r * 2 * N + p * N + c];
          if (own && r / seg == e) rs += 1.0;
          sz[r] = rs;
          s.C[(size_t)(i * zm + r / seg) * s.d + col] += rs;
        }
      }
    }
  }
  // Coarse operator.
  const int d = s.d;
  s.Gc.assign((size_t)d * d, 0.0);
  if (!s.singular) {
    std::vector<double> Ci = s.C;
    try {
      if (invert_many(opt, d, {Ci.data()})) s.dev_steps |= 4;
    } catch (const std::domain_error &) {
      throw std::domain_error("singular coarse matrix C(k)");
    }
    s.Gc = Ci;
  } else {
    // u_C: C^T u = 0 with u_{d-1} = 1 (the leading (d-1) block C_m is
    // invertible): u_m = C_m^-T b with b = -(row d-1 of C)[0..m).
    const int m = d - 1;
    std::vector<double> Cinv((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) Cinv[(size_t)i * m + j] = s.C[(size_t)i * d + j];
    try {
      if (invert_many(opt, m, {Cinv.data()})) s.dev_steps |= 4;
    } catch (const std::domain_error &) {
      throw std::domain_error("singular leading block of C");
    }
    std::vector<double> uC(d, 1.0);
    for (int i = 0; i < m; ++i) {
      double acc = 0.0;
      for (int k = 0; k < m; ++k) acc += Cinv[(size_t)k * m + i] * -s.C[(size_t)(d - 1) * d + k];
      uC[i] = acc;
    }
    const double nu = norm2(uC);
    double sum = 0.0;
    for (auto &a : uC) { a /= nu; sum += a; }
    if (sum < 0) for (auto &a : uC) a = -a;
    s.uC = uC;
    // G = M^-1 (I - u_C u_C^T) with M = P_u C P_v + alpha u_C v^T, where
    // P_u = I - u_C u_C^T, P_v = I - v v^T and v = 1_d / sqrt(d) is C's right
    // null vector (Z 1_d = 1_Gamma, S 1_Gamma = 0).  M maps v-perp as the
    // projected C does and v to alpha u_C, so it is nonsingular, and
    // G C x = x - v (v . x) for the projected C: the coarse correction takes
    // out every direction of S Z except the constant, to the rounding of C.
    // (Pinning one coarse unknown and inverting the leading block instead
    // leaves C's smallest singular value times |C_m^-1| in a whole column of
    // G C; on a 64 x 10, order-9 grid that doubled the DBJ iterations.)
    // Any solution of the consistent coarse system serves: P does not
    // change under a shift along v.
    {
      const double sv = 1.0 / std::sqrt((double)d);
      std::vector<double> ut(d, 0.0), cv(d, 0.0);   // u_C^T C and C v
      double alpha = 0.0;
      for (int i = 0; i < d; ++i) {
        const double *ci = &s.C[(size_t)i * d];
        double a = 0.0;
        for (int j = 0; j < d; ++j) {
          ut[j] += uC[i] * ci[j];
          a += ci[j];
        }
        cv[i] = a * sv;
        alpha = std::max(alpha, std::fabs(ci[i]));
      }
      double ucv = 0.0;
      for (int i = 0; i < d; ++i) ucv += uC[i] * cv[i];
      if (!(alpha > 0.0)) throw std::domain_error("zero coarse matrix C");
      std::vector<double> Mi((size_t)d * d);
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
          Mi[(size_t)i * d + j] = s.C[(size_t)i * d + j] - uC[i] * ut[j] - cv[i] * sv + uC[i] * ucv * sv +
                                  alpha * uC[i] * sv;
      try {
        if (invert_many(opt, d, {Mi.data()})) s.dev_steps |= 4;
      } catch (const std::domain_error &) {
        throw std::domain_error("singular completed coarse matrix");
      }
      for (int i = 0; i < d; ++i) {   // G = M^-1 - (M^-1 u_C) u_C^T
        const double *mi = &Mi[(size_t)i * d];
        double w = 0.0;
        for (int l = 0; l < d; ++l) w += mi[l] * uC[l];
        for (int j = 0; j < d; ++j) s.Gc[(size_t)i * d + j] = mi[j] - w * uC[j];
      }
    }
    timer.lap("deflation, coarse");
    // Null vectors of S and L.
    if (us_task.get()) s.dev_steps |= 1;
    s.uS = std::move(uS_out);
    timer.lap("u_S (the wait for it)");
    // u_L = A^-T B^T u_S (Claim 1, part 2)
    std::vector<double> uL(s.r, 0.0);
    const int n2 = s.n2;
    for (int j = 0; j < mx; ++j) {
      const StripClass &cl = s.classes[s.strip_class[j]];
      double *v = &uL[(size_t)j * mz * n2];
      for (int e = 0; e < mz; ++e)
        for (int b = 0; b < n; ++b) {
          const int row = e * n + b;
          if (j >= 1) {   // west row read by Gamma_{j-1}^L (half 2j - 2)
            const double us = s.uS[(size_t)(2 * j - 2) * N + row];
            for (int c = 0; c < n; ++c) v[(size_t)e * n2 + b * n + c] += cl.betaW[c] * us;
          }
          if (j <= mx - 2) {   // east row read by Gamma_j^R (half 2j + 1)
            const double us = s.uS[(size_t)(2 * j + 1) * N + row];
            for (int c = 0; c < n; ++c) v[(size_t)e * n2 + b * n + c] += cl.betaE[c] * us;
          }
        }
    }
    parallel_for(mx, opt.threads, [&](int j) {
      strip_solve_t(s, s.classes[s.strip_class[j]], &uL[(size_t)j * mz * n2], 1);
    });
    const double nl = norm2(uL);
    double sl = 0.0;
    for (auto &a : uL) { a /= nl; sl += a; }
    if (sl < 0) for (auto &a : uL) a = -a;
    s.uL = uL;
    timer.lap("u_L");
  }
  if (elem_task.valid()) {
    s.dev_steps |= elem_task.get();
    timer.lap("element inverses (the wait)");
  }
}

}  // namespace smpm
