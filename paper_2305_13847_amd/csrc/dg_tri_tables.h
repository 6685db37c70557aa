// Host-side reference tables of the triangle kernels: the Gauss-Legendre
// rules, the Dubiner basis with its gradient, the Duffy-mapped volume rule and
// the face points (Section 3.1 space, footnote of Section 3.4).  Plain C++,
// no device calls.
#pragma once
#include <cmath>
#include <cstring>

#include "dg_tri_dev.h"

namespace dgm {

// ---------------------------------------------------------------------------
// reference tables
// ---------------------------------------------------------------------------
// Gauss-Legendre rule of n points on [-1, 1], ascending: Newton on P_n from
// cos(pi (4i + 3) / (4n + 2)), P_n' from (x^2 - 1) P_n' = n (x P_n - P_{n-1}).
inline void gl_rule(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (4.0 * i + 3.0) / (4.0 * n + 2.0));
    double pn = 0.0, dpn = 1.0;
    for (int it = 0; it < 100; ++it) {
      double pm1 = 1.0;
      pn = t;
      for (int m = 2; m <= n; ++m) {
        const double pn1 = ((2.0 * m - 1.0) * t * pn - (m - 1.0) * pm1) / m;
        pm1 = pn;
        pn = pn1;
      }
      if (n == 1) pm1 = 1.0;
      dpn = n * (t * pn - pm1) / (t * t - 1.0);
      const double step = pn / dpn;
      t -= step;
      if (std::fabs(step) <= 1e-16) break;
    }
    // value and derivative at the converged point
    double pm1 = 1.0;
    pn = t;
    for (int m = 2; m <= n; ++m) {
      const double pn1 = ((2.0 * m - 1.0) * t * pn - (m - 1.0) * pm1) / m;
      pm1 = pn;
      pn = pn1;
    }
    dpn = n * (t * pn - pm1) / (t * t - 1.0);
    x[n - 1 - i] = t;
    w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dpn * dpn);
  }
}

// Jacobi polynomial P_n^{(al,be)}(y)
inline double jacobi(int n, double al, double be, double y) {
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = 0.5 * (al - be + (al + be + 2.0) * y);
  for (int k = 2; k <= n; ++k) {
    const double s = 2.0 * k + al + be;
    const double p2 = ((s - 1.0) * ((al * al - be * be) + s * (s - 2.0) * y) * p1
                       - 2.0 * (k + al - 1.0) * (k + be - 1.0) * s * p0)
                      / (2.0 * k * (k + al + be) * (s - 2.0));
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// Dubiner basis at (r, s) with its reference gradient:
//   psi_pq = N_pq L_p(r, s) J_q(2s - 1),  L_p = t^p P_p((2r - t)/t), t = 1 - s,
//   J_q = P_q^{(2p+1,0)}, N_pq^2 = 2 (2p+1)(p+q+1).
// L_p follows Bonnet's recurrence multiplied through by t^(p+1), with
// X = 2r - t: L_{p+1} = ((2p+1) X L_p - p t^2 L_{p-1}) / (p+1); its
// derivatives follow by differentiating that recurrence (dX/dr = 2,
// dX/ds = 1, dt/ds = -1).  J_q' = (q + 2p + 2)/2 P_{q-1}^{(2p+2,1)}.
inline void dubiner(int k, double r, double s, double* psi, double* dr, double* ds) {
  const double t = 1.0 - s, X = 2.0 * r - t;
  double L[16], Lr[16], Ls[16];
  L[0] = 1.0; Lr[0] = 0.0; Ls[0] = 0.0;
  if (k >= 1) { L[1] = X; Lr[1] = 2.0; Ls[1] = 1.0; }
  for (int p = 1; p < k; ++p) {
    const double a = 2.0 * p + 1.0, b = (double)p, c = 1.0 / (p + 1.0);
    L[p + 1] = (a * X * L[p] - b * t * t * L[p - 1]) * c;
    Lr[p + 1] = (a * (2.0 * L[p] + X * Lr[p]) - b * t * t * Lr[p - 1]) * c;
    Ls[p + 1] = (a * (L[p] + X * Ls[p]) - b * (-2.0 * t * L[p - 1] + t * t * Ls[p - 1])) * c;
  }
  int m = 0;
  for (int p = 0; p <= k; ++p)
    for (int q = 0; p + q <= k; ++q, ++m) {
      const double N = std::sqrt(2.0 * (2 * p + 1) * (p + q + 1));
      const double y = 2.0 * s - 1.0;
      const double J = jacobi(q, 2.0 * p + 1.0, 0.0, y);
      const double dJ = q == 0 ? 0.0 : 0.5 * (q + 2.0 * p + 2.0) * jacobi(q - 1, 2.0 * p + 2.0, 1.0, y);
      psi[m] = N * L[p] * J;
      if (dr) dr[m] = N * Lr[p] * J;
      if (ds) ds[m] = N * (Ls[p] * J + L[p] * 2.0 * dJ);
    }
}

constexpr double kV[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};

template <typename R, int K>
inline void fill_tab(TriTab<R, K>& T) {
  constexpr int NP = TriShape<K>::NP, NF = TriShape<K>::NF;
  double xa[K + 2], wa[K + 2], xb[K + 2], wb[K + 2];
  gl_rule(K + 1, xa, wa);
  gl_rule(K + 2, xb, wb);
  double psi[64], dr[64], ds[64];
  for (int j = 0; j < K + 2; ++j)
    for (int i = 0; i < K + 1; ++i) {
      const int q = j * (K + 1) + i;
      const double s = 0.5 * (1.0 + xb[j]);
      const double r = 0.5 * (1.0 + xa[i]) * (1.0 - s);
      const double w = wa[i] * wb[j] * (1.0 - s) * 0.25;
      dubiner(K, r, s, psi, dr, ds);
      for (int m = 0; m < NP; ++m) {
        T.psi[q][m] = (R)psi[m];
        T.dr[q][m] = (R)dr[m];
        T.ds[q][m] = (R)ds[m];
        T.psid[q][m] = psi[m];
      }
      T.w[q] = (R)w;
      T.wd[q] = w;
      T.rq[q] = r;
      T.sq[q] = s;
    }
  for (int f = 0; f < 3; ++f) {
    const int f1 = (f + 1) % 3;
    for (int i = 0; i < NF; ++i) {
      const double u = 0.5 * (1.0 + xa[i]);
      const double r = kV[f][0] + u * (kV[f1][0] - kV[f][0]);
      const double s = kV[f][1] + u * (kV[f1][1] - kV[f][1]);
      dubiner(K, r, s, psi, nullptr, nullptr);
      for (int m = 0; m < NP; ++m) {
        T.psif[f][i][m] = (R)psi[m];
        T.psifd[f][i][m] = psi[m];
      }
      T.rf[f][i] = r;
      T.sf[f][i] = s;
    }
  }
  for (int i = 0; i < NF; ++i) {
    T.wf[i] = (R)(0.5 * wa[i]);
    T.xg[i] = xa[i];
    double d = 1.0;
    for (int j = 0; j < NF; ++j)
      if (j != i) d *= xa[i] - xa[j];
    T.lagd[i] = 1.0 / d;
  }
}

}  // namespace dgm
