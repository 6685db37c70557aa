// Plain, slow FP64 reference of the moist DG right-hand side, the implicit
// condensation split and the SSP Runge-Kutta step.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the library or its Python binding may
// link, import or call this file; only the tests, the smoke check and the CPU
// baseline leg of the benchmark do.  It shares no source with the GPU path.
//
// Each routine follows the paper's statement of the problem in the order the
// paper gives it:
//   * state, pressure and energy relations .......... Section 2 (equation of
//     state; energy-temperature relation)
//   * saturation vapour pressure .................... Section 2.1 (Clausius-
//     Clapeyron form with linear latent heat)
//   * implicit condensation split ................... Section 2.2 (system for
//     rho e, rho_v = min(e_s/(R_v T), rho_m), rho_c = rho_m - rho_v)
//   * perturbation fluxes and sources ............... Section 2.3 (perturbation
//     form of the moist Euler system) and Section 2.1 (Kessler sources)
//   * DG weak form, Lax-Friedrichs flux, wave speed,
//     slip walls ..................................... Section 3.2
//   * diagonal mass, SSPRK(4,3) ...................... Section 3.3
//   * pointwise reconstruction ...................... Section 3.4
// Two spatial bases on an affine box:
//   * nodal Gauss-Lobatto collocation (nodes double as quadrature points), so
//     the L2 projection of Section 3.4 is the identity;
//   * the paper's own: a tensor Legendre (modal) basis of Q^k with its
//     diagonal mass matrix (Section 3.1) and Gauss-Legendre quadrature with
//     k+1 points per axis.  The split runs at the quadrature points and T and
//     rho_v are L2-projected onto Q^k (Section 3.4); face quadrature points
//     see the traces of these projections.  States cross the interface as
//     values at the Gauss points and are projected onto the Legendre basis on
//     entry (and evaluated there on exit).
// And on conforming triangulations of the vertical plane (Section 3.1, the
// P^k space): the orthonormal Dubiner basis with its diagonal mass, the
// Duffy-mapped product Gauss-Legendre rule of the footnote in Section 3.4,
// faces gathered through a neighbour table; states cross the interface as
// coefficients.
//
// The scalar type is a template parameter: `double` gives the reference
// values, `Dual` (value + one tangent) gives exact directional derivatives of
// the same code for the adjoint checks.  Where the method has a kink (min in
// the split, max in the wave speed, abs, clamps at zero) the derivative of the
// active branch is taken; ties go to the unsaturated branch, to the minus side
// of the face, sign(0) = 0, and a clamp has derivative 0 at or below zero.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>
#include <algorithm>
#include <omp.h>

namespace {

// ---------------------------------------------------------------------------
// forward-mode scalar
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) { return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
inline Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
inline Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual operator/(double a, Dual b) { return Dual(a / b.v, -a * b.d / (b.v * b.v)); }
inline Dual exp(Dual a) { double e = std::exp(a.v); return Dual(e, e * a.d); }
inline Dual log(Dual a) { return Dual(std::log(a.v), a.d / a.v); }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
// x^p for p > 0; at x = 0 the value and the tangent are taken as 0
inline Dual pow(Dual a, double p) {
  if (a.v == 0.0) return Dual(0.0, 0.0);
  double y = std::pow(a.v, p);
  return Dual(y, p * y / a.v * a.d);
}

using std::exp;
using std::log;
using std::sqrt;

inline double val(double a) { return a; }
inline double val(Dual a) { return a.v; }
inline double pw(double a, double p) { return std::pow(a, p); }
inline Dual pw(Dual a, double p) { return pow(a, p); }

template <class R> inline R absr(R a) {
  if (val(a) > 0) return a;
  if (val(a) < 0) return -a;
  return R(0.0);
}
template <class R> inline R pos(R a) { return val(a) > 0 ? a : R(0.0); }  // max(a, 0)
template <class R> inline R max_minus(R a, R b) { return val(a) >= val(b) ? a : b; }

}  // namespace

extern "C" {

// Parameters of the model (thermodynamic table of the paper's appendix, g, the
// rain closure and the split's stopping rule).
struct OraParams {
  double g, cvd, cvv, cl, cpd, cpv, Rd, Rv, Lref, Tref, eref, pref;
  int rain;        // 0: no rain (nvars = 3 + d), 1: Kessler warm rain (4 + d)
  int vr_mode;     // 0: constant v_r, 1: COSMO formula
  double vr_const, rho_w, N0r, v0r, q_au;
  // Rayleigh sponge (Section 3.6): bottom height z_D and
  // strength alpha of the blending function; alpha = 0 switches it off
  double sponge_zD, sponge_alpha;
  // artificial diffusion (Section 3.5): viscosity scale gamma (0: off) and
  // penalty sigma of the symmetric interior penalty form
  double sip_gamma, sip_sigma;
};

struct OraMesh {
  int dim;          // 2 or 3; axis dim-1 is vertical
  int n[3];         // elements per axis
  double lo[3], hi[3];
  int bc[3];        // 0 periodic, 1 slip wall (on both ends of that axis)
  int order;        // polynomial order k
  int basis;        // 0: Gauss-Lobatto collocation, 1: Legendre modes + Gauss quadrature
};

void ora_default_params(OraParams* p) {
  // appendix table of thermodynamic parameters
  p->cl = 4218.0; p->cpd = 1005.0; p->cpv = 1850.0; p->cvd = 718.0; p->cvv = 1390.0;
  p->eref = 610.7; p->Lref = 2.835e6; p->Rd = 287.05; p->Rv = 461.51; p->Tref = 273.15;
  p->pref = 1.0e5;
  p->g = 9.81;
  p->rain = 0; p->vr_mode = 0; p->vr_const = 5.0;
  // COSMO warm-rain distribution parameters (Section 2.1)
  p->rho_w = 1000.0; p->N0r = 8.0e6; p->v0r = 130.0; p->q_au = 0.0;
  p->sponge_zD = 0.0; p->sponge_alpha = 0.0;
  p->sip_gamma = 0.0; p->sip_sigma = 10.0;
}

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Gauss-Lobatto tables
// ---------------------------------------------------------------------------
// Legendre P_k and P_k' by the three-term recurrence.
void legendre(int k, double x, double* P, double* dP) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (k == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int m = 1; m < k; ++m) {
    double p2 = ((2.0 * m + 1.0) * x * p1 - m * p0) / (m + 1.0);
    double d2 = d0 + (2.0 * m + 1.0) * p1;   // P'_{m+1} = P'_{m-1} + (2m+1) P_m
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *P = p1; *dP = d1;
}

struct Tables {
  int k;
  std::vector<double> x, w;   // nodes and weights on [-1, 1]
  std::vector<double> D;      // D[a*(k+1)+i] = l_i'(x_a)
  std::vector<double> Dhat;   // Dhat[i*(k+1)+a] = w_a D[a][i] / w_i
};

Tables make_tables(int k) {
  Tables t;
  t.k = k;
  int p1 = k + 1;
  t.x.assign(p1, 0.0); t.w.assign(p1, 0.0);
  t.x[0] = -1.0; t.x[k] = 1.0;
  // interior nodes: roots of P_k', Newton from Chebyshev-Lobatto guesses.
  // (P_k')' = (2x P_k' - k(k+1) P_k)/(1 - x^2) from Legendre's equation.
  for (int i = 1; i < k; ++i) {
    double xx = -std::cos(M_PI * i / k);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(k, xx, &P, &dP);
      double d2P = (2.0 * xx * dP - k * (k + 1.0) * P) / (1.0 - xx * xx);
      double dx = dP / d2P;
      xx -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    t.x[i] = xx;
  }
  for (int i = 0; i < p1; ++i) {
    double P, dP;
    legendre(k, t.x[i], &P, &dP);
    t.w[i] = 2.0 / (k * (k + 1.0) * P * P);
  }
  // differentiation matrix from barycentric weights
  std::vector<double> lam(p1, 1.0);
  for (int i = 0; i < p1; ++i)
    for (int m = 0; m < p1; ++m)
      if (m != i) lam[i] /= (t.x[i] - t.x[m]);
  t.D.assign(p1 * p1, 0.0);
  for (int a = 0; a < p1; ++a) {
    double s = 0.0;
    for (int i = 0; i < p1; ++i) {
      if (i == a) continue;
      double v = (lam[i] / lam[a]) / (t.x[a] - t.x[i]);
      t.D[a * p1 + i] = v;
      s += v;
    }
    t.D[a * p1 + a] = -s;
  }
  t.Dhat.assign(p1 * p1, 0.0);
  for (int i = 0; i < p1; ++i)
    for (int a = 0; a < p1; ++a) t.Dhat[i * p1 + a] = t.w[a] * t.D[a * p1 + i] / t.w[i];
  return t;
}

// P_0..P_k and their derivatives at x by the three-term recurrence
void legendre_all(int k, double x, double* P, double* dP) {
  P[0] = 1.0; dP[0] = 0.0;
  if (k >= 1) { P[1] = x; dP[1] = 1.0; }
  for (int m = 1; m < k; ++m) {
    P[m + 1] = ((2.0 * m + 1.0) * x * P[m] - m * P[m - 1]) / (m + 1.0);
    dP[m + 1] = dP[m - 1] + (2.0 * m + 1.0) * P[m];
  }
}

// Gauss-Legendre rule with k+1 points: the roots of P_{k+1} (Newton from the
// usual cosine guesses) and the weights 2 / ((1 - x^2) P_{k+1}'(x)^2).
struct Gauss {
  std::vector<double> x, w;
};

Gauss make_gauss(int k) {
  Gauss G;
  const int p1 = k + 1;
  G.x.assign(p1, 0.0); G.w.assign(p1, 0.0);
  for (int i = 0; i < p1; ++i) {
    double xx = -std::cos(M_PI * (i + 0.75) / (p1 + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p1, xx, &P, &dP);
      double dx = P / dP;
      xx -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double P, dP;
    legendre(p1, xx, &P, &dP);
    G.x[i] = xx;
    G.w[i] = 2.0 / ((1.0 - xx * xx) * dP * dP);
  }
  return G;
}

// ---------------------------------------------------------------------------
// thermodynamics (Section 2)
// ---------------------------------------------------------------------------
// saturation vapour pressure, Clausius-Clapeyron with linear latent heat
template <class R> R esat(const OraParams& P, R T) {
  double a = (P.cpv - P.cl) / P.Rv;
  double b = (P.Lref - (P.cpv - P.cl) * P.Tref) / P.Rv;
  return P.eref * pw(T / P.Tref, a) * exp(b * (1.0 / P.Tref - 1.0 / T));
}
// saturation vapour density from the vapour equation of state p_v = rho_v R_v T
template <class R> R rho_vs(const OraParams& P, R T) { return esat(P, T) / (P.Rv * T); }

double drho_vs_dT(const OraParams& P, double T) {
  double a = (P.cpv - P.cl) / P.Rv;
  double b = (P.Lref - (P.cpv - P.cl) * P.Tref) / P.Rv;
  return rho_vs(P, T) * (a / T + b / (T * T) - 1.0 / T);
}

// internal energy density for a given temperature and vapour density
// (energy-temperature relation without the kinetic part)
template <class R> R rho_e_of(const OraParams& P, R rd, R rm, R rr, R rv, R T) {
  R Cv = P.cvd * rd + P.cvv * rv + P.cl * (rm - rv + rr);
  return Cv * (T - P.Tref) + rv * (P.Lref - P.Rv * P.Tref);
}

struct SplitOut { double T, rv; int iters; int ok; };

// Implicit condensation split (Section 2.2), in plain double precision.
// The map T -> rho e is strictly increasing on both branches, so the solution
// is unique.  All-vapour temperature first; if the air is not saturated there,
// that is the answer.  Otherwise Newton on
//   f(T) = rho_e_of(rho_v = rho_vs(T), T) - rho e,
// kept inside a bracket by bisection, then polished to the last ulp.
SplitOut split_double(const OraParams& P, double rd, double rm, double rr, double re) {
  SplitOut o{0, 0, 0, 1};
  double Cu = P.cvd * rd + P.cvv * rm + P.cl * rr;
  double Tu = P.Tref + (re - rm * (P.Lref - P.Rv * P.Tref)) / Cu;
  if (!std::isfinite(Tu) || !(Cu > 0)) { o.T = Tu; o.rv = rm; o.ok = 0; return o; }
  if (Tu > 0 && rm <= rho_vs(P, Tu)) { o.T = Tu; o.rv = rm; return o; }
  auto f = [&](double T) { return rho_e_of(P, rd, rm, rr, rho_vs(P, T), T) - re; };
  // Saturated.  Below T_floor = 50 K the state is rejected: if the all-vapour
  // temperature is that low, the root must lie above the floor.
  const double T_floor = 50.0;
  if (!(Tu > T_floor)) {
    if (!(f(T_floor) < 0.0)) { o.T = Tu; o.rv = rm; o.ok = 0; return o; }
    Tu = T_floor;
  }
  auto fp = [&](double T) {
    double rv = rho_vs(P, T);
    double Cv = P.cvd * rd + P.cvv * rv + P.cl * (rm - rv + rr);
    return Cv + drho_vs_dT(P, T) * ((P.cvv - P.cl) * (T - P.Tref) + P.Lref - P.Rv * P.Tref);
  };
  // bracket: f(Tu) < 0; march up until f > 0
  double lo = Tu, hi = Tu + 1.0;
  int guard = 0;
  while (f(hi) <= 0.0 && guard++ < 60) { lo = hi; hi = Tu + 2.0 * (hi - Tu); }
  double T = lo;
  int it = 0;
  for (; it < 200; ++it) {
    double fv = f(T);
    if (fv < 0) lo = T; else hi = T;
    double dT = -fv / fp(T);
    if (std::fabs(dT) <= 1e-14 * T) { T += dT; break; }
    double Tn = T + dT;
    if (!(Tn > lo && Tn < hi)) Tn = 0.5 * (lo + hi);   // Newton left the bracket: bisect
    T = Tn;
    if (hi - lo <= 4e-16 * hi) break;
  }
  // polish: bracket the sign change between neighbouring doubles
  double a = T, b = T;
  int g1 = 0;
  while (f(a) >= 0.0 && g1++ < 64) a = std::nextafter(a, 0.0);
  b = std::nextafter(a, INFINITY);
  int g2 = 0;
  while (f(b) < 0.0 && g2++ < 64) { a = b; b = std::nextafter(b, INFINITY); }
  T = (std::fabs(f(a)) <= std::fabs(f(b))) ? a : b;
  o.T = T;
  o.rv = rho_vs(P, T);
  o.iters = it + 1;
  return o;
}

// The same split for any scalar type: the root is found in double and the
// tangent follows from the implicit function theorem, dT = -f_theta / f_T.
template <class R> void split(const OraParams& P, R rd, R rm, R rr, R re, R* T, R* rv, int* ok,
                              int* iters) {
  SplitOut s = split_double(P, val(rd), val(rm), val(rr), val(re));
  *ok = s.ok; *iters = s.iters;
  R Cu = P.cvd * rd + P.cvv * rm + P.cl * rr;
  R Tu = P.Tref + (re - rm * (P.Lref - P.Rv * P.Tref)) / Cu;
  if (!s.ok || (val(Tu) > 0 && val(rm) <= val(rho_vs(P, R(val(Tu)))))) {
    *T = Tu; *rv = rm; return;
  }
  R T0 = R(s.T);
  R fth = rho_e_of(P, rd, rm, rr, R(s.rv), T0) - re;   // value ~0, tangent = f_theta . dtheta
  double rvs = s.rv;
  double Cv = P.cvd * val(rd) + P.cvv * rvs + P.cl * (val(rm) - rvs + val(rr));
  double fT = Cv + drho_vs_dT(P, s.T) * ((P.cvv - P.cl) * (s.T - P.Tref) + P.Lref - P.Rv * P.Tref);
  R Tt = T0 - (fth - R(val(fth))) / fT;   // value s.T, tangent -f_theta/f_T
  *T = Tt;
  *rv = rho_vs(P, Tt);
}

// ---------------------------------------------------------------------------
// the discretisation context
// ---------------------------------------------------------------------------
struct Ctx {
  OraMesh M;
  OraParams P;
  Tables tab;
  int nvars, np, ne, d, k;
  double h[3];
  std::vector<double> bg_rd, bg_rm, bg_rr, bg_E, bg_p;   // per node height
  // modal basis (basis = 1): Gauss rule, positions and weights of the nodal
  // representation, the Legendre basis at the volume quadrature points
  // (Phi[m*np+q], dPhi[(j*np+m)*np+q] = d/dxi_j), and the split of the
  // background at the node heights
  int basis = 0;
  Gauss gq;
  std::vector<double> xn, wn;
  std::vector<double> Phi, dPhi;
  std::vector<double> bg_T, bg_rv;
  long iters_total = 0;
  int max_iters = 0;
  int bad = 0;
};

// node multi-index: n = i + (k+1)(j + (k+1) l), axis 0 fastest
inline int node_axis(int n, int axis, int p1) {
  for (int a = 0; a < axis; ++a) n /= p1;
  return n % p1;
}
inline int node_set_axis(int n, int axis, int val_, int p1) {
  int stride = 1;
  for (int a = 0; a < axis; ++a) stride *= p1;
  int cur = (n / stride) % p1;
  return n + (val_ - cur) * stride;
}
inline int elem_axis(const Ctx& c, int e, int axis) {
  for (int a = 0; a < axis; ++a) e /= c.M.n[a];
  return e % c.M.n[axis];
}
inline int elem_shift(const Ctx& c, int e, int axis, int delta) {
  int stride = 1;
  for (int a = 0; a < axis; ++a) stride *= c.M.n[a];
  int cur = elem_axis(c, e, axis);
  int nxt = (cur + delta + c.M.n[axis]) % c.M.n[axis];
  return e + (nxt - cur) * stride;
}
inline int height_of(const Ctx& c, int e, int n) {
  int p1 = c.k + 1;
  return elem_axis(c, e, c.d - 1) * p1 + node_axis(n, c.d - 1, p1);
}

// variable indices in the paper's order (rho_d', rho_m', [rho_r'], m_1..m_d, E')
inline int v_rd() { return 0; }
inline int v_rm() { return 1; }
inline int v_rr(const Ctx& c) { return c.P.rain ? 2 : -1; }
inline int v_m(const Ctx& c, int i) { return (c.P.rain ? 3 : 2) + i; }
inline int v_E(const Ctx& c) { return c.nvars - 1; }

// everything the flux, wave speed and sources need at one node
template <class R> struct Point {
  R rd, rm, rr, rho, m[3], u[3], E, T, rv, rc, pp, cm, vr;
  R F[3][8];   // F[j][v]
  R G[8];
  R lam[3];    // |u_j| + |v_r delta_jz| + c_m
};

// Pointwise state, fluxes (Section 2.3 perturbation form) and sources from the
// perturbation Uq, the split result (T, rho_v) and the background values
// (rho_d, rho_m, rho_r, E, p) at the point.
template <class R> void point_core(const Ctx& c, const R* Uq, R T, R rv, double bgd, double bgm,
                                   double bgr, double bgE, double bgp, Point<R>& q) {
  const OraParams& P = c.P;
  int d = c.d;
  R rdp = Uq[v_rd()], rmp = Uq[v_rm()];
  R rrp = P.rain ? Uq[v_rr(c)] : R(0.0);
  q.rd = bgd + rdp;
  q.rm = bgm + rmp;
  q.rr = P.rain ? R(bgr) + rrp : R(0.0);
  q.rho = q.rd + q.rm + q.rr;                                   // total density
  for (int i = 0; i < d; ++i) {
    q.m[i] = Uq[v_m(c, i)];
    q.u[i] = q.m[i] / q.rho;
  }
  q.E = bgE + Uq[v_E(c)];
  q.T = T;
  q.rv = rv;
  q.rc = q.rm - q.rv;
  R p = (q.rd * P.Rd + q.rv * P.Rv) * q.T;                      // equation of state
  q.pp = p - bgp;
  R Cv = P.cvd * q.rd + P.cvv * q.rv + P.cl * (q.rc + q.rr);
  R gam = 1.0 + (q.rd * P.Rd + q.rv * P.Rv) / Cv;               // moist isentropic factor
  q.cm = sqrt(gam * p / q.rho);
  // terminal rain speed
  if (!P.rain) q.vr = R(0.0);
  else if (P.vr_mode == 0) q.vr = R(P.vr_const);
  else {
    double pref = std::pow(M_PI * P.rho_w * P.N0r, -0.125) * P.v0r * std::tgamma(4.5) / 6.0;
    q.vr = pref * pw(pos(q.rr), 0.125);
  }
  int z = d - 1;
  R u2 = R(0.0);
  for (int i = 0; i < d; ++i) u2 += q.u[i] * q.u[i];
  for (int j = 0; j < d; ++j) {
    R vz = (j == z) ? q.vr : R(0.0);
    q.F[j][v_rd()] = q.rd * q.u[j];
    q.F[j][v_rm()] = q.rm * q.u[j];
    if (P.rain) q.F[j][v_rr(c)] = q.rr * (q.u[j] - vz);
    for (int i = 0; i < d; ++i)
      q.F[j][v_m(c, i)] = q.m[i] * q.u[j] + (i == j ? q.pp : R(0.0)) - q.rr * vz * q.u[i];
    q.F[j][v_E(c)] = (q.E + bgp + q.pp) * q.u[j]
                     - (P.cl * (q.T - P.Tref) + 0.5 * u2) * q.rr * vz;
    q.lam[j] = absr(q.u[j]) + absr(vz) + q.cm;
  }
  // sources: gravity and Kessler microphysics (Section 2.1)
  for (int v = 0; v < c.nvars; ++v) q.G[v] = R(0.0);
  R rhop = rdp + rmp + rrp;
  q.G[v_m(c, z)] = -rhop * P.g;
  q.G[v_E(c)] = -q.rho * P.g * q.u[z];
  if (P.rain) {
    R rrp_ = pos(q.rr);
    R Sev = (3.86e-3 - 9.41e-5 * (q.T - P.Tref)) * (1.0 + 9.1 * pw(rrp_, 3.0 / 16.0))
            * (rho_vs(P, q.T) - q.rv) * pw(rrp_, 0.5);
    R Sau = 1e-3 * pos(q.rc - P.q_au * q.rho);
    R Sac = 1.72 * q.rc * pw(rrp_, 7.0 / 8.0);
    q.G[v_rm()] = Sev - Sau - Sac;
    q.G[v_rr(c)] = Sau + Sac - Sev;
  }
}

// Pointwise reconstruction (Section 3.4): the split of the full state at node
// height iz, then point_core.
struct SplitStats {
  long iters_total = 0;
  int max_iters = 0;
  int bad = 0;
};

template <class R> void pointwise(Ctx& c, const R* Uq, int iz, Point<R>& q, SplitStats* st = nullptr) {
  const OraParams& P = c.P;
  int d = c.d;
  R rd = c.bg_rd[iz] + Uq[v_rd()];
  R rm = c.bg_rm[iz] + Uq[v_rm()];
  R rr = P.rain ? R(c.bg_rr[iz]) + Uq[v_rr(c)] : R(0.0);
  R rho = rd + rm + rr;
  R ke = R(0.0);
  for (int i = 0; i < d; ++i) {
    R mi = Uq[v_m(c, i)];
    ke += 0.5 * mi * (mi / rho);
  }
  R re = (c.bg_E[iz] + Uq[v_E(c)]) - ke;                        // rho e = E - rho u.u/2
  int ok = 1, iters = 0;
  R T, rv;
  split(P, rd, rm, rr, re, &T, &rv, &ok, &iters);
  if (st) {
    st->iters_total += iters;
    st->max_iters = std::max(st->max_iters, iters);
    if (!ok) st->bad++;
  } else {
    c.iters_total += iters;
    c.max_iters = std::max(c.max_iters, iters);
    if (!ok) c.bad++;
  }
  point_core(c, Uq, T, rv, c.bg_rd[iz], c.bg_rm[iz], P.rain ? c.bg_rr[iz] : 0.0, c.bg_E[iz],
             c.bg_p[iz], q);
}

// Lax-Friedrichs flux with normal +e_j: (F(U-) + F(U+)).n / 2 + Lambda/2 (U- - U+)
template <class R> void lf_flux(const Ctx& c, const Point<R>& a, const R* Ua, const Point<R>& b,
                                const R* Ub, int j, R* Fs) {
  R L = max_minus(a.lam[j], b.lam[j]);
  for (int v = 0; v < c.nvars; ++v) Fs[v] = 0.5 * (a.F[j][v] + b.F[j][v]) + 0.5 * L * (Ua[v] - Ub[v]);
}


// ---------------------------------------------------------------------------
// right-hand side (Section 3.2 weak form with the diagonal mass of Section 3.3)
// ---------------------------------------------------------------------------
// Slip-wall ghost (Section 3.2): momentum reflected in the wall normal e_j,
// all other components copied.
template <class R> void ghost_state(const Ctx& c, const R* Ua, int j, R* Ug) {
  for (int v = 0; v < c.nvars; ++v) Ug[v] = Ua[v];
  Ug[v_m(c, j)] = -Ua[v_m(c, j)];
}

// dU/dt = M^{-1} [ (F, grad V)_K - sum_faces (F_n, [V]) + (G, V)_K ] on every node.
// ---------------------------------------------------------------------------
// artificial diffusion (Section 3.5), Lobatto basis: the symmetric interior
// penalty form on the interior faces
//   A_h(U, V) = sum_K (alpha grad U, grad V)_K
//             + sum_F [ -(alpha {grad U}.n, [V])_F - (alpha {grad V}.n, [U])_F
//                       + sigma k^2 / h_n (alpha [U], [V])_F ]
// acting on the perturbation unknowns, with the element-wise viscosity
//   alpha_K = gamma 0.5 h^(1 - d/2) ||u||_{0,K}   (||u - v_r e_z||_{0,K} for rho_r),
// h = |K|^(1/d), carried to a continuous Q1 field by the mean over the
// elements that share each vertex.  Slip walls carry no diffusive terms.
// ---------------------------------------------------------------------------
double elem_h(const Ctx& c) {
  double v = 1.0;
  for (int a = 0; a < c.d; ++a) v *= c.h[a];
  return std::pow(v, 1.0 / c.d);
}

// nodal viscosity from the velocities of the points q: an[0] for every
// variable but rho_r, an[1] for rho_r
template <class R> void sip_alpha(const Ctx& c, const std::vector<Point<R>>& q, std::vector<double>* an) {
  const int ne = c.ne, np = c.np, d = c.d, p1 = c.k + 1;
  double J = 1.0;
  for (int a = 0; a < d; ++a) J *= 0.5 * c.h[a];
  const double pre = c.P.sip_gamma * 0.5 * std::pow(elem_h(c), 1.0 - 0.5 * d);
  std::vector<double> aK[2] = {std::vector<double>(ne), std::vector<double>(ne)};
  for (int e = 0; e < ne; ++e) {
    double s0 = 0.0, s1 = 0.0;
    for (int n = 0; n < np; ++n) {
      double w = J;
      for (int a = 0; a < d; ++a) w *= c.tab.w[node_axis(n, a, p1)];
      const Point<R>& qq = q[(long)e * np + n];
      double u2 = 0.0, ur2 = 0.0;
      for (int i = 0; i < d; ++i) {
        const double ui = val(qq.u[i]);
        const double ur = (i == d - 1) ? ui - val(qq.vr) : ui;
        u2 += ui * ui;
        ur2 += ur * ur;
      }
      s0 += w * u2;
      s1 += w * ur2;
    }
    aK[0][e] = pre * std::sqrt(s0);
    aK[1][e] = pre * std::sqrt(s1);
  }
  // vertex means; a periodic axis has n vertices, a walled one n + 1
  int nvx[3] = {1, 1, 1};
  for (int a = 0; a < d; ++a) nvx[a] = c.M.n[a] + (c.M.bc[a] == 0 ? 0 : 1);
  const int nvert = nvx[0] * nvx[1] * nvx[2];
  std::vector<double> vs[2] = {std::vector<double>(nvert, 0.0), std::vector<double>(nvert, 0.0)};
  std::vector<int> cnt(nvert, 0);
  auto vid = [&](int e, int corner) {
    int id = 0, stride = 1;
    for (int a = 0; a < d; ++a) {
      int va = elem_axis(c, e, a) + ((corner >> a) & 1);
      if (c.M.bc[a] == 0) va %= c.M.n[a];
      id += va * stride;
      stride *= nvx[a];
    }
    return id;
  };
  for (int e = 0; e < ne; ++e)
    for (int corner = 0; corner < (1 << d); ++corner) {
      const int id = vid(e, corner);
      vs[0][id] += aK[0][e];
      vs[1][id] += aK[1][e];
      cnt[id] += 1;
    }
  for (int f = 0; f < 2; ++f) an[f].assign((size_t)ne * np, 0.0);
  for (int e = 0; e < ne; ++e)
    for (int n = 0; n < np; ++n)
      for (int corner = 0; corner < (1 << d); ++corner) {
        double wq = 1.0;
        for (int a = 0; a < d; ++a) {
          const double xi = c.tab.x[node_axis(n, a, p1)];
          wq *= ((corner >> a) & 1) ? 0.5 * (1.0 + xi) : 0.5 * (1.0 - xi);
        }
        const int id = vid(e, corner);
        for (int f = 0; f < 2; ++f) an[f][(long)e * np + n] += wq * vs[f][id] / cnt[id];
      }
}

// dU -= M^{-1} A_h(U, .): for every nodal basis function phi_i, A_h(U, phi_i)
// evaluated on the support of phi_i (its element and that element's faces)
template <class R> void sip_add(const Ctx& c, const R* U, R* dU, const std::vector<double>* an) {
  const int nv = c.nvars, np = c.np, ne = c.ne, d = c.d, k = c.k, p1 = k + 1;
  const long N = (long)ne * np;
  auto at = [&](int v, int e, int n) -> long { return (long)v * N + (long)e * np + n; };
  double J = 1.0;
  for (int a = 0; a < d; ++a) J *= 0.5 * c.h[a];
  const Tables& t = c.tab;
  // gradient of every variable at every node
  std::vector<R> G((size_t)d * nv * N);
  auto g_at = [&](int j, int v, int e, int n) -> R& { return G[((size_t)j * nv + v) * N + (long)e * np + n]; };
  for (int j = 0; j < d; ++j)
    for (int v = 0; v < nv; ++v)
#pragma omp parallel for schedule(static)
      for (int e = 0; e < ne; ++e)
        for (int n = 0; n < np; ++n) {
          const int a = node_axis(n, j, p1);
          R sacc = R(0.0);
          for (int b = 0; b < p1; ++b) sacc += t.D[a * p1 + b] * U[at(v, e, node_set_axis(n, j, b, p1))];
          g_at(j, v, e, n) = (2.0 / c.h[j]) * sacc;
        }
  // d/dx_j phi_i at node q of the same element
  auto dphi = [&](int i, int q, int j) -> double {
    for (int a = 0; a < d; ++a)
      if (a != j && node_axis(i, a, p1) != node_axis(q, a, p1)) return 0.0;
    return (2.0 / c.h[j]) * t.D[node_axis(q, j, p1) * p1 + node_axis(i, j, p1)];
  };
  const double sig = c.P.sip_sigma * k * k;
#pragma omp parallel for schedule(static)
  for (int e = 0; e < ne; ++e)
    for (int i = 0; i < np; ++i)
      for (int v = 0; v < nv; ++v) {
        const std::vector<double>& al = an[(c.P.rain && v == v_rr(c)) ? 1 : 0];
        R A = R(0.0);
        // volume
        for (int q = 0; q < np; ++q) {
          double wq = J;
          for (int a = 0; a < d; ++a) wq *= t.w[node_axis(q, a, p1)];
          for (int j = 0; j < d; ++j) {
            const double dp = dphi(i, q, j);
            if (dp != 0.0) A += (wq * al[(long)e * np + q] * dp) * g_at(j, v, e, q);
          }
        }
        // faces of e, normal +e_j from the lower to the upper element
        for (int j = 0; j < d; ++j)
          for (int side = 0; side < 2; ++side) {
            const int ej = elem_axis(c, e, j);
            const bool at_end = side ? ej == c.M.n[j] - 1 : ej == 0;
            if (at_end && c.M.bc[j] == 1) continue;
            const int e2 = elem_shift(c, e, j, side ? +1 : -1);
            for (int nf = 0; nf < np; ++nf) {
              if (node_axis(nf, j, p1) != (side ? k : 0)) continue;
              const int nf2 = node_set_axis(nf, j, side ? 0 : k, p1);
              double wf = 1.0;
              for (int a = 0; a < d; ++a)
                if (a != j) wf *= t.w[node_axis(nf, a, p1)] * 0.5 * c.h[a];
              const R Ue = U[at(v, e, nf)], Uo = U[at(v, e2, nf2)];
              const R jumpU = side ? Ue - Uo : Uo - Ue;
              const R avgG = 0.5 * (g_at(j, v, e, nf) + g_at(j, v, e2, nf2));
              const double phi = (i == nf) ? 1.0 : 0.0;
              const double jumpPhi = side ? phi : -phi;
              const double avgPhi = 0.5 * dphi(i, nf, j);
              const double alf = al[(long)e * np + nf];
              A += wf * alf * (-(avgG * jumpPhi) - avgPhi * jumpU + (sig / c.h[j]) * jumpU * jumpPhi);
            }
          }
        double wi = J;
        for (int a = 0; a < d; ++a) wi *= t.w[node_axis(i, a, p1)];
        dU[at(v, e, i)] -= A / wi;
      }
}

template <class R> void rhs(Ctx& c, const R* U, R* dU, double* wall_rain_flux) {
  const int nv = c.nvars, np = c.np, ne = c.ne, d = c.d, k = c.k, p1 = k + 1;
  const long N = (long)ne * np;
  auto at = [&](int v, int e, int n) -> long { return (long)v * N + (long)e * np + n; };
  // Loops over elements may run on several threads (OpenMP); every value is
  // computed by the same arithmetic in the same order whatever the thread
  // count, so the result does not depend on it.
  // 1. pointwise reconstruction + fluxes at every node
  std::vector<Point<R>> q(N);
  {
    SplitStats tot;
#pragma omp parallel
    {
      SplitStats st;
      std::vector<R> Uq(nv);
#pragma omp for schedule(static)
      for (int e = 0; e < ne; ++e)
        for (int n = 0; n < np; ++n) {
          for (int v = 0; v < nv; ++v) Uq[v] = U[at(v, e, n)];
          pointwise(c, Uq.data(), height_of(c, e, n), q[(long)e * np + n], &st);
        }
#pragma omp critical
      {
        tot.iters_total += st.iters_total;
        tot.max_iters = std::max(tot.max_iters, st.max_iters);
        tot.bad += st.bad;
      }
    }
    c.iters_total += tot.iters_total;
    c.max_iters = std::max(c.max_iters, tot.max_iters);
    c.bad += tot.bad;
  }
  // 2. volume term: sum_j (2/h_j) sum_a Dhat[i_j][a] F_j(node a on the j-line)
#pragma omp parallel for schedule(static)
  for (int e = 0; e < ne; ++e)
    for (int n = 0; n < np; ++n)
      for (int v = 0; v < nv; ++v) {
        R acc = R(0.0);
        for (int j = 0; j < d; ++j) {
          int ij = node_axis(n, j, p1);
          R s = R(0.0);
          for (int a = 0; a < p1; ++a)
            s += c.tab.Dhat[ij * p1 + a] * q[(long)e * np + node_set_axis(n, j, a, p1)].F[j][v];
          acc += (2.0 / c.h[j]) * s;
        }
        dU[at(v, e, n)] = acc;
      }
  // 3. faces with normal +e_j between K- = e and K+ = its +j neighbour.  For
  // a fixed j the iteration for e writes only the +j face nodes of e and the
  // -j face nodes of its +j neighbour (or, at a bottom wall, of e itself), so
  // no two iterations touch the same node.  The wall rain flux is summed
  // afterwards in the loop order.
  double wflux = 0.0;
  std::vector<double> wtop, wbot;
  if (c.P.rain) {
    wtop.assign((size_t)N, 0.0);
    wbot.assign((size_t)N, 0.0);
  }
  for (int j = 0; j < d; ++j) {
    const double liftK = (2.0 / c.h[j]) / c.tab.w[k];
    const double lift0 = (2.0 / c.h[j]) / c.tab.w[0];
    const bool wall = c.M.bc[j] == 1;
    SplitStats tot;
#pragma omp parallel
    {
      SplitStats st;
      std::vector<R> Um(nv), Up(nv), Fs(nv), Ui(nv), Ug(nv);
#pragma omp for schedule(static)
      for (int e = 0; e < ne; ++e) {
        const int ej = elem_axis(c, e, j);
        const bool top = ej == c.M.n[j] - 1;
        const bool bottom = ej == 0;
        for (int n = 0; n < np; ++n) {
          if (node_axis(n, j, p1) != k) continue;     // nodes of e on its +j face
          const int nb = node_set_axis(n, j, 0, p1);  // matching node on the other side
          // face weight times face Jacobian, for the boundary flux diagnostic
          double wf = 1.0;
          for (int a = 0; a < d; ++a)
            if (a != j) wf *= c.tab.w[node_axis(n, a, p1)] * 0.5 * c.h[a];
          for (int v = 0; v < nv; ++v) Um[v] = U[at(v, e, n)];
          const Point<R>& qm = q[(long)e * np + n];
          if (wall && top) {
            // top wall: U+ is the ghost of U-; only K- is updated
            ghost_state(c, Um.data(), j, Up.data());
            Point<R> qg;
            pointwise(c, Up.data(), height_of(c, e, n), qg, &st);
            lf_flux(c, qm, Um.data(), qg, Up.data(), j, Fs.data());
            for (int v = 0; v < nv; ++v) dU[at(v, e, n)] -= liftK * Fs[v];
            if (c.P.rain) wtop[(long)e * np + n] = wf * val(Fs[v_rr(c)]);
          } else {
            const int e2 = elem_shift(c, e, j, +1);
            for (int v = 0; v < nv; ++v) Up[v] = U[at(v, e2, nb)];
            const Point<R>& qp = q[(long)e2 * np + nb];
            lf_flux(c, qm, Um.data(), qp, Up.data(), j, Fs.data());
            for (int v = 0; v < nv; ++v) {
              dU[at(v, e, n)] -= liftK * Fs[v];
              dU[at(v, e2, nb)] += lift0 * Fs[v];
            }
          }
          if (wall && bottom) {
            // bottom wall of e: K- is the ghost below, K+ = e at its node index 0
            const int n0 = node_set_axis(n, j, 0, p1);
            for (int v = 0; v < nv; ++v) Ui[v] = U[at(v, e, n0)];
            ghost_state(c, Ui.data(), j, Ug.data());
            Point<R> qg;
            pointwise(c, Ug.data(), height_of(c, e, n0), qg, &st);
            const Point<R>& qi = q[(long)e * np + n0];
            lf_flux(c, qg, Ug.data(), qi, Ui.data(), j, Fs.data());
            for (int v = 0; v < nv; ++v) dU[at(v, e, n0)] += lift0 * Fs[v];
            if (c.P.rain) wbot[(long)e * np + n] = wf * val(Fs[v_rr(c)]);
          }
        }
      }
#pragma omp critical
      {
        tot.iters_total += st.iters_total;
        tot.max_iters = std::max(tot.max_iters, st.max_iters);
        tot.bad += st.bad;
      }
    }
    c.iters_total += tot.iters_total;
    c.max_iters = std::max(c.max_iters, tot.max_iters);
    c.bad += tot.bad;
    if (c.P.rain && wall)
      for (int e = 0; e < ne; ++e) {
        const int ej = elem_axis(c, e, j);
        const bool top = ej == c.M.n[j] - 1, bottom = ej == 0;
        if (!top && !bottom) continue;
        for (int n = 0; n < np; ++n) {
          if (node_axis(n, j, p1) != k) continue;
          if (top) wflux += wtop[(long)e * np + n];
          if (bottom) wflux -= wbot[(long)e * np + n];
        }
      }
  }
  // 4. sources
#pragma omp parallel for schedule(static)
  for (int e = 0; e < ne; ++e)
    for (int n = 0; n < np; ++n)
      for (int v = 0; v < nv; ++v) dU[at(v, e, n)] += q[(long)e * np + n].G[v];
  // 5. artificial diffusion
  if (c.P.sip_gamma > 0.0) {
    std::vector<double> an[2];
    sip_alpha(c, q, an);
    sip_add(c, U, dU, an);
  }
  if (wall_rain_flux) *wall_rain_flux = wflux;
}

// Blending function of the sponge layer (Section 3.6):
// delta(z) = alpha/2 (1 - cos(pi (z - z_D)/(z_T - z_D))) above z_D, 0 below,
// with z_T the top of the domain.
double sponge_delta(const Ctx& c, double z) {
  const double zD = c.P.sponge_zD, zT = c.M.hi[c.d - 1];
  if (!(c.P.sponge_alpha > 0.0) || z < zD) return 0.0;
  return 0.5 * c.P.sponge_alpha * (1.0 - std::cos(M_PI * (z - zD) / (zT - zD)));
}

// height of node n of element e
double node_z(const Ctx& c, int e, int n) {
  const int a = c.d - 1;
  return c.M.lo[a] + c.h[a] * (elem_axis(c, e, a) + 0.5 * (1.0 + c.xn[node_axis(n, a, c.k + 1)]));
}

// The sponge at the end of a time step, node by node (with Lobatto
// collocation the L2 projection of the product is its nodal value): the
// moist perturbations, the momentum and E' relax towards the far field
// (0, 0, rho u_bar = 0, 0), U = (1 - delta) U_pred + delta U_far, and the
// moist mass removed is added to rho_d' at the same node, so the total
// density is unchanged.
template <class R> void sponge(Ctx& c, R* U) {
  if (!(c.P.sponge_alpha > 0.0)) return;
  const long N = (long)c.ne * c.np;
  for (int e = 0; e < c.ne; ++e)
    for (int n = 0; n < c.np; ++n) {
      const double dl = sponge_delta(c, node_z(c, e, n));
      if (dl == 0.0) continue;
      const long i = (long)e * c.np + n;
      R lost = U[v_rm() * N + i] * dl;
      if (c.P.rain) lost = lost + U[v_rr(c) * N + i] * dl;
      for (int v = 1; v < c.nvars; ++v) U[v * N + i] = U[v * N + i] * (1.0 - dl);
      U[v_rd() * N + i] = U[v_rd() * N + i] + lost;
    }
}

// ---------------------------------------------------------------------------
// the modal basis (basis = 1)
// ---------------------------------------------------------------------------
// ||phi_m||^2 on the reference element: prod_a 2 / (2 m_a + 1)
double mode_norm(const Ctx& c, int m) {
  double s = 1.0;
  for (int a = 0; a < c.d; ++a) s *= 2.0 / (2.0 * node_axis(m, a, c.k + 1) + 1.0);
  return s;
}

// product weight of volume quadrature point q
double quad_w(const Ctx& c, int q) {
  double w = 1.0;
  for (int a = 0; a < c.d; ++a) w *= c.gq.w[node_axis(q, a, c.k + 1)];
  return w;
}

// every basis function at the reference point xi
void basis_at(const Ctx& c, const double* xi, double* phi) {
  double P[3][16], dP[16];
  for (int a = 0; a < c.d; ++a) legendre_all(c.k, xi[a], P[a], dP);
  for (int m = 0; m < c.np; ++m) {
    double v = 1.0;
    for (int a = 0; a < c.d; ++a) v *= P[a][node_axis(m, a, c.k + 1)];
    phi[m] = v;
  }
}

void make_modal_tables(Ctx& c) {
  const int np = c.np, d = c.d, p1 = c.k + 1;
  c.Phi.assign((size_t)np * np, 0.0);
  c.dPhi.assign((size_t)d * np * np, 0.0);
  for (int q = 0; q < np; ++q) {
    double P[3][16], dP[3][16];
    for (int a = 0; a < d; ++a) legendre_all(c.k, c.gq.x[node_axis(q, a, p1)], P[a], dP[a]);
    for (int m = 0; m < np; ++m) {
      double v = 1.0;
      for (int a = 0; a < d; ++a) v *= P[a][node_axis(m, a, p1)];
      c.Phi[(size_t)m * np + q] = v;
      for (int j = 0; j < d; ++j) {
        double g = 1.0;
        for (int a = 0; a < d; ++a) {
          int ma = node_axis(m, a, p1);
          g *= (a == j) ? dP[a][ma] : P[a][ma];
        }
        c.dPhi[((size_t)j * np + m) * np + q] = g;
      }
    }
  }
}

// L2 projection onto the Legendre modes of values at the volume quadrature
// points, element by element: c_m = sum_q w_q phi_m(x_q) u_q / ||phi_m||^2
template <class R> void to_modal(const Ctx& c, int nfields, const R* U, R* C) {
  const int np = c.np;
  for (long b = 0; b < (long)nfields * c.ne; ++b)
    for (int m = 0; m < np; ++m) {
      R s = R(0.0);
      for (int q = 0; q < np; ++q) s += (quad_w(c, q) * c.Phi[(size_t)m * np + q]) * U[b * np + q];
      C[b * np + m] = s / mode_norm(c, m);
    }
}

// values at the volume quadrature points: u_q = sum_m c_m phi_m(x_q)
template <class R> void to_points(const Ctx& c, int nfields, const R* C, R* U) {
  const int np = c.np;
  for (long b = 0; b < (long)nfields * c.ne; ++b)
    for (int q = 0; q < np; ++q) {
      R s = R(0.0);
      for (int m = 0; m < np; ++m) s += c.Phi[(size_t)m * np + q] * C[b * np + m];
      U[b * np + q] = s;
    }
}

template <class R> R expand(const Ctx& c, const R* cm, const double* phi) {
  R s = R(0.0);
  for (int m = 0; m < c.np; ++m) s += cm[m] * phi[m];
  return s;
}

// The background in element row ez at reference height xi_z, as the Legendre
// expansion (projection onto P^k) of its values at the row's node heights:
// out = (rho_d, rho_m, rho_r, E, T, rho_v).
void bg_trace(const Ctx& c, int ez, double xi_z, double* out) {
  const int p1 = c.k + 1;
  double P[16], dP[16];
  legendre_all(c.k, xi_z, P, dP);
  const std::vector<double>* f[6] = {&c.bg_rd, &c.bg_rm, &c.bg_rr, &c.bg_E, &c.bg_T, &c.bg_rv};
  for (int i = 0; i < 6; ++i) {
    double v = 0.0;
    for (int m = 0; m < p1; ++m) {
      double beta = 0.0;
      for (int l = 0; l < p1; ++l) {
        double Pl[16], dPl[16];
        legendre_all(c.k, c.gq.x[l], Pl, dPl);
        beta += c.gq.w[l] * Pl[m] * (*f[i])[ez * p1 + l];
      }
      v += (2.0 * m + 1.0) / 2.0 * beta * P[m];
    }
    out[i] = v;
  }
}

// State at a face quadrature point of element e (reference point xi) from the
// modal coefficients of U, T and rho_v.  The background pressure there is the
// equation of state of the traced background, so that an unperturbed state
// carries no pressure perturbation on faces either.
template <class R> void face_point(const Ctx& c, const R* C, const R* Tc, const R* Rvc, int e,
                                   const double* xi, R* Ut, Point<R>& q, double* bgo) {
  const long N = (long)c.ne * c.np;
  std::vector<double> phi(c.np);
  basis_at(c, xi, phi.data());
  for (int v = 0; v < c.nvars; ++v) Ut[v] = expand(c, C + (long)v * N + (long)e * c.np, phi.data());
  R T = expand(c, Tc + (long)e * c.np, phi.data());
  R rv = expand(c, Rvc + (long)e * c.np, phi.data());
  double b[6];
  bg_trace(c, elem_axis(c, e, c.d - 1), xi[c.d - 1], b);
  bgo[0] = b[0]; bgo[1] = b[1]; bgo[2] = c.P.rain ? b[2] : 0.0; bgo[3] = b[3];
  bgo[4] = (b[0] * c.P.Rd + b[5] * c.P.Rv) * b[4];
  point_core(c, Ut, T, rv, bgo[0], bgo[1], bgo[2], bgo[3], bgo[4], q);
}

// slip-wall ghost of a face point: momentum reflected, the traced T, rho_v
// and background kept
template <class R> void face_ghost(const Ctx& c, const R* Ut, const Point<R>& qi, const double* bgo, int j,
                                   R* Ug, Point<R>& qg) {
  ghost_state(c, Ut, j, Ug);
  point_core(c, Ug, qi.T, qi.rv, bgo[0], bgo[1], bgo[2], bgo[3], bgo[4], qg);
}

// dC/dt on the modal coefficients C (Section 3.2 weak form, Section 3.3
// diagonal mass, Section 3.4 reconstruction):
//   M dC/dt = (F(U_h), grad phi)_K - <F*, phi>_dK + (G, phi)_K,
// every integral by the Gauss rule of k+1 points per axis.
template <class R> void modal_rhs(Ctx& c, const R* C, R* dC, double* wall_rain_flux) {
  const int nv = c.nvars, np = c.np, ne = c.ne, d = c.d, k = c.k, p1 = k + 1;
  const long N = (long)ne * np;
  auto at = [&](int v, int e, int n) -> long { return (long)v * N + (long)e * np + n; };
  // 1. the state at the volume quadrature points, its split, fluxes and sources
  std::vector<R> Uq((size_t)nv * N);
  to_points(c, nv, C, Uq.data());
  std::vector<Point<R>> q(N);
  std::vector<R> Tq(N), Rvq(N), u(nv);
  for (int e = 0; e < ne; ++e)
    for (int n = 0; n < np; ++n) {
      for (int v = 0; v < nv; ++v) u[v] = Uq[at(v, e, n)];
      Point<R>& qq = q[(long)e * np + n];
      pointwise(c, u.data(), height_of(c, e, n), qq);
      Tq[(long)e * np + n] = qq.T;
      Rvq[(long)e * np + n] = qq.rv;
    }
  // 2. L2 projections of T and rho_v onto Q^k
  std::vector<R> Tc(N), Rvc(N);
  to_modal(c, 1, Tq.data(), Tc.data());
  to_modal(c, 1, Rvq.data(), Rvc.data());
  // 3. volume and source integrals
  for (int e = 0; e < ne; ++e)
    for (int m = 0; m < np; ++m)
      for (int v = 0; v < nv; ++v) {
        R acc = R(0.0);
        for (int n = 0; n < np; ++n) {
          const Point<R>& qq = q[(long)e * np + n];
          const double w = quad_w(c, n);
          for (int j = 0; j < d; ++j)
            acc += (w * (2.0 / c.h[j]) * c.dPhi[((size_t)j * np + m) * np + n]) * qq.F[j][v];
          acc += (w * c.Phi[(size_t)m * np + n]) * qq.G[v];
        }
        dC[at(v, e, m)] = acc;
      }
  // 4. faces with normal +e_j, Gauss points on the face
  int nf = 1;
  for (int a = 0; a < d - 1; ++a) nf *= p1;
  std::vector<R> Um(nv), Up(nv), Ug(nv), Fs(nv);
  std::vector<double> phiM(np), phiP(np);
  double wflux = 0.0;
  for (int j = 0; j < d; ++j) {
    const bool wall = c.M.bc[j] == 1;
    for (int e = 0; e < ne; ++e) {
      const int ej = elem_axis(c, e, j);
      const bool top = ej == c.M.n[j] - 1, bottom = ej == 0;
      for (int f = 0; f < nf; ++f) {
        double xi[3], wf = 1.0, wphys = 1.0;
        int o = f;
        for (int a = 0; a < d; ++a) {
          if (a == j) continue;
          int ia = o % p1;
          o /= p1;
          xi[a] = c.gq.x[ia];
          wf *= c.gq.w[ia];
          wphys *= c.gq.w[ia] * 0.5 * c.h[a];
        }
        const double lift = 2.0 / c.h[j];
        // plus face of e (xi_j = +1)
        xi[j] = 1.0;
        basis_at(c, xi, phiM.data());
        Point<R> qm, qp;
        double bm[5], bp[5];
        face_point(c, C, Tc.data(), Rvc.data(), e, xi, Um.data(), qm, bm);
        if (wall && top) {
          Point<R> qg;
          face_ghost(c, Um.data(), qm, bm, j, Ug.data(), qg);
          lf_flux(c, qm, Um.data(), qg, Ug.data(), j, Fs.data());
          for (int m = 0; m < np; ++m)
            for (int v = 0; v < nv; ++v) dC[at(v, e, m)] -= (lift * wf * phiM[m]) * Fs[v];
          if (c.P.rain) wflux += wphys * val(Fs[v_rr(c)]);
        } else {
          const int e2 = elem_shift(c, e, j, +1);
          xi[j] = -1.0;
          basis_at(c, xi, phiP.data());
          face_point(c, C, Tc.data(), Rvc.data(), e2, xi, Up.data(), qp, bp);
          lf_flux(c, qm, Um.data(), qp, Up.data(), j, Fs.data());
          for (int m = 0; m < np; ++m)
            for (int v = 0; v < nv; ++v) {
              dC[at(v, e, m)] -= (lift * wf * phiM[m]) * Fs[v];
              dC[at(v, e2, m)] += (lift * wf * phiP[m]) * Fs[v];
            }
        }
        if (wall && bottom) {
          // minus face of e (xi_j = -1) on the wall: the ghost is the minus side
          xi[j] = -1.0;
          basis_at(c, xi, phiP.data());
          Point<R> qi, qg;
          face_point(c, C, Tc.data(), Rvc.data(), e, xi, Up.data(), qi, bp);
          face_ghost(c, Up.data(), qi, bp, j, Ug.data(), qg);
          lf_flux(c, qg, Ug.data(), qi, Up.data(), j, Fs.data());
          for (int m = 0; m < np; ++m)
            for (int v = 0; v < nv; ++v) dC[at(v, e, m)] += (lift * wf * phiP[m]) * Fs[v];
          if (c.P.rain) wflux -= wphys * val(Fs[v_rr(c)]);
        }
      }
    }
  }
  // 5. inverse of the diagonal mass matrix (J cancels against the 2/h factors)
  for (int v = 0; v < nv; ++v)
    for (int e = 0; e < ne; ++e)
      for (int m = 0; m < np; ++m) dC[at(v, e, m)] = dC[at(v, e, m)] / mode_norm(c, m);
  if (wall_rain_flux) *wall_rain_flux = wflux;
}

// The sponge on modal coefficients: the pointwise update at the volume
// quadrature points, then the L2 projection back onto Q^k (Section 3.6).
template <class R> void sponge_modal(Ctx& c, R* C) {
  if (!(c.P.sponge_alpha > 0.0)) return;
  const long n = (long)c.nvars * c.ne * c.np;
  std::vector<R> U(n);
  to_points(c, c.nvars, C, U.data());
  sponge(c, U.data());
  to_modal(c, c.nvars, U.data(), C);
}

template <class R> void any_rhs(Ctx& c, const R* U, R* dU, double* wall_rain_flux) {
  if (c.basis == 1) modal_rhs(c, U, dU, wall_rain_flux);
  else rhs(c, U, dU, wall_rain_flux);
}

template <class R> void any_sponge(Ctx& c, R* U) {
  if (c.basis == 1) sponge_modal(c, U);
  else sponge(c, U);
}

// SSP Runge-Kutta step in Shu-Osher form (Section 3.3 remark): SSPRK(4,3) of
// Kraaijevanger, or the three-stage SSPRK(3,3), on N unknowns U with the
// right-hand side any_rhs(u, L, &wall_rain_flux).
template <class R, class Rhs> void ssprk(long N, R* U, double dt, int scheme, Rhs&& any_rhs,
                                         double* outflow) {
  std::vector<R> u0(U, U + N), us(N), L(N);
  double fl = 0.0, f = 0.0;
  if (scheme == 0) {
    // u1 = u0 + dt/2 L(u0); u2 = u1 + dt/2 L(u1);
    // u3 = 2/3 u0 + 1/3 u2 + dt/6 L(u2); u4 = u3 + dt/2 L(u3)
    any_rhs(u0.data(), L.data(), &f); fl += f / 6.0;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) us[i] = u0[i] + (0.5 * dt) * L[i];
    any_rhs(us.data(), L.data(), &f); fl += f / 6.0;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) us[i] = us[i] + (0.5 * dt) * L[i];
    any_rhs(us.data(), L.data(), &f); fl += f / 6.0;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) us[i] = (2.0 / 3.0) * u0[i] + (1.0 / 3.0) * us[i] + (dt / 6.0) * L[i];
    any_rhs(us.data(), L.data(), &f); fl += f / 2.0;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) U[i] = us[i] + (0.5 * dt) * L[i];
  } else {
    // u1 = u0 + dt L(u0); u2 = 3/4 u0 + 1/4 u1 + dt/4 L(u1);
    // u3 = 1/3 u0 + 2/3 u2 + 2/3 dt L(u2)
    any_rhs(u0.data(), L.data(), &f); fl += f / 6.0;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) us[i] = u0[i] + dt * L[i];
    any_rhs(us.data(), L.data(), &f); fl += f / 6.0;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) us[i] = 0.75 * u0[i] + 0.25 * us[i] + (0.25 * dt) * L[i];
    any_rhs(us.data(), L.data(), &f); fl += f * (2.0 / 3.0);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) U[i] = (1.0 / 3.0) * u0[i] + (2.0 / 3.0) * us[i] + ((2.0 / 3.0) * dt) * L[i];
  }
  if (outflow) *outflow = fl * dt;
}

// The step of the box meshes; the sponge, when on, closes the step.
template <class R> void rk_step(Ctx& c, R* U, double dt, int scheme, double* outflow) {
  ssprk((long)c.ne * c.np * c.nvars, U, dt, scheme,
        [&](const R* u, R* L, double* f) { any_rhs(c, u, L, f); }, outflow);
  any_sponge(c, U);
}

}  // namespace

// ---------------------------------------------------------------------------
// C entry points used by the tests through ctypes
// ---------------------------------------------------------------------------
extern "C" {

int ora_tables(int k, double* x, double* w, double* D, double* Dhat) {
  if (k < 1 || k > 12) return -1;
  Tables t = make_tables(k);
  int p1 = k + 1;
  std::memcpy(x, t.x.data(), p1 * sizeof(double));
  std::memcpy(w, t.w.data(), p1 * sizeof(double));
  std::memcpy(D, t.D.data(), p1 * p1 * sizeof(double));
  std::memcpy(Dhat, t.Dhat.data(), p1 * p1 * sizeof(double));
  return 0;
}

double ora_esat(const OraParams* P, double T) { return esat(*P, T); }
double ora_rho_vs(const OraParams* P, double T) { return rho_vs(*P, T); }

// Split of one state; returns the Newton iteration count (0 on the unsaturated
// branch) or -1 if no temperature above 50 K solves the system.
int ora_split(const OraParams* P, double rd, double rm, double rr, double re, double* T,
              double* rv, double* rc) {
  SplitOut s = split_double(*P, rd, rm, rr, re);
  *T = s.T; *rv = s.rv; *rc = rm - s.rv;
  return s.ok ? s.iters : -1;
}

// tangent of the split: (dT, drho_v) along (drd, drm, drr, dre)
int ora_split_jvp(const OraParams* P, double rd, double rm, double rr, double re, double drd,
                  double drm, double drr, double dre, double* T, double* dT, double* rv,
                  double* drv) {
  Dual Tt, rvt;
  int ok, it;
  split(*P, Dual(rd, drd), Dual(rm, drm), Dual(rr, drr), Dual(re, dre), &Tt, &rvt, &ok, &it);
  *T = Tt.v; *dT = Tt.d; *rv = rvt.v; *drv = rvt.d;
  return ok ? 0 : -1;
}

// Set up a mesh, tables and background.  The background arrays hold rho_d,
// rho_m, rho_r, E at the n_z (k+1) node heights; the background pressure is the
// equation of state applied to the split of the background state.
void* ora_create(const OraMesh* M, const OraParams* P, int nvars, const double* rd,
                 const double* rm, const double* rr, const double* E) {
  if (M->dim < 2 || M->dim > 3 || M->order < 1 || M->order > 8) return nullptr;
  if (M->basis != 0 && M->basis != 1) return nullptr;
  if (M->basis == 1 && P->sip_gamma > 0.0) return nullptr;   // diffusion: Lobatto basis only
  if (nvars != (P->rain ? 4 : 3) + M->dim) return nullptr;
  Ctx* c = new Ctx();
  c->M = *M; c->P = *P;
  c->d = M->dim; c->k = M->order; c->nvars = nvars;
  c->tab = make_tables(c->k);
  c->np = 1; c->ne = 1;
  for (int a = 0; a < c->d; ++a) {
    c->np *= (c->k + 1);
    c->ne *= M->n[a];
    c->h[a] = (M->hi[a] - M->lo[a]) / M->n[a];
  }
  int nzq = M->n[c->d - 1] * (c->k + 1);
  c->bg_rd.assign(rd, rd + nzq); c->bg_rm.assign(rm, rm + nzq);
  c->bg_rr.assign(rr, rr + nzq); c->bg_E.assign(E, E + nzq);
  c->bg_p.assign(nzq, 0.0);
  c->bg_T.assign(nzq, 0.0);
  c->bg_rv.assign(nzq, 0.0);
  for (int iz = 0; iz < nzq; ++iz) {
    double rrr = P->rain ? rr[iz] : 0.0;
    SplitOut s = split_double(*P, rd[iz], rm[iz], rrr, E[iz]);
    c->bg_p[iz] = (rd[iz] * P->Rd + s.rv * P->Rv) * s.T;
    c->bg_T[iz] = s.T;
    c->bg_rv[iz] = s.rv;
  }
  c->basis = M->basis;
  if (c->basis == 1) {
    c->gq = make_gauss(c->k);
    c->xn = c->gq.x;
    c->wn = c->gq.w;
    make_modal_tables(*c);
  } else {
    c->xn = c->tab.x;
    c->wn = c->tab.w;
  }
  return c;
}

// Gauss-Legendre rule of k+1 points
int ora_gauss_tables(int k, double* x, double* w) {
  if (k < 0 || k > 12) return -1;
  Gauss G = make_gauss(k);
  std::memcpy(x, G.x.data(), (k + 1) * sizeof(double));
  std::memcpy(w, G.w.data(), (k + 1) * sizeof(double));
  return 0;
}

void ora_destroy(void* h) { delete (Ctx*)h; }

void ora_background_pressure(void* h, double* p) {
  Ctx* c = (Ctx*)h;
  std::copy(c->bg_p.begin(), c->bg_p.end(), p);
}

// split of every node: T, rho_v, rho_c, p' and c_m in U's node order
int ora_split_field(void* h, const double* U, double* T, double* rv, double* rc, double* pp,
                    double* cm) {
  Ctx* c = (Ctx*)h;
  long N = (long)c->ne * c->np;
  std::vector<double> Uq(c->nvars);
  int bad = c->bad;
  for (int e = 0; e < c->ne; ++e)
    for (int n = 0; n < c->np; ++n) {
      long i = (long)e * c->np + n;
      for (int v = 0; v < c->nvars; ++v) Uq[v] = U[(long)v * N + i];
      Point<double> q;
      pointwise(*c, Uq.data(), height_of(*c, e, n), q);
      if (T) T[i] = q.T;
      if (rv) rv[i] = q.rv;
      if (rc) rc[i] = q.rc;
      if (pp) pp[i] = q.pp;
      if (cm) cm[i] = q.cm;
    }
  return c->bad - bad;
}

}  // extern "C"

namespace {
// right-hand side of a state given by its node values (Gauss points for the
// modal basis: projected on entry, the result evaluated there on exit)
template <class R> void nodal_rhs(Ctx& c, const R* U, R* dU, double* wall_rain_flux) {
  if (c.basis == 0) { rhs(c, U, dU, wall_rain_flux); return; }
  const long n = (long)c.nvars * c.ne * c.np;
  std::vector<R> C(n), dC(n);
  to_modal(c, c.nvars, U, C.data());
  modal_rhs(c, C.data(), dC.data(), wall_rain_flux);
  to_points(c, c.nvars, dC.data(), dU);
}

// nsteps RK steps of a nodal state in place
template <class R> void nodal_rk(Ctx& c, R* U, double dt, int nsteps, int scheme, double* outflow) {
  const long n = (long)c.nvars * c.ne * c.np;
  std::vector<R> C;
  R* X = U;
  if (c.basis == 1) {
    C.resize(n);
    to_modal(c, c.nvars, U, C.data());
    X = C.data();
  }
  double acc = 0.0;
  for (int s = 0; s < nsteps; ++s) {
    double f = 0.0;
    rk_step(c, X, dt, scheme, outflow ? &f : nullptr);
    acc += f;
  }
  if (c.basis == 1) to_points(c, c.nvars, C.data(), U);
  if (outflow) *outflow = acc;
}
}  // namespace

extern "C" {

int ora_rhs(void* h, const double* U, double* dU, double* wall_rain_flux) {
  Ctx* c = (Ctx*)h;
  int bad = c->bad;
  nodal_rhs(*c, U, dU, wall_rain_flux);
  return c->bad - bad;
}

// nsteps steps of size dt in place; outflow accumulates dt * sum_s b_s * (wall
// rain flux of stage s), the total rain mass that left through the walls
int ora_rk_step(void* h, double* U, double dt, int nsteps, int scheme, double* outflow) {
  Ctx* c = (Ctx*)h;
  int bad = c->bad;
  double acc = 0.0;
  nodal_rk(*c, U, dt, nsteps, scheme, &acc);
  if (outflow) *outflow = acc;
  return c->bad - bad;
}

// exact directional derivative of the right-hand side: JV = d rhs(U + eps V)/d eps
int ora_rhs_jvp(void* h, const double* U, const double* V, double* dU, double* JV) {
  Ctx* c = (Ctx*)h;
  long N = (long)c->ne * c->np * c->nvars;
  std::vector<Dual> Ud(N), Rd(N);
  for (long i = 0; i < N; ++i) Ud[i] = Dual(U[i], V[i]);
  int bad = c->bad;
  nodal_rhs(*c, Ud.data(), Rd.data(), nullptr);
  for (long i = 0; i < N; ++i) { if (dU) dU[i] = Rd[i].v; JV[i] = Rd[i].d; }
  return c->bad - bad;
}

// nsteps RK steps of (U, V) in place: U the state, V its tangent
int ora_rk_jvp(void* h, double* U, double* V, double dt, int nsteps, int scheme) {
  Ctx* c = (Ctx*)h;
  long N = (long)c->ne * c->np * c->nvars;
  std::vector<Dual> Ud(N);
  for (long i = 0; i < N; ++i) Ud[i] = Dual(U[i], V[i]);
  int bad = c->bad;
  nodal_rk(*c, Ud.data(), dt, nsteps, scheme, nullptr);
  for (long i = 0; i < N; ++i) { U[i] = Ud[i].v; V[i] = Ud[i].d; }
  return c->bad - bad;
}

// sponge blending function at height z, and the sponge applied once to U
double ora_sponge_delta(void* h, double z) { return sponge_delta(*(Ctx*)h, z); }
void ora_sponge_apply(void* h, double* U) {
  Ctx* c = (Ctx*)h;
  if (c->basis == 0) { sponge(*c, U); return; }
  const long n = (long)c->nvars * c->ne * c->np;
  std::vector<double> C(n);
  to_modal(*c, c->nvars, U, C.data());
  sponge_modal(*c, C.data());
  to_points(*c, c->nvars, C.data(), U);
}

// M_d = sum w J rho_d', M_w = sum w J (rho_m' + rho_r'), and the instantaneous
// rain mass flux out through the walls
void ora_mass(void* h, const double* U, double* out3) {
  Ctx* c = (Ctx*)h;
  long N = (long)c->ne * c->np;
  int p1 = c->k + 1;
  double J = 1.0;
  for (int a = 0; a < c->d; ++a) J *= 0.5 * c->h[a];
  double md = 0.0, mw = 0.0;
  for (int e = 0; e < c->ne; ++e)
    for (int n = 0; n < c->np; ++n) {
      double w = J;
      for (int a = 0; a < c->d; ++a) w *= c->wn[node_axis(n, a, p1)];
      long i = (long)e * c->np + n;
      md += w * U[i];
      mw += w * (U[N + i] + (c->P.rain ? U[2 * N + i] : 0.0));
    }
  out3[0] = md; out3[1] = mw;
  std::vector<double> dU(N * c->nvars);
  double f = 0.0;
  nodal_rhs(*c, U, dU.data(), &f);
  out3[2] = f;
}

// pointwise physical fluxes F[j*nvars+v], sources G[v] and wave speeds lam[j]
// of one state Uq at node height iz
void ora_point(void* h, const double* Uq, int iz, double* F, double* G, double* lam) {
  Ctx* c = (Ctx*)h;
  Point<double> q;
  pointwise(*c, Uq, iz, q);
  for (int j = 0; j < c->d; ++j) {
    for (int v = 0; v < c->nvars; ++v) F[j * c->nvars + v] = q.F[j][v];
    lam[j] = q.lam[j];
  }
  for (int v = 0; v < c->nvars; ++v) G[v] = q.G[v];
}

// Lax-Friedrichs flux with normal +e_j between the states Um (node height
// izm) and Up (izp)
void ora_face(void* h, const double* Um, int izm, const double* Up, int izp, int j, double* Fs) {
  Ctx* c = (Ctx*)h;
  Point<double> a, b;
  pointwise(*c, Um, izm, a);
  pointwise(*c, Up, izp, b);
  lf_flux(*c, a, Um, b, Up, j, Fs);
}

// The diffusive term alone, -M^{-1} A_h(U, .), with the viscosity taken from
// the velocities of the state W (Lobatto basis, sip_gamma > 0)
int ora_sip(void* h, const double* U, const double* W, double* out) {
  Ctx* c = (Ctx*)h;
  if (c->basis != 0 || !(c->P.sip_gamma > 0.0)) return -1;
  const long N = (long)c->ne * c->np;
  std::vector<Point<double>> q(N);
  std::vector<double> Wq(c->nvars);
  for (int e = 0; e < c->ne; ++e)
    for (int n = 0; n < c->np; ++n) {
      for (int v = 0; v < c->nvars; ++v) Wq[v] = W[(long)v * N + (long)e * c->np + n];
      pointwise(*c, Wq.data(), height_of(*c, e, n), q[(long)e * c->np + n]);
    }
  std::vector<double> an[2];
  sip_alpha(*c, q, an);
  std::fill(out, out + N * c->nvars, 0.0);
  sip_add(*c, U, out, an);
  return 0;
}

// The nodal viscosity of Section 3.5 from the velocities of the state W
// (Lobatto basis, sip_gamma > 0): a0 for every variable but rho_r, a1 for
// rho_r, one value per node in W's node order
int ora_sip_alpha(void* h, const double* W, double* a0, double* a1) {
  Ctx* c = (Ctx*)h;
  if (c->basis != 0 || !(c->P.sip_gamma > 0.0)) return -1;
  const long N = (long)c->ne * c->np;
  std::vector<Point<double>> q(N);
  std::vector<double> Wq(c->nvars);
  for (int e = 0; e < c->ne; ++e)
    for (int n = 0; n < c->np; ++n) {
      for (int v = 0; v < c->nvars; ++v) Wq[v] = W[(long)v * N + (long)e * c->np + n];
      pointwise(*c, Wq.data(), height_of(*c, e, n), q[(long)e * c->np + n]);
    }
  std::vector<double> an[2];
  sip_alpha(*c, q, an);
  std::copy(an[0].begin(), an[0].end(), a0);
  std::copy(an[1].begin(), an[1].end(), a1);
  return 0;
}

// Threads of the element loops (OpenMP); n < 1 restores the default.
void ora_set_threads(int n) { omp_set_num_threads(n > 0 ? n : omp_get_num_procs()); }
int ora_get_threads(void) { return omp_get_max_threads(); }

// Legendre coefficients (the L2 projection by the Gauss rule) of a state given
// at the Gauss points; modal basis only
int ora_project(void* h, const double* U, double* C) {
  Ctx* c = (Ctx*)h;
  if (c->basis != 1) return -1;
  to_modal(*c, c->nvars, U, C);
  return 0;
}

void ora_stats(void* h, long* iters_total, int* max_iters, int* bad) {
  Ctx* c = (Ctx*)h;
  *iters_total = c->iters_total; *max_iters = c->max_iters; *bad = c->bad;
}

}  // extern "C"

// ===========================================================================
// Triangles (Section 3.1: the space P^k on a simplicial mesh)
// ===========================================================================
// A conforming triangulation in the vertical (x, z) plane, every element an
// affine image x = V0 + A (r, s) of the unit triangle {r, s >= 0, r + s <= 1}
// with counter-clockwise vertices V0, V1, V2, so det A > 0.  Face f joins V_f
// and V_{f+1 mod 3}; the mesh supplies, per face, the neighbouring element
// and its face (periodic pairs included), or -1 for a slip wall.  Two
// counter-clockwise triangles run along their shared edge in opposite
// directions.
//
//  * basis: the orthonormal Dubiner basis, the Legendre-Jacobi products of the
//    collapsed coordinates, so the element mass matrix is det A times the
//    identity (Section 3.1; diagonal mass);
//  * volume rule: the footnote of Section 3.4, a product of Gauss-Legendre
//    rules, k+1 points across and k+2 points up, carried onto the triangle by
//    the Duffy map (exact for total degree 2k+1, as the k+1 point rule on an
//    interval);
//  * faces: the (k+1)-point Gauss-Legendre rule on every edge;
//  * the split runs at the volume points; T and rho_v are L2-projected onto P^k
//    and the fluxes and sources are assembled with the projected fields at
//    every quadrature point (Section 3.4);
//  * the background depends on height only.  It is given, like that of the box
//    meshes with the Gauss basis, at the Gauss heights of n_z uniform layers;
//    its pressure is the equation of state of its split there.  An element
//    belongs to the layer that holds its centroid, and at every point of the
//    element (volume and face points alike) each background field is the
//    degree-k interpolant of that layer (so a triangulation whose rows are the
//    layers sees a P^k background on every element).
// Coefficients are stored C[v][e][m], mode m running over p = 0..k and, for
// each p, q = 0..k-p.
namespace {

// Jacobi polynomial P_n^{(al,be)}(x), three-term recurrence
template <class R> R jacobi(int n, double al, double be, R x) {
  if (n == 0) return R(1.0);
  R p0 = R(1.0);
  R p1 = 0.5 * ((al - be) + (al + be + 2.0) * x);
  for (int m = 2; m <= n; ++m) {
    const double c = 2.0 * m + al + be;
    const double a1 = 2.0 * m * (m + al + be) * (c - 2.0);
    const double a2 = (c - 1.0) * (al * al - be * be);
    const double a3 = (c - 1.0) * c * (c - 2.0);
    const double a4 = 2.0 * (m + al - 1.0) * (m + be - 1.0) * c;
    R p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

inline int tri_np(int k) { return (k + 1) * (k + 2) / 2; }

// Every basis function at (r, s):
//   psi_pq = N_pq t^p P_p((2r - t)/t) P_q^{(2p+1,0)}(2s - 1),  t = 1 - s,
// with t^p P_p((2r - t)/t) by the Legendre recurrence multiplied through by
// t^(m+1) (no division by t) and N_pq^2 = 2 (2p+1) (p+q+1), the inverse of
// the squared norm on the unit triangle.
template <class R> void tri_basis(int k, R r, R s, R* psi) {
  R t = 1.0 - s, X = 2.0 * r - t;
  R L[16];
  L[0] = R(1.0);
  if (k >= 1) L[1] = X;
  for (int m = 1; m < k; ++m) L[m + 1] = ((2.0 * m + 1.0) * X * L[m] - (double)m * t * t * L[m - 1]) / (m + 1.0);
  int i = 0;
  for (int p = 0; p <= k; ++p)
    for (int q = 0; p + q <= k; ++q)
      psi[i++] = std::sqrt(2.0 * (2 * p + 1) * (p + q + 1)) * L[p] * jacobi(q, 2.0 * p + 1.0, 0.0, 2.0 * s - 1.0);
}

// values and reference gradients (d/dr, d/ds), the derivatives by forward mode
void tri_basis_grad(int k, double r, double s, double* psi, double* dr, double* ds) {
  Dual a[136], b[136];
  tri_basis(k, Dual(r, 1.0), Dual(s, 0.0), a);
  tri_basis(k, Dual(r, 0.0), Dual(s, 1.0), b);
  for (int m = 0; m < tri_np(k); ++m) {
    psi[m] = a[m].v;
    if (dr) dr[m] = a[m].d;
    if (ds) ds[m] = b[m].d;
  }
}

// The Duffy-mapped product rule: a in [-1, 1] across (k+1 Gauss points), b in
// [-1, 1] up (k+2 points); s = (1 + b)/2, r = (1 + a)(1 - s)/2 and
// dr ds = (1 - s)/4 da db.  Point q = j (k+1) + i for a_i, b_j.
struct TriRule {
  std::vector<double> r, s, w;
};

TriRule tri_volume_rule(int k) {
  Gauss ga = make_gauss(k), gb = make_gauss(k + 1);
  TriRule R;
  for (int j = 0; j < k + 2; ++j)
    for (int i = 0; i < k + 1; ++i) {
      const double s = 0.5 * (1.0 + gb.x[j]);
      R.s.push_back(s);
      R.r.push_back(0.5 * (1.0 + ga.x[i]) * (1.0 - s));
      R.w.push_back(ga.w[i] * gb.w[j] * (1.0 - s) / 4.0);
    }
  return R;
}

const double kRefV[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};

struct TriCtx {
  Ctx base;                  // parameters, dimension 2 and the variable count
  int k, np, nq, nf, ne;
  std::vector<double> xy;    // ne x 3 vertices x (x, z)
  std::vector<int> nb, nbf;  // ne x 3
  TriRule vol;
  Gauss gf;                  // k+1 points: faces and background layers
  std::vector<double> psi_q, dr_q, ds_q;   // [q*np + m]
  std::vector<double> psi_f;               // [(f*nf + i)*np + m]
  double z0, dz;
  int nz;
  std::vector<double> bgl[5];              // rho_d, rho_m, rho_r, E, p at the layer heights
};

struct TriGeom {
  double V[3][2];
  double det;
  double G[2][2];        // A^{-T}: grad_x = G grad_(r,s)
  double n[3][2], len[3];
};

TriGeom tri_geom(const TriCtx& c, int e) {
  TriGeom g;
  for (int v = 0; v < 3; ++v)
    for (int a = 0; a < 2; ++a) g.V[v][a] = c.xy[(size_t)e * 6 + 2 * v + a];
  const double a00 = g.V[1][0] - g.V[0][0], a01 = g.V[2][0] - g.V[0][0];
  const double a10 = g.V[1][1] - g.V[0][1], a11 = g.V[2][1] - g.V[0][1];
  g.det = a00 * a11 - a01 * a10;
  // A^{-1} = [a11 -a01; -a10 a00] / det, and G = A^{-T}
  g.G[0][0] = a11 / g.det;  g.G[0][1] = -a10 / g.det;
  g.G[1][0] = -a01 / g.det; g.G[1][1] = a00 / g.det;
  for (int f = 0; f < 3; ++f) {
    const double dx = g.V[(f + 1) % 3][0] - g.V[f][0], dzz = g.V[(f + 1) % 3][1] - g.V[f][1];
    g.len[f] = std::sqrt(dx * dx + dzz * dzz);
    // outward normal of a counter-clockwise triangle: the edge turned clockwise
    g.n[f][0] = dzz / g.len[f];
    g.n[f][1] = -dx / g.len[f];
  }
  return g;
}

double tri_z(const TriGeom& g, double r, double s) {
  return g.V[0][1] + (g.V[1][1] - g.V[0][1]) * r + (g.V[2][1] - g.V[0][1]) * s;
}

// the layer that holds height z
int tri_layer_of(const TriCtx& c, double z) {
  int l = (int)std::floor((z - c.z0) / c.dz);
  return std::max(0, std::min(l, c.nz - 1));
}

// the layer of an element: that of its centroid
int tri_layer(const TriCtx& c, const TriGeom& g) {
  return tri_layer_of(c, (g.V[0][1] + g.V[1][1] + g.V[2][1]) / 3.0);
}

// background (rho_d, rho_m, rho_r, E, p) at height z: the Lagrange interpolant
// through the Gauss heights of layer l
void tri_bg(const TriCtx& c, int l, double z, double* out) {
  const int p1 = c.k + 1;
  const double xi = 2.0 * (z - c.z0 - l * c.dz) / c.dz - 1.0;
  double ell[16];
  for (int i = 0; i < p1; ++i) {
    ell[i] = 1.0;
    for (int j = 0; j < p1; ++j)
      if (j != i) ell[i] *= (xi - c.gf.x[j]) / (c.gf.x[i] - c.gf.x[j]);
  }
  for (int f = 0; f < 5; ++f) {
    double v = 0.0;
    for (int i = 0; i < p1; ++i) v += ell[i] * c.bgl[f][(size_t)l * p1 + i];
    out[f] = v;
  }
}

template <class R> R tri_expand(const R* cm, const double* psi, int np) {
  R v = R(0.0);
  for (int m = 0; m < np; ++m) v += cm[m] * psi[m];
  return v;
}

// the state U' of element e at a point with basis values psi
template <class R> void tri_state_at(const TriCtx& c, const R* C, int e, const double* psi, R* Ut) {
  const long N = (long)c.ne * c.np;
  for (int v = 0; v < c.base.nvars; ++v) Ut[v] = tri_expand(C + (long)v * N + (long)e * c.np, psi, c.np);
}

// the split of the full state at a point (Section 2.2): T and rho_v
template <class R> void tri_split_point(const TriCtx& c, const R* Ut, const double* b, R* T, R* rv,
                                        SplitStats* st) {
  const Ctx& x = c.base;
  const OraParams& P = x.P;
  R rd = b[0] + Ut[v_rd()];
  R rm = b[1] + Ut[v_rm()];
  R rr = P.rain ? R(b[2]) + Ut[v_rr(x)] : R(0.0);
  R rho = rd + rm + rr;
  R ke = R(0.0);
  for (int i = 0; i < 2; ++i) {
    R mi = Ut[v_m(x, i)];
    ke += 0.5 * mi * (mi / rho);
  }
  R re = (b[3] + Ut[v_E(x)]) - ke;
  int ok = 1, iters = 0;
  split(P, rd, rm, rr, re, T, rv, &ok, &iters);
  st->iters_total += iters;
  st->max_iters = std::max(st->max_iters, iters);
  if (!ok) st->bad++;
}

// Lax-Friedrichs flux along the unit normal n (Section 3.2):
// {F}.n + Lambda/2 (U- - U+), Lambda the larger of |u.n| + |v_r n_z| + c_m
template <class R> void tri_lf(const TriCtx& c, const Point<R>& a, const R* Ua, const Point<R>& b,
                               const R* Ub, const double* n, R* Fs) {
  const int nv = c.base.nvars;
  R la = absr(a.u[0] * n[0] + a.u[1] * n[1]) + absr(a.vr * n[1]) + a.cm;
  R lb = absr(b.u[0] * n[0] + b.u[1] * n[1]) + absr(b.vr * n[1]) + b.cm;
  R L = max_minus(la, lb);
  for (int v = 0; v < nv; ++v)
    Fs[v] = 0.5 * ((a.F[0][v] + b.F[0][v]) * n[0] + (a.F[1][v] + b.F[1][v]) * n[1]) + 0.5 * L * (Ua[v] - Ub[v]);
}

// T_h and rho_v,h: the split at the volume points, L2-projected onto P^k
// (orthonormal basis: c_m = sum_q w_q psi_m(q) f(q), det A cancels)
template <class R> void tri_project_split(TriCtx& c, const R* C, R* Tc, R* Rvc) {
  const int np = c.np, nq = c.nq, nv = c.base.nvars;
  SplitStats tot;
#pragma omp parallel
  {
    SplitStats st;
    std::vector<R> Ut(nv), Tq(nq), Rq(nq);
#pragma omp for schedule(static)
    for (int e = 0; e < c.ne; ++e) {
      TriGeom g = tri_geom(c, e);
      for (int q = 0; q < nq; ++q) {
        double b[5];
        tri_bg(c, tri_layer(c, g), tri_z(g, c.vol.r[q], c.vol.s[q]), b);
        tri_state_at(c, C, e, &c.psi_q[(size_t)q * np], Ut.data());
        tri_split_point(c, Ut.data(), b, &Tq[q], &Rq[q], &st);
      }
      for (int m = 0; m < np; ++m) {
        R a = R(0.0), r = R(0.0);
        for (int q = 0; q < nq; ++q) {
          a += (c.vol.w[q] * c.psi_q[(size_t)q * np + m]) * Tq[q];
          r += (c.vol.w[q] * c.psi_q[(size_t)q * np + m]) * Rq[q];
        }
        Tc[(long)e * np + m] = a;
        Rvc[(long)e * np + m] = r;
      }
    }
#pragma omp critical
    {
      tot.iters_total += st.iters_total;
      tot.max_iters = std::max(tot.max_iters, st.max_iters);
      tot.bad += st.bad;
    }
  }
  c.base.iters_total += tot.iters_total;
  c.base.max_iters = std::max(c.base.max_iters, tot.max_iters);
  c.base.bad += tot.bad;
}

// Everything the flux needs at a point of element e (geometry g) with basis
// values psi: U', the projected T and rho_v, and the background at height z.
template <class R> void tri_point(const TriCtx& c, const R* C, const R* Tc, const R* Rvc, int e,
                                  const TriGeom& g, const double* psi, double z, R* Ut, Point<R>& q,
                                  double* b) {
  tri_state_at(c, C, e, psi, Ut);
  R T = tri_expand(Tc + (long)e * c.np, psi, c.np);
  R rv = tri_expand(Rvc + (long)e * c.np, psi, c.np);
  tri_bg(c, tri_layer(c, g), z, b);
  point_core(c.base, Ut, T, rv, b[0], b[1], c.base.P.rain ? b[2] : 0.0, b[3], b[4], q);
}

// dC/dt (Section 3.2 weak form; Section 3.3 diagonal mass; Section 3.4
// reconstruction), element by element:
//   det A dC_m/dt = det A sum_q w_q (F . grad psi_m + G psi_m)(x_q)
//                   - sum_f |e_f| sum_i (w_i / 2) F_n(x_fi) psi_m(x_fi),
// F_n the Lax-Friedrichs flux along the element's outward normal; the
// neighbour's trace at x_fi is its face point k - i.
template <class R> void tri_rhs(TriCtx& c, const R* C, R* dC, double* wall_rain_flux) {
  const int np = c.np, nq = c.nq, nf = c.nf, nv = c.base.nvars, k = c.k;
  const long N = (long)c.ne * np;
  std::vector<R> Tc(N), Rvc(N);
  tri_project_split(c, C, Tc.data(), Rvc.data());
  std::vector<double> wflux(c.ne, 0.0);
#pragma omp parallel
  {
    std::vector<R> Ut(nv), Un(nv), Ug(nv), Fs(nv), acc((size_t)nv * np);
#pragma omp for schedule(static)
    for (int e = 0; e < c.ne; ++e) {
      TriGeom g = tri_geom(c, e);
      std::fill(acc.begin(), acc.end(), R(0.0));
      // volume: flux against the physical gradient, sources against psi
      for (int q = 0; q < nq; ++q) {
        const double* psi = &c.psi_q[(size_t)q * np];
        Point<R> pt;
        double b[5];
        tri_point(c, C, Tc.data(), Rvc.data(), e, g, psi, tri_z(g, c.vol.r[q], c.vol.s[q]), Ut.data(), pt, b);
        for (int m = 0; m < np; ++m) {
          const double gr = c.dr_q[(size_t)q * np + m], gs = c.ds_q[(size_t)q * np + m];
          const double gx = g.G[0][0] * gr + g.G[0][1] * gs;
          const double gz = g.G[1][0] * gr + g.G[1][1] * gs;
          for (int v = 0; v < nv; ++v)
            acc[(size_t)v * np + m] += c.vol.w[q] * (pt.F[0][v] * gx + pt.F[1][v] * gz + pt.G[v] * psi[m]);
        }
      }
      // faces
      for (int f = 0; f < 3; ++f) {
        const int e2 = c.nb[(size_t)e * 3 + f], f2 = c.nbf[(size_t)e * 3 + f];
        for (int i = 0; i < nf; ++i) {
          const double t = 0.5 * (1.0 + c.gf.x[i]);
          const double r = kRefV[f][0] + t * (kRefV[(f + 1) % 3][0] - kRefV[f][0]);
          const double s = kRefV[f][1] + t * (kRefV[(f + 1) % 3][1] - kRefV[f][1]);
          const double z = tri_z(g, r, s);
          const double* psi = &c.psi_f[((size_t)f * nf + i) * np];
          Point<R> pm, pp;
          double bm[5], bp[5];
          tri_point(c, C, Tc.data(), Rvc.data(), e, g, psi, z, Ut.data(), pm, bm);
          if (e2 < 0) {
            // slip wall: m+ = m- - 2 (m-.n) n, every other component and the
            // reconstructed T, rho_v copied
            for (int v = 0; v < nv; ++v) Ug[v] = Ut[v];
            R mn = Ut[v_m(c.base, 0)] * g.n[f][0] + Ut[v_m(c.base, 1)] * g.n[f][1];
            for (int a = 0; a < 2; ++a) Ug[v_m(c.base, a)] = Ut[v_m(c.base, a)] - 2.0 * mn * g.n[f][a];
            point_core(c.base, Ug.data(), pm.T, pm.rv, bm[0], bm[1], c.base.P.rain ? bm[2] : 0.0, bm[3], bm[4], pp);
            tri_lf(c, pm, Ut.data(), pp, Ug.data(), g.n[f], Fs.data());
            if (c.base.P.rain) wflux[e] += g.len[f] * 0.5 * c.gf.w[i] * val(Fs[v_rr(c.base)]);
          } else {
            // the neighbour's own trace at the same physical point
            const double* psi2 = &c.psi_f[((size_t)f2 * nf + (k - i)) * np];
            TriGeom g2 = tri_geom(c, e2);
            const double t2 = 0.5 * (1.0 + c.gf.x[k - i]);
            const double r2 = kRefV[f2][0] + t2 * (kRefV[(f2 + 1) % 3][0] - kRefV[f2][0]);
            const double s2 = kRefV[f2][1] + t2 * (kRefV[(f2 + 1) % 3][1] - kRefV[f2][1]);
            tri_point(c, C, Tc.data(), Rvc.data(), e2, g2, psi2, tri_z(g2, r2, s2), Un.data(), pp, bp);
            tri_lf(c, pm, Ut.data(), pp, Un.data(), g.n[f], Fs.data());
          }
          const double wf = g.len[f] * 0.5 * c.gf.w[i] / g.det;
          for (int m = 0; m < np; ++m)
            for (int v = 0; v < nv; ++v) acc[(size_t)v * np + m] -= (wf * psi[m]) * Fs[v];
        }
      }
      for (int v = 0; v < nv; ++v)
        for (int m = 0; m < np; ++m) dC[(long)v * N + (long)e * np + m] = acc[(size_t)v * np + m];
    }
  }
  if (wall_rain_flux) {
    double s = 0.0;
    for (int e = 0; e < c.ne; ++e) s += wflux[e];
    *wall_rain_flux = s;
  }
}

}  // namespace

extern "C" {

struct OraTriMesh {
  int ne;
  const double* xy;   // ne x 3 x 2: counter-clockwise vertices (x, z)
  const int* nb;      // ne x 3: element across face f (V_f to V_f+1), -1 = slip wall
  const int* nbf;     // ne x 3: that element's face index
  int order;
  // background layers: n_z layers of height dz from z0
  double z0, dz;
  int nz;
};

// the unit-triangle volume rule: (r, s) pairs and weights, (k+1)(k+2) points
int ora_tri_rule(int k, double* rs, double* w) {
  if (k < 1 || k > 8) return -1;
  TriRule R = tri_volume_rule(k);
  for (size_t q = 0; q < R.w.size(); ++q) {
    rs[2 * q] = R.r[q];
    rs[2 * q + 1] = R.s[q];
    w[q] = R.w[q];
  }
  return (int)R.w.size();
}

// every basis function and its reference gradient at n points (r, s):
// psi[i*np + m], dr[i*np + m], ds[i*np + m]
int ora_tri_basis(int k, const double* rs, int n, double* psi, double* dr, double* ds) {
  if (k < 1 || k > 8) return -1;
  const int np = tri_np(k);
  for (int i = 0; i < n; ++i)
    tri_basis_grad(k, rs[2 * i], rs[2 * i + 1], psi + (size_t)i * np, dr ? dr + (size_t)i * np : nullptr,
                   ds ? ds + (size_t)i * np : nullptr);
  return np;
}

// A triangulation, its tables and its background (rho_d, rho_m, rho_r, E at
// the n_z (k+1) Gauss heights of the layers, lowest layer first).
void* ora_tri_create(const OraTriMesh* M, const OraParams* P, int nvars, const double* rd,
                     const double* rm, const double* rr, const double* E) {
  if (M->order < 1 || M->order > 8 || M->ne < 1 || M->nz < 1 || !(M->dz > 0.0)) return nullptr;
  if (nvars != (P->rain ? 6 : 5)) return nullptr;
  if (P->sip_gamma > 0.0 || P->sponge_alpha > 0.0) return nullptr;   // not on triangles
  TriCtx* c = new TriCtx();
  c->base.P = *P;
  c->base.d = 2;
  c->base.nvars = nvars;
  c->base.k = M->order;
  c->k = M->order;
  c->np = tri_np(c->k);
  c->ne = M->ne;
  c->base.ne = M->ne;
  c->base.np = c->np;
  c->xy.assign(M->xy, M->xy + (size_t)M->ne * 6);
  c->nb.assign(M->nb, M->nb + (size_t)M->ne * 3);
  c->nbf.assign(M->nbf, M->nbf + (size_t)M->ne * 3);
  for (int e = 0; e < c->ne; ++e) {
    if (!(tri_geom(*c, e).det > 0.0)) { delete c; return nullptr; }
    for (int f = 0; f < 3; ++f) {
      const int e2 = c->nb[(size_t)e * 3 + f], f2 = c->nbf[(size_t)e * 3 + f];
      if (e2 >= c->ne || (e2 >= 0 && (f2 < 0 || f2 > 2 || c->nb[(size_t)e2 * 3 + f2] != e))) { delete c; return nullptr; }
    }
  }
  c->vol = tri_volume_rule(c->k);
  c->nq = (int)c->vol.w.size();
  c->gf = make_gauss(c->k);
  c->nf = c->k + 1;
  c->psi_q.resize((size_t)c->nq * c->np);
  c->dr_q.resize((size_t)c->nq * c->np);
  c->ds_q.resize((size_t)c->nq * c->np);
  for (int q = 0; q < c->nq; ++q)
    tri_basis_grad(c->k, c->vol.r[q], c->vol.s[q], &c->psi_q[(size_t)q * c->np], &c->dr_q[(size_t)q * c->np],
                   &c->ds_q[(size_t)q * c->np]);
  c->psi_f.resize((size_t)3 * c->nf * c->np);
  for (int f = 0; f < 3; ++f)
    for (int i = 0; i < c->nf; ++i) {
      const double t = 0.5 * (1.0 + c->gf.x[i]);
      const double r = kRefV[f][0] + t * (kRefV[(f + 1) % 3][0] - kRefV[f][0]);
      const double s = kRefV[f][1] + t * (kRefV[(f + 1) % 3][1] - kRefV[f][1]);
      tri_basis_grad(c->k, r, s, &c->psi_f[((size_t)f * c->nf + i) * c->np], nullptr, nullptr);
    }
  c->z0 = M->z0; c->dz = M->dz; c->nz = M->nz;
  const int nzq = M->nz * (c->k + 1);
  c->bgl[0].assign(rd, rd + nzq);
  c->bgl[1].assign(rm, rm + nzq);
  c->bgl[2].assign(nzq, 0.0);
  if (P->rain) c->bgl[2].assign(rr, rr + nzq);
  c->bgl[3].assign(E, E + nzq);
  c->bgl[4].assign(nzq, 0.0);
  for (int iz = 0; iz < nzq; ++iz) {
    SplitOut s = split_double(*P, rd[iz], rm[iz], c->bgl[2][iz], E[iz]);
    c->bgl[4][iz] = (rd[iz] * P->Rd + s.rv * P->Rv) * s.T;
  }
  return c;
}

void ora_tri_destroy(void* h) { delete (TriCtx*)h; }

// physical coordinates of the volume points, xz[(e*nq + q)*2 + a]
void ora_tri_points(void* h, double* xz) {
  TriCtx* c = (TriCtx*)h;
  for (int e = 0; e < c->ne; ++e) {
    TriGeom g = tri_geom(*c, e);
    for (int q = 0; q < c->nq; ++q)
      for (int a = 0; a < 2; ++a)
        xz[((size_t)e * c->nq + q) * 2 + a] = g.V[0][a] + (g.V[1][a] - g.V[0][a]) * c->vol.r[q]
                                              + (g.V[2][a] - g.V[0][a]) * c->vol.s[q];
  }
}

// L2 projection onto P^k of nfields fields given at the volume points:
// vals[(f*ne + e)*nq + q] -> C[(f*ne + e)*np + m]
void ora_tri_project(void* h, const double* vals, int nfields, double* C) {
  TriCtx* c = (TriCtx*)h;
  for (long b = 0; b < (long)nfields * c->ne; ++b)
    for (int m = 0; m < c->np; ++m) {
      double s = 0.0;
      for (int q = 0; q < c->nq; ++q) s += c->vol.w[q] * c->psi_q[(size_t)q * c->np + m] * vals[b * c->nq + q];
      C[b * c->np + m] = s;
    }
}

// nfields fields C evaluated at n reference points of every element:
// out[(f*ne + e)*n + i]
void ora_tri_eval(void* h, const double* C, int nfields, const double* rs, int n, double* out) {
  TriCtx* c = (TriCtx*)h;
  std::vector<double> psi((size_t)n * c->np);
  for (int i = 0; i < n; ++i) tri_basis_grad(c->k, rs[2 * i], rs[2 * i + 1], &psi[(size_t)i * c->np], nullptr, nullptr);
  for (long b = 0; b < (long)nfields * c->ne; ++b)
    for (int i = 0; i < n; ++i) out[b * n + i] = tri_expand(C + b * c->np, &psi[(size_t)i * c->np], c->np);
}

// background (rho_d, rho_m, rho_r, E, p) at height z (the layer that holds z)
void ora_tri_background(void* h, double z, double* out5) {
  TriCtx* c = (TriCtx*)h;
  tri_bg(*c, tri_layer_of(*c, z), z, out5);
}

// T_h and rho_v,h coefficients of a state (Section 3.4 reconstruction)
int ora_tri_split(void* h, const double* C, double* Tc, double* Rvc) {
  TriCtx* c = (TriCtx*)h;
  int bad = c->base.bad;
  tri_project_split(*c, C, Tc, Rvc);
  return c->base.bad - bad;
}

int ora_tri_rhs(void* h, const double* C, double* dC, double* wall_rain_flux) {
  TriCtx* c = (TriCtx*)h;
  int bad = c->base.bad;
  tri_rhs(*c, C, dC, wall_rain_flux);
  return c->base.bad - bad;
}

// nsteps steps of size dt in place; outflow as for the box meshes
int ora_tri_rk_step(void* h, double* C, double dt, int nsteps, int scheme, double* outflow) {
  TriCtx* c = (TriCtx*)h;
  int bad = c->base.bad;
  double acc = 0.0;
  for (int s = 0; s < nsteps; ++s) {
    double f = 0.0;
    ssprk((long)c->ne * c->np * c->base.nvars, C, dt, scheme,
          [&](const double* u, double* L, double* fl) { tri_rhs(*c, u, L, fl); }, &f);
    acc += f;
  }
  if (outflow) *outflow = acc;
  return c->base.bad - bad;
}

// M_d = int rho_d', M_w = int (rho_m' + rho_r') and the wall rain flux
void ora_tri_mass(void* h, const double* C, double* out3) {
  TriCtx* c = (TriCtx*)h;
  const long N = (long)c->ne * c->np;
  double md = 0.0, mw = 0.0;
  for (int e = 0; e < c->ne; ++e) {
    const double det = tri_geom(*c, e).det;
    for (int q = 0; q < c->nq; ++q) {
      const double* psi = &c->psi_q[(size_t)q * c->np];
      md += det * c->vol.w[q] * tri_expand(C + (long)e * c->np, psi, c->np);
      mw += det * c->vol.w[q] * (tri_expand(C + N + (long)e * c->np, psi, c->np)
                                 + (c->base.P.rain ? tri_expand(C + 2 * N + (long)e * c->np, psi, c->np) : 0.0));
    }
  }
  out3[0] = md;
  out3[1] = mw;
  std::vector<double> dC(N * c->base.nvars);
  double f = 0.0;
  tri_rhs(*c, C, dC.data(), &f);
  out3[2] = f;
}

// Lax-Friedrichs flux along the unit normal n between the states Um and Up,
// both split at height z
void ora_tri_face(void* h, const double* Um, const double* Up, double z, const double* n, double* Fs) {
  TriCtx* c = (TriCtx*)h;
  double b[5];
  tri_bg(*c, tri_layer_of(*c, z), z, b);
  Point<double> a, bb;
  SplitStats st;
  double T, rv;
  tri_split_point(*c, Um, b, &T, &rv, &st);
  point_core(c->base, Um, T, rv, b[0], b[1], c->base.P.rain ? b[2] : 0.0, b[3], b[4], a);
  tri_split_point(*c, Up, b, &T, &rv, &st);
  point_core(c->base, Up, T, rv, b[0], b[1], c->base.P.rain ? b[2] : 0.0, b[3], b[4], bb);
  tri_lf(*c, a, Um, bb, Up, n, Fs);
}

void ora_tri_stats(void* h, long* iters_total, int* max_iters, int* bad) {
  TriCtx* c = (TriCtx*)h;
  *iters_total = c->base.iters_total; *max_iters = c->base.max_iters; *bad = c->base.bad;
}

}  // extern "C"
