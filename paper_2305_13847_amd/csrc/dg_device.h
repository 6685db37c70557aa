// Device code of libdgmoist: the pointwise implicit-condensation split, the
// pointwise state/flux/source evaluation and the fused right-hand-side kernel.
//
// Precision: the split (Newton on the implicit condensation system of
// Section 2.2), the reconstruction of full densities, p' = p - p_bar and
// rho e from the stored perturbations are always FP64.  Fluxes, the
// sum-factorised volume contraction, face fluxes, sources and the stage
// update run in the state's precision R (double, or float in FP32-bulk mode)
// with accumulation in R.
#pragma once
#include "dg_common.h"

namespace dgm {

template <int D, int RAIN>
struct Vars {
  static constexpr int NV = 3 + D + RAIN;
  static constexpr int RD = 0, RM = 1, RR = 2, M0 = 2 + RAIN, E = NV - 1;
};

template <int K, int D>
struct Shape {
  static constexpr int P1 = K + 1;
  static constexpr int NP = (D == 2) ? P1 * P1 : P1 * P1 * P1;
  static constexpr int EPB = (256 / NP) > 0 ? 256 / NP : 1;   // elements per block
  static constexpr int NT = EPB * NP;                          // threads per block
};

// ---------------------------------------------------------------------------
// saturation vapour density and the split (FP64)
// ---------------------------------------------------------------------------
// rho_vs(T) = e_s(T) / (R_v T) with the Clausius-Clapeyron e_s of Section 2.1,
// written as one exponential: C0 exp((a - 1) ln(T/T_ref) + b (1/T_ref - 1/T)).
__device__ __forceinline__ double rho_vs(const KArgs& a, double T) {
  return a.C0 * exp(a.am1 * log(T * a.inv_Tref) + a.b * (a.inv_Tref - 1.0 / T));
}

struct SplitOut {
  double T;     // temperature
  double rvs;   // rho_vs(T); rho_v = min(rvs, rho_m)
  int iters;    // Newton iterations (0 when unsaturated)
  int bad;      // 1: no valid temperature, 2: iteration cap reached
};

// Implicit condensation (Section 2.2): find T with
//   rho e = (c_vd rd + c_vv rv + c_l (rm - rv + rr)) (T - T_ref) + rv (L_ref - R_v T_ref),
//   rv = min(rho_vs(T), rm).
// The all-vapour temperature Tu decides the branch exactly.  On the saturated
// branch f(T) is increasing and convex, so Newton from any start at or above
// the root's lower bound converges; iterates are kept above that bound.
__device__ __forceinline__ SplitOut split_point(const KArgs& a, double rd, double rm, double rr,
                                                double re, double guess) {
  SplitOut o;
  o.iters = 0;
  o.bad = 0;
  const double Cu = a.cvd * rd + a.cvv * rm + a.cl * rr;
  const double Tu = a.Tref + (re - rm * a.Lp) / Cu;
  if (!isfinite(Tu) || !(Cu > 0.0)) {
    o.T = Tu; o.rvs = rm; o.bad = 1;
    return o;
  }
  if (Tu > 0.0) {
    const double r = rho_vs(a, Tu);
    if (rm <= r) { o.T = Tu; o.rvs = r; return o; }
  }
  const double dc = a.cvv - a.cl;
  double lo = Tu;
  if (!(Tu > 50.0)) {
    const double r = rho_vs(a, 50.0);
    const double f = (Cu + dc * (r - rm)) * (50.0 - a.Tref) + r * a.Lp - re;
    if (!(f < 0.0)) { o.T = Tu; o.rvs = rm; o.bad = 1; return o; }
    lo = 50.0;
  }
  double T = (guess > lo && guess < 1.0e4) ? guess : lo;
  double rvs = 0.0;
  int it = 0;
  bool conv = false;
  while (it < a.maxit) {
    const double inv = 1.0 / T;
    rvs = a.C0 * exp(a.am1 * log(T * a.inv_Tref) + a.b * (a.inv_Tref - inv));
    const double Cv = Cu + dc * (rvs - rm);
    const double Tm = T - a.Tref;
    const double f = Cv * Tm + rvs * a.Lp - re;
    const double drvs = rvs * (a.am1 + a.b * inv) * inv;
    const double fp = Cv + drvs * (dc * Tm + a.Lp);
    const double dT = -f / fp;
    ++it;
    if (fabs(dT) <= a.rtol * T) {
      T += dT;
      rvs += drvs * dT;          // first-order update; the step is below rounding
      conv = true;
      break;
    }
    double Tn = T + dT;
    if (!(Tn > lo)) Tn = 0.5 * (T + lo);
    T = Tn;
  }
  if (!conv) {
    rvs = rho_vs(a, T);
    o.bad = 2;
  }
  o.T = T;
  o.rvs = rvs;
  o.iters = it;
  return o;
}

// Accumulate split statistics of a whole block into the status words.
template <int NT>
__device__ __forceinline__ void record_stats(const KArgs& a, int iters, int bad, bool active) {
  __shared__ int s_max, s_nc, s_bad, s_cnt;
  if (threadIdx.x == 0) { s_max = 0; s_nc = 0; s_bad = 0; s_cnt = 0; }
  __syncthreads();
  if (active) {
    if (iters > 0) atomicMax(&s_max, iters);
    if (bad == 2) atomicAdd(&s_nc, 1);
    if (bad == 1) atomicOr(&s_bad, 1);
    atomicAdd(&s_cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_max) atomicMax(&a.stats[0], (unsigned)s_max);
    if (s_nc) atomicAdd(&a.stats[1], (unsigned)s_nc);
    if (s_bad) atomicOr(&a.stats[2], 1u);
    if (s_cnt) atomicAdd((unsigned long long*)&a.stats[4], (unsigned long long)s_cnt);
  }
}

// ---------------------------------------------------------------------------
// pointwise state, fluxes, wave speed and sources
// ---------------------------------------------------------------------------
template <typename R, int D, int RAIN>
struct Pt {
  R m[D], u[D];
  R rd, rm, rr;     // full densities
  R rho;            // total density
  R H;              // E + p_bar + p'
  R pp;             // p'
  R cm;             // moist sound speed
  R vr;             // terminal rain speed
  R rrvr;           // rho_r v_r
  R rain_e;         // (c_l (T - T_ref) + u.u/2) rho_r v_r
  R rc, dvs, Tm;    // rho_c, rho_vs(T) - rho_v, T - T_ref (rain only)
};

// Full state from the stored perturbation U at vertical index iz and the
// split result (T, rho_vs(T)).  The reconstruction is FP64.
template <typename R, int D, int RAIN>
__device__ __forceinline__ void eval_point(const KArgs& a, const R* Uq, double T, double rvs, int iz,
                                           Pt<R, D, RAIN>& q) {
  using V = Vars<D, RAIN>;
  const double rd = a.bg_rd[iz] + (double)Uq[V::RD];
  const double rm = a.bg_rm[iz] + (double)Uq[V::RM];
  const double rr = RAIN ? a.bg_rr[iz] + (double)Uq[V::RR] : 0.0;
  const double rv = fmin(rvs, rm);
  const double rc = rm - rv;
  const double gasR = rd * a.Rd + rv * a.Rv;
  const double p = gasR * T;
  const double ppd = p - a.bg_p[iz];
  const double rho = rd + rm + rr;
  const double Cv = a.cvd * rd + a.cvv * rv + a.cl * (rc + rr);
  q.rd = (R)rd; q.rm = (R)rm; q.rr = (R)rr; q.rho = (R)rho;
  q.pp = (R)ppd;
  q.H = (R)(a.bg_E[iz] + a.bg_p[iz] + (double)Uq[V::E] + ppd);
  R uu = R(0);
  for (int i = 0; i < D; ++i) {
    q.m[i] = Uq[V::M0 + i];
    q.u[i] = q.m[i] / q.rho;
    uu += q.u[i] * q.u[i];
  }
  const R gam = R(1) + (R)gasR / (R)Cv;
  q.cm = sqrt(gam * (R)p / q.rho);
  if (RAIN) {
    if (a.vr_mode == 0) q.vr = (R)a.vr_const;
    else q.vr = (R)a.vr_pref * (rr > 0.0 ? (R)pow(rr, 0.125) : R(0));
    q.rrvr = q.rr * q.vr;
    q.rain_e = ((R)(a.cl * (T - a.Tref)) + R(0.5) * uu) * q.rrvr;
    q.rc = (R)rc;
    q.dvs = (R)(rvs - rv);
    q.Tm = (R)(T - a.Tref);
  } else {
    q.vr = R(0); q.rrvr = R(0); q.rain_e = R(0);
    q.rc = R(0); q.dvs = R(0); q.Tm = R(0);
  }
}

// Physical flux in direction j (Section 2.3 perturbation form).
template <typename R, int D, int RAIN, int J>
__device__ __forceinline__ void flux(const Pt<R, D, RAIN>& q, R* F) {
  using V = Vars<D, RAIN>;
  constexpr bool VERT = (J == D - 1);
  const R uj = q.u[J];
  F[V::RD] = q.rd * uj;
  F[V::RM] = q.rm * uj;
  if (RAIN) F[V::RR] = VERT ? q.rr * uj - q.rrvr : q.rr * uj;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    R f = q.m[i] * uj;
    if (i == J) f += q.pp;
    if (RAIN && VERT) f -= q.rrvr * q.u[i];
    F[V::M0 + i] = f;
  }
  F[V::E] = (RAIN && VERT) ? q.H * uj - q.rain_e : q.H * uj;
}

template <typename R, int D, int RAIN, int J>
__device__ __forceinline__ R wave_speed(const Pt<R, D, RAIN>& q) {
  R l = fabs(q.u[J]) + q.cm;
  if (RAIN && J == D - 1) l += fabs(q.vr);
  return l;
}

// Slip-wall ghost (Section 3.2): momentum reflected in the wall normal e_j.
template <typename R, int D, int RAIN, int J>
__device__ __forceinline__ void reflect(Pt<R, D, RAIN>& q) {
  q.m[J] = -q.m[J];
  q.u[J] = -q.u[J];
}

// Sources: gravity on the vertical momentum and the energy (Section 2.3),
// Kessler warm rain (Section 2.1) moving mass between rho_m and rho_r.
template <typename R, int D, int RAIN>
__device__ __forceinline__ void sources(const KArgs& a, const R* Uq, const Pt<R, D, RAIN>& q, R* G) {
  using V = Vars<D, RAIN>;
  R rhop = Uq[V::RD] + Uq[V::RM];
  if (RAIN) rhop += Uq[V::RR];
  G[V::M0 + D - 1] -= rhop * (R)a.g;
  G[V::E] -= q.rho * (R)a.g * q.u[D - 1];
  if (RAIN) {
    const R rrp = q.rr > R(0) ? q.rr : R(0);
    R p316 = R(0), p12 = R(0), p78 = R(0);
    if (rrp > R(0)) {
      p316 = pow(rrp, R(0.1875));
      p12 = sqrt(rrp);
      p78 = pow(rrp, R(0.875));
    }
    const R Sev = (R(3.86e-3) - R(9.41e-5) * q.Tm) * (R(1) + R(9.1) * p316) * q.dvs * p12;
    const R au = q.rc - (R)a.q_au * q.rho;
    const R Sau = au > R(0) ? R(1e-3) * au : R(0);
    const R Sac = R(1.72) * q.rc * p78;
    const R S = Sev - Sau - Sac;
    G[V::RM] += S;
    G[V::RR] -= S;
  }
}

}  // namespace dgm
