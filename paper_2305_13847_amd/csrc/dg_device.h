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

// Threads per block: 256 in FP32; 128 in FP64, where the LDS tiles are twice
// as large and 256-thread blocks would leave room for only two per CU.
template <typename R>
constexpr int block_threads() { return sizeof(R) == 4 ? 256 : 128; }

template <int K, int D, int BT = 256>
struct Shape {
  static constexpr int P1 = K + 1;
  static constexpr int NP = (D == 2) ? P1 * P1 : P1 * P1 * P1;
  static constexpr int EPB = (BT / NP) > 0 ? BT / NP : 1;   // elements per block
  static constexpr int NT = EPB * NP;                          // threads per block
};

// ---------------------------------------------------------------------------
// per-variable device arrays through buffer resources
// ---------------------------------------------------------------------------
// One 128-bit descriptor (base address, byte size, raw 32-bit data format)
// per array, built with scalar instructions; accesses take a 32-bit byte
// offset, so no 64-bit address arithmetic per load, and the hardware drops
// accesses past the end (reads return 0).  Array byte sizes stay below 4 GiB
// (the handle limits its node count accordingly).
constexpr int kRawBufferWord3 = 0x00020000;

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const T* base, unsigned n) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(n * (unsigned)sizeof(T)), kRawBufferWord3);
}

__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, unsigned i, float*) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, i * 4u, 0, 0));
}
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, unsigned i, double*) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8u, 0, 0));
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned i, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, i * 4u, 0, 0);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned i, double v) {
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, i * 8u, 0, 0);
}

// element i of variable v of an SoA state (v-major, n nodes per variable)
template <typename T>
__device__ __forceinline__ T ld(const T* base, unsigned n, int v, unsigned i) {
  return buf_load(buf_rsrc(base + (size_t)v * n, n), i, (T*)nullptr);
}
template <typename T>
__device__ __forceinline__ void st(T* base, unsigned n, int v, unsigned i, T x) {
  buf_store(buf_rsrc(base + (size_t)v * n, n), i, x);
}

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

// rho_vs near an anchor temperature T0 where r0 = rho_vs(T0) is known:
//   rho_vs(T) = r0 exp(phi(T) - phi(T0)),
//   phi(T) - phi(T0) = (a - 1) log(1 + x) + b x / (T0 (1 + x)),  x = (T - T0)/T0,
// with log(1 + x), 1/(1 + x) and exp(.) - 1 summed as Taylor series.  For
// |x| <= kAnchorX the truncation errors are below 1e-19 relative (|x|^8/8,
// |x|^8 and |dphi|^11/11! with |dphi| < 0.09 for T0 >= 200 K).
constexpr double kAnchorX = 2.0e-3;

struct Anchor {
  double T0, r0, inv0;
};

__device__ __forceinline__ Anchor make_anchor(const KArgs& a, double T) {
  Anchor A;
  A.T0 = T;
  A.inv0 = 1.0 / T;
  A.r0 = a.C0 * exp(a.am1 * log(T * a.inv_Tref) + a.b * (a.inv_Tref - A.inv0));
  return A;
}

__device__ __forceinline__ bool in_anchor(const Anchor& A, double T) {
  return fabs(T - A.T0) <= kAnchorX * A.T0;
}

// Between two stages T moves by far less than the anchor range, and for
// |x| <= kShortX shorter series suffice (anchors lie above 150 K, so
// b / T0 < 46): log(1 + x) to x^4 (error |x|^5/5 < 3e-21), 1/(1 + x) to x^3
// (error x^4 = 1e-16, entering d multiplied by b x / T0 < 5e-3) and
// exp(d) - 1 to d^5 (|d| < 5.2e-3, error d^6/720 < 3e-17).  The choice is
// made per wavefront.
constexpr double kShortX = 1.0e-4;

// rho_vs(T) and d rho_vs / dT from the anchor
__device__ __forceinline__ double rvs_near(const KArgs& a, const Anchor& A, double T, double* drvs) {
  const double x = (T - A.T0) * A.inv0;
  double l, q, e;
  if (__all(x == 0.0)) {
    // at the anchor itself (the first step of a warm-started solve): the
    // series below give exactly these values for x = 0
    *drvs = A.r0 * (a.am1 + a.b * A.inv0) * A.inv0;
    return A.r0;
  }
  if (__all(fabs(x) <= kShortX)) {
    l = x * (1.0 + x * (-0.5 + x * (1.0 / 3.0 - x * 0.25)));
    q = 1.0 + x * (-1.0 + x * (1.0 - x));
    const double d = a.am1 * l + a.b * A.inv0 * x * q;
    e = d * (1.0 + d * (1.0 / 2 + d * (1.0 / 6 + d * (1.0 / 24 + d * (1.0 / 120)))));
  } else {
    l = x * (1.0 + x * (-0.5 + x * (1.0 / 3.0 + x * (-0.25 + x * (0.2 + x * (-1.0 / 6.0 + x * (1.0 / 7.0)))))));
    q = 1.0 + x * (-1.0 + x * (1.0 + x * (-1.0 + x * (1.0 + x * (-1.0 + x * (1.0 - x))))));
    const double d = a.am1 * l + a.b * A.inv0 * x * q;
    e = d * (1.0 + d * (1.0 / 2 + d * (1.0 / 6 + d * (1.0 / 24 + d * (1.0 / 120 + d * (1.0 / 720 +
        d * (1.0 / 5040 + d * (1.0 / 40320 + d * (1.0 / 362880 + d * (1.0 / 3628800))))))))));
  }
  const double r = A.r0 + A.r0 * e;
  const double invT = A.inv0 * q;
  *drvs = r * (a.am1 + a.b * invT) * invT;
  return r;
}

// FP64 reciprocal: hardware estimate refined by two Newton steps
__device__ __forceinline__ double rcp64(double v) {
  double r = __builtin_amdgcn_rcp(v);
  r = fma(fma(-v, r, 1.0), r, r);
  r = fma(fma(-v, r, 1.0), r, r);
  return r;
}

// Implicit condensation (Section 2.2): find T with
//   rho e = (c_vd rd + c_vv rv + c_l (rm - rv + rr)) (T - T_ref) + rv (L_ref - R_v T_ref),
//   rv = min(rho_vs(T), rm).
// The map T -> rho e is strictly increasing, so the root is unique.  Each
// branch gives a candidate and an exact test:
//   unsaturated: T = Tu (all water as vapour), valid iff rm <= rho_vs(Tu);
//   saturated:   the root Ts of f(T) = rho e(T, rv = rho_vs(T)) - rho e,
//                valid iff rho_vs(Ts) <= rm (then Ts is the unique root).
// `sat_first` names the branch to try first (with a warm start, the branch
// that held before), so a node normally evaluates one branch.  On the
// saturated branch f is increasing and convex; Newton evaluates rho_vs by
// series around an anchor that is re-based when an iterate leaves its range.
// The Newton step uses the hardware reciprocal of f' (relative error far
// below the step's own size, so convergence stays quadratic).  Stopping:
// |dT| <= rtol T, or, above 150 K, the quadratic-convergence bound: after a
// step dT the error is at most M dT^2 with M = max |f''| / (2 min f').  With
// f' >= rho_vs' L_eff and f'' <= rho_vs'' L_eff (the c_vv - c_l term is below
// 2e-3 of it), M <= (q + q'/q)/2 + 2e-3 with q = d ln rho_vs / dT, which is
// 0.15 K^-1 at 150 K and falls with T; M = 0.25 K^-1 is used, so
// |dT| <= sqrt(rtol T / M) already leaves an error below rtol T.
// If `A` holds a valid anchor (A.T0 > 0) it is used and updated in place.
struct NewtonOut {
  double T, rvs;
  int iters;
  int state;   // 0 converged, 1 root lies below Tu (not saturated), 2 iteration cap
};

__device__ __forceinline__ NewtonOut newton_sat(const KArgs& a, double Cu, double rm, double re,
                                                double Tu, double lo, double T, Anchor& A) {
  const double dc = a.cvv - a.cl;
  if (!(A.T0 > 0.0) || !in_anchor(A, T)) A = make_anchor(a, T);
  // |dT| <= tol with tol = rtol T, or above 150 K max(rtol T, 2 sqrt(rtol T)),
  // compared as squares
  const double tol_lin = a.rtol * T;
  const double tol2 = T > 150.0 ? fmax(tol_lin * tol_lin, 4.0 * tol_lin) : tol_lin * tol_lin;
  NewtonOut o;
  o.state = 2;
  double rvs = 0.0;
  int it = 0;
  while (it < a.maxit) {
    if (!in_anchor(A, T)) A = make_anchor(a, T);
    double drvs;
    rvs = rvs_near(a, A, T, &drvs);
    const double Cv = Cu + dc * (rvs - rm);
    const double Tm = T - a.Tref;
    const double f = Cv * Tm + rvs * a.Lp - re;
    const double fp = Cv + drvs * (dc * Tm + a.Lp);
    const double dT = -f * __builtin_amdgcn_rcp(fp);
    ++it;
    if (dT * dT <= tol2) {
      T += dT;
      rvs += drvs * dT;          // first order is exact to rounding for this step size
      o.state = 0;
      break;
    }
    double Tn = T + dT;
    if (!(Tn > lo)) {
      // f is convex: from the right of the root Newton never overshoots, so a
      // step below the bound means the saturated root lies below Tu
      if (f > 0.0 && lo == Tu) { o.state = 1; break; }
      Tn = 0.5 * (T + lo);
    }
    T = Tn;
  }
  o.T = T;
  o.rvs = rvs;
  o.iters = it;
  return o;
}

__device__ __forceinline__ SplitOut split_point_anchor(const KArgs& a, double rd, double rm, double rr,
                                                       double re, double guess, Anchor& A,
                                                       bool sat_first = false) {
  SplitOut o;
  o.iters = 0;
  o.bad = 0;
  const double Cu = a.cvd * rd + a.cvv * rm + a.cl * rr;
  const double Tu = a.Tref + (re - rm * a.Lp) * rcp64(Cu);
  if (!isfinite(Tu) || !(Cu > 0.0)) {
    o.T = __builtin_nan(""); o.rvs = rm; o.bad = 1;
    return o;
  }
  // unsaturated test
  bool unsat = false;
  double rTu = 0.0;
  if (!sat_first && Tu > 0.0) {
    double dr;
    rTu = (A.T0 > 0.0 && in_anchor(A, Tu)) ? rvs_near(a, A, Tu, &dr) : rho_vs(a, Tu);
    unsat = rm <= rTu;
  }
  if (!unsat) {
    // saturated branch: Newton from the warm start if it lies above the
    // branch's lower bound max(Tu, 50 K)
    double lo = Tu;
    if (!(Tu > 50.0)) {
      const double r = rho_vs(a, 50.0);
      const double f = (Cu + (a.cvv - a.cl) * (r - rm)) * (50.0 - a.Tref) + r * a.Lp - re;
      if (!(f < 0.0)) { o.T = __builtin_nan(""); o.rvs = rm; o.bad = 1; return o; }
      lo = 50.0;
    }
    const double T0 = (guess > lo && guess < 600.0) ? guess : lo;
    const NewtonOut n = newton_sat(a, Cu, rm, re, Tu, lo, T0, A);
    o.iters = n.iters;
    if (n.state == 2) { o.T = n.T; o.rvs = rho_vs(a, n.T); o.bad = 2; return o; }
    if (n.state == 0 && (n.rvs <= rm || !(Tu > 0.0))) { o.T = n.T; o.rvs = n.rvs; return o; }
    // the saturated root is not a solution: the air is unsaturated
    if (!sat_first) { o.T = Tu; o.rvs = rm; return o; }   // ties at the branch point
    rTu = rho_vs(a, Tu);
  }
  o.T = Tu;
  o.rvs = rTu;
  return o;
}

__device__ __forceinline__ SplitOut split_point(const KArgs& a, double rd, double rm, double rr,
                                                double re, double guess) {
  Anchor A;
  A.T0 = 0.0; A.r0 = 0.0; A.inv0 = 0.0;
  return split_point_anchor(a, rd, rm, rr, re, guess, A);
}

// Status words: only exceptional events touch global memory.  Iteration
// maxima are merged per wave and written only when they exceed the stored
// value; counts of non-converged or invalid states are rare.
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ void record_stats(const KArgs& a, int iters, int bad) {
  const int m = wave_max(iters);
  const int anybad = wave_max(bad);
  const int lane = threadIdx.x & 63;
  if (lane == 0) {
    if (m > 0 && (unsigned)m > __builtin_nontemporal_load(&a.stats[0])) atomicMax(&a.stats[0], (unsigned)m);
  }
  if (anybad) {
    if (bad == 2) atomicAdd(&a.stats[1], 1u);
    if (bad == 1) atomicOr(&a.stats[2], 1u);
  }
}

// ---------------------------------------------------------------------------
// pointwise state, fluxes, wave speed and sources
// ---------------------------------------------------------------------------
// reciprocal and fractional power in the bulk precision: hardware
// reciprocal/log2/exp2 in FP32 (about 1 ulp), refined or library forms in FP64
__device__ __forceinline__ float inv_b(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double inv_b(double x) { return rcp64(x); }
__device__ __forceinline__ float pow_b(float x, float p) {
  return __builtin_amdgcn_exp2f(p * __builtin_amdgcn_logf(x));
}
__device__ __forceinline__ double pow_b(double x, double p) { return pow(x, p); }

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

// Full state from the perturbation Uq, the temperature T, the vapour density
// rho_v and the background (rho_d, rho_m, rho_r, E, p) at the point; rho_vs
// enters only the evaporation source.  The reconstruction is FP64.
template <typename R, int D, int RAIN>
__device__ __forceinline__ void eval_core(const KArgs& a, const R* Uq, double T, double rv, double rvs,
                                          double bd, double bm, double br, double bE, double bp,
                                          Pt<R, D, RAIN>& q) {
  using V = Vars<D, RAIN>;
  const double rd = bd + (double)Uq[V::RD];
  const double rm = bm + (double)Uq[V::RM];
  const double rr = RAIN ? br + (double)Uq[V::RR] : 0.0;
  const double rc = rm - rv;
  const double gasR = rd * a.Rd + rv * a.Rv;
  const double p = gasR * T;
  const double ppd = p - bp;
  const double rho = rd + rm + rr;
  const double Cv = a.cvd * rd + a.cvv * rv + a.cl * (rc + rr);
  q.rd = (R)rd; q.rm = (R)rm; q.rr = (R)rr; q.rho = (R)rho;
  q.pp = (R)ppd;
  q.H = (R)(bE + bp + (double)Uq[V::E] + ppd);
  R uu = R(0);
  const R irho = inv_b(q.rho);
  for (int i = 0; i < D; ++i) {
    q.m[i] = Uq[V::M0 + i];
    q.u[i] = q.m[i] * irho;
    uu += q.u[i] * q.u[i];
  }
  const R gam = R(1) + (R)gasR * inv_b((R)Cv);
  q.cm = sqrt(gam * (R)p * irho);
  if (RAIN) {
    if (a.vr_mode == 0) q.vr = (R)a.vr_const;
    else q.vr = (R)a.vr_pref * (rr > 0.0 ? pow_b((R)rr, R(0.125)) : R(0));
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

// Full state at a node from the stored perturbation U at vertical index iz and
// the split result (T, rho_vs(T)): rho_v = min(rho_vs, rho_m).
template <typename R, int D, int RAIN>
__device__ __forceinline__ void eval_point(const KArgs& a, const R* Uq, double T, double rvs, int iz,
                                           Pt<R, D, RAIN>& q) {
  using V = Vars<D, RAIN>;
  const double rm = a.bg_rm[iz] + (double)Uq[V::RM];
  const double rv = fmin(rvs, rm);
  eval_core<R, D, RAIN>(a, Uq, T, rv, rvs, a.bg_rd[iz], a.bg_rm[iz], RAIN ? a.bg_rr[iz] : 0.0, a.bg_E[iz],
                        a.bg_p[iz], q);
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
      p316 = pow_b(rrp, R(0.1875));
      p12 = sqrt(rrp);
      p78 = pow_b(rrp, R(0.875));
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
