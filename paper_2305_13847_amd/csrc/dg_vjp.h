// Adjoint kernels of libdgmoist: vector-Jacobian products of the right-hand
// side, of the implicit-condensation split and of an SSP-RK stage.
//
// The pointwise reverse pass recomputes the forward quantities of one node in
// FP64 and propagates adjoints back through the fluxes, the wave speed, the
// sources, the equation of state and the split.  The split's derivative is
// the implicit-function derivative of the root (Section 2.2 system):
//   saturated:   f(T; rd, rm, rr, re) = 0  =>  dT = -(df/dtheta) dtheta / f_T,
//                rho_v = rho_vs(T);
//   unsaturated: T = T_ref + (re - rm (L - R_v T_ref)) / (c_vd rd + c_vv rm + c_l rr),
//                rho_v = rm.
// At kinks the active branch is differentiated: ties of the split go to the
// unsaturated branch, ties of the face maximum to the minus side, sign(0) = 0,
// and clamps at zero have derivative 0 there.
#pragma once
#include "dg_kernels.h"

namespace dgm {

// Adjoint seeds of one node's pointwise outputs.
template <int D, int RAIN>
struct PwSeed {
  double F[D][Vars<D, RAIN>::NV];   // physical fluxes per direction
  double lam[D];                    // wave speeds |u_j| + |v_r e_z.e_j| + c_m
  double G[Vars<D, RAIN>::NV];      // sources
};

template <int D, int RAIN>
__device__ __forceinline__ void seed_zero(PwSeed<D, RAIN>& s) {
  constexpr int NV = Vars<D, RAIN>::NV;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    s.lam[j] = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) s.F[j][v] = 0.0;
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) s.G[v] = 0.0;
}

// Reverse pass of the split: adjoints (Tb, rvb) of (T, rho_v) -> adjoints of
// (rd, rm, rr, re), added to the outputs.  `sat` is the branch of the forward
// split; T and rvs = rho_vs(T) come from it.
__device__ __forceinline__ void split_reverse(const KArgs& a, bool sat, double rd, double rm, double rr,
                                              double T, double rvs, double Tb, double rvb,
                                              double& rdb, double& rmb, double& rrb, double& reb) {
  const double Tm = T - a.Tref;
  if (!sat) {
    const double Cu = a.cvd * rd + a.cvv * rm + a.cl * rr;
    const double t = Tb / Cu;
    reb += t;
    rmb += t * (-a.Lp - a.cvv * Tm) + rvb;
    rdb += -t * a.cvd * Tm;
    rrb += -t * a.cl * Tm;
    return;
  }
  const double dc = a.cvv - a.cl;
  const double Cv = a.cvd * rd + a.cvv * rvs + a.cl * (rm - rvs + rr);
  const double drvs = rvs * (a.am1 + a.b / T) / T;
  const double fT = Cv + drvs * (dc * Tm + a.Lp);
  const double tt = (Tb + rvb * drvs) / fT;
  reb += tt;
  rdb += -tt * a.cvd * Tm;
  rmb += -tt * a.cl * Tm;
  rrb += -tt * a.cl * Tm;
}

// Pointwise reverse pass of one node: seeds on (F_j, lambda_j, G) -> U_bar.
// `Uq` is the node's stored state, (T, rvs) its forward split, iz its height.
template <typename R, int D, int RAIN>
__device__ __forceinline__ void pointwise_vjp(const KArgs& a, const R* Uq, double T, double rvs, int iz,
                                              const PwSeed<D, RAIN>& sd, double* Ub) {
  using V = Vars<D, RAIN>;
  constexpr int NV = V::NV;
  constexpr int Z = D - 1;
  // forward recomputation (FP64)
  const double rd = a.bg_rd[iz] + (double)Uq[V::RD];
  const double rm = a.bg_rm[iz] + (double)Uq[V::RM];
  const double rr = RAIN ? a.bg_rr[iz] + (double)Uq[V::RR] : 0.0;
  const double rho = rd + rm + rr;
  double m[D], u[D], uu = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    m[i] = (double)Uq[V::M0 + i];
    u[i] = m[i] / rho;
    uu += u[i] * u[i];
  }
  const double E = a.bg_E[iz] + (double)Uq[V::E];
  const bool sat = rvs < rm;
  const double rv = sat ? rvs : rm;
  const double rc = rm - rv;
  const double Rg = rd * a.Rd + rv * a.Rv;
  const double p = Rg * T;
  const double pp = p - a.bg_p[iz];
  const double Cv = a.cvd * rd + a.cvv * rv + a.cl * (rc + rr);
  const double gam = 1.0 + Rg / Cv;
  const double c2 = gam * p / rho;
  const double cm = sqrt(c2);
  const double H = E + p;
  const double Tm = T - a.Tref;
  double vr = 0.0;
  if (RAIN) vr = (a.vr_mode == 0) ? a.vr_const : (rr > 0.0 ? a.vr_pref * pow(rr, 0.125) : 0.0);
  const double X = a.cl * Tm + 0.5 * uu;            // rain energy factor
  // adjoint accumulators
  double rdb = 0, rmb = 0, rrb = 0, rhob = 0, Eb = 0, Tb = 0, rvb = 0, ppb = 0, Hb = 0, cmb = 0, vrb = 0;
  double mb[D], ub[D];
#pragma unroll
  for (int i = 0; i < D; ++i) { mb[i] = 0.0; ub[i] = 0.0; }
  // fluxes
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const bool vert = (j == Z);
    const double* Fb = sd.F[j];
    rdb += Fb[V::RD] * u[j];
    ub[j] += Fb[V::RD] * rd;
    rmb += Fb[V::RM] * u[j];
    ub[j] += Fb[V::RM] * rm;
    if (RAIN) {
      rrb += Fb[V::RR] * (u[j] - (vert ? vr : 0.0));
      ub[j] += Fb[V::RR] * rr;
      if (vert) vrb -= Fb[V::RR] * rr;
    }
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double fb = Fb[V::M0 + i];
      mb[i] += fb * u[j];
      ub[j] += fb * m[i];
      if (i == j) ppb += fb;
      if (RAIN && vert) {
        rrb -= fb * vr * u[i];
        vrb -= fb * rr * u[i];
        ub[i] -= fb * rr * vr;
      }
    }
    const double fe = Fb[V::E];
    Hb += fe * u[j];
    ub[j] += fe * H;
    if (RAIN && vert) {
      Tb -= fe * a.cl * rr * vr;
#pragma unroll
      for (int i = 0; i < D; ++i) ub[i] -= fe * u[i] * rr * vr;
      rrb -= fe * X * vr;
      vrb -= fe * X * rr;
    }
    // wave speed |u_j| + v_r [j vertical] + c_m
    const double lb = sd.lam[j];
    ub[j] += lb * (u[j] > 0.0 ? 1.0 : (u[j] < 0.0 ? -1.0 : 0.0));
    if (RAIN && vert) vrb += lb;
    cmb += lb;
  }
  // sources: gravity
  {
    const double gz = sd.G[V::M0 + Z];
    rdb -= gz * a.g;   // rho' = rho_d' + rho_m' + rho_r'
    rmb -= gz * a.g;
    if (RAIN) rrb -= gz * a.g;
    const double ge = sd.G[V::E];
    rhob -= ge * a.g * u[Z];
    ub[Z] -= ge * rho * a.g;
  }
  // Kessler
  if (RAIN) {
    const double Sb = sd.G[V::RM] - sd.G[V::RR];
    const double rrp = rr > 0.0 ? rr : 0.0;
    const double dvs = rvs - rv;                    // 0 on the saturated branch
    double rrpb = 0.0, rcb = 0.0, dvsb = 0.0;
    if (rrp > 0.0) {
      const double Aev = 3.86e-3 - 9.41e-5 * Tm;
      const double p316 = pow(rrp, 0.1875), p12 = sqrt(rrp), p78 = pow(rrp, 0.875);
      const double Bev = 1.0 + 9.1 * p316;
      Tb += Sb * (-9.41e-5) * Bev * dvs * p12;
      dvsb += Sb * Aev * Bev * p12;
      rrpb += Sb * Aev * dvs * (9.1 * 0.1875 * p316 / rrp * p12 + Bev * 0.5 / p12);
      // accretion
      rcb -= Sb * 1.72 * p78;
      rrpb -= Sb * 1.72 * rc * 0.875 * p78 / rrp;
    }
    if (rc - a.q_au * rho > 0.0) {                    // autoconversion
      rcb -= Sb * 1e-3;
      rhob += Sb * 1e-3 * a.q_au;
    }
    if (rr > 0.0) rrb += rrpb;
    if (!sat) {                                       // dvs = rho_vs(T) - rm
      Tb += dvsb * rvs * (a.am1 + a.b / T) / T;
      rmb -= dvsb;
    }
    rmb += rcb;
    rvb -= rcb;
    if (a.vr_mode != 0 && rr > 0.0) rrb += vrb * vr * 0.125 / rr;
  }
  // H = E + p, p' = p - p_bar
  Eb += Hb;
  double pb = Hb + ppb;
  // c_m = sqrt(gamma p / rho), gamma = 1 + Rg / Cv
  {
    const double c2b = cmb * 0.5 / cm;
    const double gb = c2b * p / rho;
    pb += c2b * gam / rho;
    rhob -= c2b * c2 / rho;
    const double Rgb = gb / Cv;
    const double Cvb = -gb * Rg / (Cv * Cv);
    rdb += Rgb * a.Rd + Cvb * a.cvd;
    rvb += Rgb * a.Rv + Cvb * (a.cvv - a.cl);
    rmb += Cvb * a.cl;
    rrb += Cvb * a.cl;
  }
  // p = (rd R_d + rv R_v) T
  rdb += pb * a.Rd * T;
  rvb += pb * a.Rv * T;
  Tb += pb * Rg;
  // u_i = m_i / rho
#pragma unroll
  for (int i = 0; i < D; ++i) {
    mb[i] += ub[i] / rho;
    rhob -= ub[i] * u[i] / rho;
  }
  // split: (rd, rm, rr, re) -> (T, rv)
  double reb = 0.0;
  split_reverse(a, sat, rd, rm, rr, T, rvs, Tb, rvb, rdb, rmb, rrb, reb);
  // re = E - |m|^2 / (2 rho)
  Eb += reb;
#pragma unroll
  for (int i = 0; i < D; ++i) mb[i] -= reb * u[i];
  rhob += reb * 0.5 * uu;
  // rho = rd + rm + rr
  rdb += rhob;
  rmb += rhob;
  if (RAIN) rrb += rhob;
  Ub[V::RD] += rdb;
  Ub[V::RM] += rmb;
  if (RAIN) Ub[V::RR] += rrb;
#pragma unroll
  for (int i = 0; i < D; ++i) Ub[V::M0 + i] += mb[i];
  Ub[V::E] += Eb;
}

// ---------------------------------------------------------------------------
// adjoint of the right-hand side
// ---------------------------------------------------------------------------
// One face of the node in direction J: accumulate the node's seeds and the
// direct (jump-term) adjoint.  lam_o / lam_n: adjoint of dU/dt at this node and
// at the neighbour's matching node.  For a wall the ghost's own pointwise
// reverse pass is added to Ub with the reflected momentum.
template <typename R, int K, int D, int RAIN, int J>
__device__ __forceinline__ void face_vjp(const KArgs& a, const MemberDesc& md, int ij, int iz,
                                         const R* Uq, const Pt<R, D, RAIN>& q, double T, double rvs,
                                         const Nb<R, D, RAIN>& nb, const R* lam_o, const R* lam_n,
                                         bool wall, int izn_off, PwSeed<D, RAIN>& sd, double* Ub) {
  using V = Vars<D, RAIN>;
  constexpr int NV = V::NV;
  const bool plus = (ij == K);     // own node on its +J face: own side is K-
  const double lK = md.two_over_h[J] / a.w[K], l0 = md.two_over_h[J] / a.w[0];
  double Fsb[NV];                  // adjoint of the face flux F*
  R Un[NV];
  Pt<R, D, RAIN> qn;
  if (wall) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Un[v] = Uq[v];
      Fsb[v] = plus ? -lK * (double)lam_o[v] : l0 * (double)lam_o[v];
    }
    Un[V::M0 + J] = -Uq[V::M0 + J];
    qn = q;
    reflect<R, D, RAIN, J>(qn);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Un[v] = nb.U[v];
      // R(K-) -= lK F*, R(K+) += l0 F*
      Fsb[v] = plus ? (-lK * (double)lam_o[v] + l0 * (double)lam_n[v])
                    : (-lK * (double)lam_n[v] + l0 * (double)lam_o[v]);
    }
    const int izn = (J == D - 1) ? md.hoff + izn_off : iz;
    eval_point<R, D, RAIN>(a, Un, nb.T, nb.rvs, izn, qn);
  }
  const double lo = (double)wave_speed<R, D, RAIN, J>(q);
  const double ln = (double)wave_speed<R, D, RAIN, J>(qn);
  // F* = (F(U-) + F(U+)).n / 2 + Lambda (U- - U+) / 2, Lambda = max(l-, l+),
  // ties to the minus side
  const bool own_sel = plus ? (lo >= ln) : (lo > ln);
  const double Lam = own_sel ? lo : ln;
  double jump_dot = 0.0;           // Fsb . (U- - U+)
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double d = plus ? ((double)Uq[v] - (double)Un[v]) : ((double)Un[v] - (double)Uq[v]);
    jump_dot += Fsb[v] * d;
  }
  // the node's own flux and (if selected) its wave speed
#pragma unroll
  for (int v = 0; v < NV; ++v) sd.F[J][v] += 0.5 * Fsb[v];
  // jump term: +Lambda/2 on U-, -Lambda/2 on U+
  const double sgn = plus ? 0.5 : -0.5;
#pragma unroll
  for (int v = 0; v < NV; ++v) Ub[v] += sgn * Lam * Fsb[v];
  if (wall) {
    // the ghost g(U) reverses the normal momentum: the jump term's ghost part
    // maps back through g (R = dg/dU), giving -sgn Lambda R Fsb
    sd.lam[J] += 0.5 * jump_dot;           // Lambda = l(U) = l(g(U)) identically
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double rf = (v == V::M0 + J) ? -Fsb[v] : Fsb[v];
      Ub[v] -= sgn * Lam * rf;
    }
    // ghost flux F(g(U)): pointwise reverse at the ghost state, reflected back
    PwSeed<D, RAIN> gs;
    seed_zero<D, RAIN>(gs);
#pragma unroll
    for (int v = 0; v < NV; ++v) gs.F[J][v] = 0.5 * Fsb[v];
    double Ug[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Ug[v] = 0.0;
    pointwise_vjp<R, D, RAIN>(a, Un, T, rvs, iz, gs, Ug);
    Ug[V::M0 + J] = -Ug[V::M0 + J];
#pragma unroll
    for (int v = 0; v < NV; ++v) Ub[v] += Ug[v];
  } else if (own_sel) {
    sd.lam[J] += 0.5 * jump_dot;
  }
}

template <typename R, int K, int D, int RAIN>
__global__ void __launch_bounds__(256)
rhs_vjp_kernel(KArgs a, const R* __restrict__ U, const double* __restrict__ auxT,
               const double* __restrict__ auxS, const R* __restrict__ lam, R* __restrict__ out,
               const R* __restrict__ X1, const R* __restrict__ X2, const double* __restrict__ dt_m,
               double cx1, double cx2, double c1, double c2) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NP = S::NP, NV = V::NV;
  __shared__ R sL[NV * S::NT];
  __shared__ R sD[P1 * P1];
  const int NT = blockDim.x;
  const int t = threadIdx.x;
  if (t < P1 * P1) sD[t] = (R)a.Dhat[t];
  const ItemWalk walk(a.nitems);
  for (int kk = 0;; ++kk) {
  const int it_ = walk.item(kk);
  if (it_ < 0) break;
  __syncthreads();   // sL of the previous item is no longer read
  const Item item = a.items[it_];
  const MemberDesc& md = a.mem[item.member];
  const int le = t / NP, n = t - le * NP;
  const int e = item.e0 + le;
  const bool active = e < md.ne;
  const unsigned N = a.nnodes;
  const unsigned g = (unsigned)(md.eoff + (active ? e : 0)) * NP + n;
  const ElemCoord<D> ec = item_coord<D>(md, item, active ? le : 0);
  int idx[3];
  idx[0] = n % P1;
  idx[1] = (n / P1) % P1;
  idx[2] = (D == 3) ? n / (P1 * P1) : 0;
  const int iz = md.hoff + ec.c[D - 1] * P1 + idx[D - 1];
  R Uq[NV], Lq[NV];
  double T = 300.0, rvs = 0.0;
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Uq[v] = (U + (size_t)v * N)[g];
      Lq[v] = (lam + (size_t)v * N)[g];
    }
    T = auxT[g];
    rvs = auxS[g];
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) { Uq[v] = R(0); Lq[v] = R(0); }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) sL[v * NT + t] = Lq[v];
  __syncthreads();
  if (!active) continue;
  Pt<R, D, RAIN> q;
  eval_point<R, D, RAIN>(a, Uq, T, rvs, iz, q);
  PwSeed<D, RAIN> sd;
  seed_zero<D, RAIN>(sd);
  double Ub[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Ub[v] = 0.0;
  // volume: transposed contraction, Fbar_J(own) = (2/h_J) sum_a Dhat[a][i_J] lam(node a)
#pragma unroll
  for (int J = 0; J < D; ++J) {
    const int str = (J == 0) ? 1 : (J == 1 ? P1 : P1 * P1);
    const int ij = idx[J];
    const int base = t - ij * str;
    const double s = md.two_over_h[J];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double acc = 0.0;
#pragma unroll
      for (int b = 0; b < P1; ++b) acc += (double)sD[b * P1 + ij] * (double)sL[v * NT + base + b * str];
      sd.F[J][v] += s * acc;
    }
  }
  // faces
#pragma unroll
  for (int J = 0; J < D; ++J) {
    const int ij = idx[J];
    if (ij != 0 && ij != K) continue;
    Nb<R, D, RAIN> nb;
    bool wall = false;
    int zoff = -1;
    R Ln[NV];
    if (J == 0) gather_nb<R, K, D, RAIN, 0>(md, ec, e, n, ij, U, auxT, auxS, N, nb, wall, zoff);
    else if (J == 1) gather_nb<R, K, D, RAIN, 1>(md, ec, e, n, ij, U, auxT, auxS, N, nb, wall, zoff);
    else gather_nb<R, K, D, RAIN, (D == 3 ? 2 : 0)>(md, ec, e, n, ij, U, auxT, auxS, N, nb, wall, zoff);
    if (!wall) {
      // the neighbour's matching node: same rule as gather_nb
      const int str = (J == 0) ? 1 : (J == 1 ? P1 : P1 * P1);
      const bool plus = (ij == K);
      int cn = plus ? ec.c[J] + 1 : ec.c[J] - 1;
      if (cn < 0) cn += md.n[J];
      if (cn >= md.n[J]) cn -= md.n[J];
      const int en = e + (cn - ec.c[J]) * elem_stride(md, J);
      const int nn = plus ? n - K * str : n + K * str;
      const unsigned gn = (unsigned)(md.eoff + en) * NP + nn;
#pragma unroll
      for (int v = 0; v < NV; ++v) Ln[v] = (lam + (size_t)v * N)[gn];
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) Ln[v] = R(0);
    }
    if (J == 0) face_vjp<R, K, D, RAIN, 0>(a, md, ij, iz, Uq, q, T, rvs, nb, Lq, Ln, wall, zoff, sd, Ub);
    else if (J == 1) face_vjp<R, K, D, RAIN, 1>(a, md, ij, iz, Uq, q, T, rvs, nb, Lq, Ln, wall, zoff, sd, Ub);
    else face_vjp<R, K, D, RAIN, (D == 3 ? 2 : 0)>(a, md, ij, iz, Uq, q, T, rvs, nb, Lq, Ln, wall, zoff, sd, Ub);
  }
  // sources: dU/dt = ... + G
#pragma unroll
  for (int v = 0; v < NV; ++v) sd.G[v] = (double)Lq[v];
  pointwise_vjp<R, D, RAIN>(a, Uq, T, rvs, iz, sd, Ub);
  // out = cx1 X1 + cx2 X2 + c1 lam + c2 dt (d rhs/dU)^T lam
  const double k2 = c2 * (dt_m ? dt_m[item.member] : 1.0);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double o = c1 * (double)Lq[v] + k2 * Ub[v];
    if (X1) o += cx1 * (double)(X1 + (size_t)v * N)[g];
    if (X2) o += cx2 * (double)(X2 + (size_t)v * N)[g];
    (out + (size_t)v * N)[g] = (R)o;
  }
  }
}

// adjoint of the split alone: (T_bar, rho_v_bar, rho_c_bar) -> U_bar
template <typename R, int K, int D, int RAIN>
__global__ void __launch_bounds__(256)
split_vjp_kernel(KArgs a, const R* __restrict__ U, const double* __restrict__ auxT,
                 const double* __restrict__ auxS, const double* __restrict__ Tbar,
                 const double* __restrict__ rvbar, const double* __restrict__ rcbar,
                 R* __restrict__ out) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NP = S::NP, NV = V::NV;
  const ItemWalk walk(a.nitems);
  for (int kk = 0;; ++kk) {
  const int it_ = walk.item(kk);
  if (it_ < 0) break;
  const int t = threadIdx.x;
  const Item item = a.items[it_];
  const MemberDesc& md = a.mem[item.member];
  const int le = t / NP, n = t - le * NP;
  const int e = item.e0 + le;
  if (e >= md.ne) continue;
  const unsigned N = a.nnodes;
  const unsigned g = (unsigned)(md.eoff + e) * NP + n;
  const ElemCoord<D> ec = item_coord<D>(md, item, le);
  const int l = (D == 2) ? n / P1 : n / (P1 * P1);
  const int iz = md.hoff + ec.c[D - 1] * P1 + l;
  double Uq[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Uq[v] = (double)(U + (size_t)v * N)[g];
  const double rd = a.bg_rd[iz] + Uq[V::RD];
  const double rm = a.bg_rm[iz] + Uq[V::RM];
  const double rr = RAIN ? a.bg_rr[iz] + Uq[V::RR] : 0.0;
  const double rho = rd + rm + rr;
  double uu = 0.0, u[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    u[i] = Uq[V::M0 + i] / rho;
    uu += u[i] * u[i];
  }
  const double T = auxT[g], rvs = auxS[g];
  const bool sat = rvs < rm;
  const double Tb = Tbar ? Tbar[g] : 0.0;
  const double rcb = rcbar ? rcbar[g] : 0.0;
  const double rvb = (rvbar ? rvbar[g] : 0.0) - rcb;   // rho_c = rm - rho_v
  double rdb = 0, rmb = rcb, rrb = 0, reb = 0;
  split_reverse(a, sat, rd, rm, rr, T, rvs, Tb, rvb, rdb, rmb, rrb, reb);
  double Ub[NV];
  double rhob = reb * 0.5 * uu;
  Ub[V::RD] = rdb + rhob;
  Ub[V::RM] = rmb + rhob;
  if (RAIN) Ub[V::RR] = rrb + rhob;
#pragma unroll
  for (int i = 0; i < D; ++i) Ub[V::M0 + i] = -reb * u[i];
  Ub[V::E] = reb;
#pragma unroll
  for (int v = 0; v < NV; ++v) (out + (size_t)v * N)[g] = (R)Ub[v];
  }
}

}  // namespace dgm
