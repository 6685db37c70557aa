// Kernels of libdgmoist and their launch dispatch (instantiated per precision
// in dg_f64.hip and dg_f32.hip).
//
// Work decomposition: a block owns EPB consecutive elements of one member
// (a work item); one thread owns one node of one element and computes every
// variable there.  Elements are consecutive in x, so a block's loads are
// contiguous per variable.
#pragma once
#include "dg_device.h"

namespace dgm {

template <int D>
struct ElemCoord {
  int c[3];
};

template <int D>
__device__ __forceinline__ ElemCoord<D> elem_coord(const MemberDesc& md, int e) {
  ElemCoord<D> ec;
  ec.c[0] = e % md.n[0];
  if (D == 2) {
    ec.c[1] = e / md.n[0];
    ec.c[2] = 0;
  } else {
    ec.c[1] = (e / md.n[0]) % md.n[1];
    ec.c[2] = e / (md.n[0] * md.n[1]);
  }
  return ec;
}

__device__ __forceinline__ int elem_stride(const MemberDesc& md, int j) {
  return j == 0 ? 1 : (j == 1 ? md.n[0] : md.n[0] * md.n[1]);
}

// ---------------------------------------------------------------------------
// split kernel: (T, rho_vs) per node, or the API outputs (T, rho_v, rho_c)
// ---------------------------------------------------------------------------
template <typename R, int K, int D, int RAIN, int API>
__global__ void __launch_bounds__(256)
split_kernel(KArgs a, int item0, const R* __restrict__ U, const double* __restrict__ Tguess,
             double* __restrict__ oT, double* __restrict__ o1, double* __restrict__ o2) {
  using S = Shape<K, D>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NP = S::NP, NV = V::NV;
  const int t = threadIdx.x;
  const int2 item = a.items[item0 + blockIdx.x];
  const MemberDesc& md = a.mem[item.x];
  const int le = t / NP, n = t - le * NP;
  const int e = item.y + le;
  const bool active = e < md.ne;
  int iters = 0, bad = 0;
  if (active) {
    const long long N = a.etot * NP;
    const long long g = (md.eoff + e) * NP + n;
    const ElemCoord<D> ec = elem_coord<D>(md, e);
    const int l = (D == 2) ? n / P1 : n / (P1 * P1);
    const int iz = md.hoff + ec.c[D - 1] * P1 + l;
    R Uq[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Uq[v] = U[v * N + g];
    const double rd = a.bg_rd[iz] + (double)Uq[V::RD];
    const double rm = a.bg_rm[iz] + (double)Uq[V::RM];
    const double rr = RAIN ? a.bg_rr[iz] + (double)Uq[V::RR] : 0.0;
    const double rho = rd + rm + rr;
    double ke = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double mi = (double)Uq[V::M0 + i];
      ke += mi * mi;
    }
    const double re = a.bg_E[iz] + (double)Uq[V::E] - 0.5 * ke / rho;
    const double guess = Tguess ? Tguess[g] : 0.0;
    const SplitOut s = split_point(a, rd, rm, rr, re, guess);
    iters = s.iters;
    bad = s.bad;
    oT[g] = s.T;
    if (API) {
      const double rv = fmin(s.rvs, rm);
      if (o1) o1[g] = rv;
      if (o2) o2[g] = rm - rv;
    } else {
      o1[g] = s.rvs;
    }
  }
  record_stats<S::NT>(a, iters, bad, active);
}

// ---------------------------------------------------------------------------
// right-hand side / stage kernel
// ---------------------------------------------------------------------------
// out = dU/dt                                  (MODE 0)
// out = c0 U0 + c1 U + c2 dt_member dU/dt       (MODE 1, a Shu-Osher stage)
template <typename R, int K, int D, int RAIN, int J>
__device__ __forceinline__ void direction(const KArgs& a, const MemberDesc& md, const ElemCoord<D>& ec,
                                          int e, int n, const int* idx, bool active, const R* Uq,
                                          const Pt<R, D, RAIN>& q, R* Rv, R (*sF)[Shape<K, D>::NT],
                                          const R* sD, const R* __restrict__ U,
                                          const double* __restrict__ auxT,
                                          const double* __restrict__ auxS, long long N, int iz) {
  using S = Shape<K, D>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NV = V::NV;
  constexpr int STR = (J == 0) ? 1 : (J == 1 ? P1 : P1 * P1);
  const int t = threadIdx.x;
  R F[NV];
  flux<R, D, RAIN, J>(q, F);
#pragma unroll
  for (int v = 0; v < NV; ++v) sF[v][t] = F[v];
  __syncthreads();
  const int ij = idx[J];
  if (active) {
    const R s = (R)md.two_over_h[J];
    const int base = t - ij * STR;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      R acc = R(0);
#pragma unroll
      for (int b = 0; b < P1; ++b) acc += sD[ij * P1 + b] * sF[v][base + b * STR];
      Rv[v] += s * acc;
    }
  }
  __syncthreads();
  if (!active || (ij != 0 && ij != K)) return;
  // face with normal +e_J through this node: own side is K- when ij == K
  const bool plus = (ij == K);
  const int c = ec.c[J];
  const bool at_end = plus ? (c == md.n[J] - 1) : (c == 0);
  const bool wall = at_end && md.bc[J] == 1;
  R Un[NV];
  Pt<R, D, RAIN> qn;
  if (wall) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[v] = Uq[v];
    Un[V::M0 + J] = -Uq[V::M0 + J];
    qn = q;
    reflect<R, D, RAIN, J>(qn);
  } else {
    int cn = plus ? c + 1 : c - 1;
    if (cn < 0) cn += md.n[J];
    if (cn >= md.n[J]) cn -= md.n[J];
    const int en = e + (cn - c) * elem_stride(md, J);
    const int nn = plus ? n - K * STR : n + K * STR;
    const long long gn = (md.eoff + en) * (long long)S::NP + nn;
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[v] = U[v * N + gn];
    int izn = iz;
    if (J == D - 1) izn = md.hoff + cn * P1 + (plus ? 0 : K);
    eval_point<R, D, RAIN>(a, Un, auxT[gn], auxS[gn], izn, qn);
  }
  R Fn[NV];
  flux<R, D, RAIN, J>(qn, Fn);
  const R lo = wave_speed<R, D, RAIN, J>(q);
  const R ln = wave_speed<R, D, RAIN, J>(qn);
  // Lambda = max over the two sides, ties to the minus side
  R Lam;
  if (plus) Lam = (lo >= ln) ? lo : ln;
  else Lam = (ln >= lo) ? ln : lo;
  const R half = R(0.5);
  if (plus) {
    const R lift = (R)(md.two_over_h[J] / a.w[K]);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const R Fs = half * (F[v] + Fn[v]) + half * Lam * (Uq[v] - Un[v]);
      Rv[v] -= lift * Fs;
    }
  } else {
    const R lift = (R)(md.two_over_h[J] / a.w[0]);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const R Fs = half * (Fn[v] + F[v]) + half * Lam * (Un[v] - Uq[v]);
      Rv[v] += lift * Fs;
    }
  }
}

template <typename R, int K, int D, int RAIN, int MODE>
__global__ void __launch_bounds__(256)
rhs_kernel(KArgs a, const R* __restrict__ U, const double* __restrict__ auxT,
           const double* __restrict__ auxS, R* __restrict__ out, const R* __restrict__ U0,
           const double* __restrict__ dt_m, double c0, double c1, double c2) {
  using S = Shape<K, D>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NP = S::NP, NV = V::NV;
  __shared__ R sF[NV][S::NT];
  __shared__ R sD[P1 * P1];
  const int t = threadIdx.x;
  if (t < P1 * P1) sD[t] = (R)a.Dhat[t];
  const int2 item = a.items[blockIdx.x];
  const MemberDesc& md = a.mem[item.x];
  const int le = t / NP, n = t - le * NP;
  const int e = item.y + le;
  const bool active = e < md.ne;
  const long long N = a.etot * NP;
  const long long g = (md.eoff + (active ? e : 0)) * NP + n;
  const ElemCoord<D> ec = elem_coord<D>(md, active ? e : 0);
  int idx[3];
  idx[0] = n % P1;
  idx[1] = (n / P1) % P1;
  idx[2] = (D == 3) ? n / (P1 * P1) : 0;
  const int iz = md.hoff + ec.c[D - 1] * P1 + idx[D - 1];
  R Uq[NV];
  Pt<R, D, RAIN> q;
  double T = 0.0, rvs = 0.0;
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Uq[v] = U[v * N + g];
    T = auxT[g];
    rvs = auxS[g];
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) Uq[v] = R(0);
    Uq[V::RD] = R(0);
    T = 300.0;
    rvs = 0.0;
  }
  eval_point<R, D, RAIN>(a, Uq, T, rvs, active ? iz : md.hoff, q);
  R Rv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Rv[v] = R(0);
  __syncthreads();
  direction<R, K, D, RAIN, 0>(a, md, ec, e, n, idx, active, Uq, q, Rv, sF, sD, U, auxT, auxS, N, iz);
  direction<R, K, D, RAIN, 1>(a, md, ec, e, n, idx, active, Uq, q, Rv, sF, sD, U, auxT, auxS, N, iz);
  if constexpr (D == 3)
    direction<R, K, D, RAIN, 2>(a, md, ec, e, n, idx, active, Uq, q, Rv, sF, sD, U, auxT, auxS, N, iz);
  if (!active) return;
  sources<R, D, RAIN>(a, Uq, q, Rv);
  if (MODE == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v * N + g] = Rv[v];
  } else {
    const R k2 = (R)(c2 * dt_m[item.x]);
    const R k1 = (R)c1;
    if (c0 != 0.0) {
      const R k0 = (R)c0;
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v * N + g] = k0 * U0[v * N + g] + k1 * Uq[v] + k2 * Rv[v];
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v * N + g] = k1 * Uq[v] + k2 * Rv[v];
    }
  }
}

// ---------------------------------------------------------------------------
// conservation diagnostics: per-block FP64 partial sums in a fixed order
// ---------------------------------------------------------------------------
template <typename R, int K, int D, int RAIN>
__global__ void __launch_bounds__(256)
mass_kernel(KArgs a, int item0, const R* __restrict__ U, double* __restrict__ partial) {
  using S = Shape<K, D>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NP = S::NP, NT = S::NT;
  __shared__ double sm[3][NT];
  const int t = threadIdx.x;
  const int2 item = a.items[item0 + blockIdx.x];
  const MemberDesc& md = a.mem[item.x];
  const int le = t / NP, n = t - le * NP;
  const int e = item.y + le;
  double md_ = 0.0, mw = 0.0, fl = 0.0;
  if (e < md.ne) {
    const long long N = a.etot * NP;
    const long long g = (md.eoff + e) * NP + n;
    int idx[3] = {n % P1, (n / P1) % P1, (D == 3) ? n / (P1 * P1) : 0};
    double w = md.J;
#pragma unroll
    for (int j = 0; j < D; ++j) w *= a.w[idx[j]];
    md_ = w * (double)U[V::RD * N + g];
    mw = w * ((double)U[V::RM * N + g] + (RAIN ? (double)U[V::RR * N + g] : 0.0));
    if (RAIN && md.bc[D - 1] == 1) {
      const ElemCoord<D> ec = elem_coord<D>(md, e);
      const int l = idx[D - 1];
      const bool bottom = ec.c[D - 1] == 0 && l == 0;
      const bool top = ec.c[D - 1] == md.n[D - 1] - 1 && l == K;
      if (bottom || top) {
        const int iz = md.hoff + ec.c[D - 1] * P1 + l;
        const double rr = a.bg_rr[iz] + (double)U[V::RR * N + g];
        double vr = a.vr_const;
        if (a.vr_mode != 0) vr = rr > 0.0 ? a.vr_pref * pow(rr, 0.125) : 0.0;
        double wf = md.face_J[D - 1];
#pragma unroll
        for (int j = 0; j < D - 1; ++j) wf *= a.w[idx[j]];
        // wall flux of rain is -rho_r v_r along +e_z: out at the floor, in at the lid
        fl = bottom ? wf * rr * vr : -wf * rr * vr;
      }
    }
  }
  sm[0][t] = md_; sm[1][t] = mw; sm[2][t] = fl;
  __syncthreads();
  // fixed-order tree over the block (NT need not be a power of two)
  for (int s = 1; s < NT; s <<= 1) {
    if ((t % (2 * s)) == 0 && t + s < NT) {
      sm[0][t] += sm[0][t + s];
      sm[1][t] += sm[1][t + s];
      sm[2][t] += sm[2][t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    partial[3 * blockIdx.x + 0] = sm[0][0];
    partial[3 * blockIdx.x + 1] = sm[1][0];
    partial[3 * blockIdx.x + 2] = sm[2][0];
  }
}

}  // namespace dgm
