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

// Coordinates of element e0 + le of a work item (items may run past the end of
// an x-row; the carry moves to the next row).
template <int D>
__device__ __forceinline__ ElemCoord<D> item_coord(const MemberDesc& md, const Item& it, int le) {
  ElemCoord<D> ec;
  ec.c[0] = it.c0 + le;
  ec.c[1] = it.c12 & 0xffff;
  ec.c[2] = it.c12 >> 16;
  while (ec.c[0] >= md.n[0]) {
    ec.c[0] -= md.n[0];
    if (++ec.c[1] >= md.n[1] && D == 3) {
      ec.c[1] = 0;
      ++ec.c[2];
    }
  }
  return ec;
}

__device__ __forceinline__ int elem_stride(const MemberDesc& md, int j) {
  return j == 0 ? 1 : (j == 1 ? md.n[0] : md.n[0] * md.n[1]);
}

// Work items (member, first element) of EPB elements are dealt to blocks.
// Consecutive blocks go round-robin to the 8 XCDs; XCD x owns the contiguous
// item range [x per, (x+1) per), so neighbouring elements share an L2.  With a
// persistent grid (fewer blocks than items) each block walks its XCD's range
// with stride gridDim/8.  gridDim.x is always a multiple of 8.
struct ItemWalk {
  int per, g8, x, l, nitems;
  __device__ __forceinline__ explicit ItemWalk(int n) {
    nitems = n;
    per = (n + 7) >> 3;
    g8 = gridDim.x >> 3;
    x = blockIdx.x & 7;
    l = blockIdx.x >> 3;
  }
  // item of the k-th iteration, or -1 when the walk is over (uniform per block)
  __device__ __forceinline__ int item(int k) const {
    const int li = l + k * g8;
    if (li >= per) return -1;
    const int it = x * per + li;
    return it < nitems ? it : -1;
  }
};

__host__ __device__ inline int grid_for_items(int nitems) { return ((nitems + 7) >> 3) << 3; }

// ---------------------------------------------------------------------------
// split kernel: (T, rho_vs) per node, or the API outputs (T, rho_v, rho_c)
// ---------------------------------------------------------------------------
template <typename R, int K, int D, int RAIN, int API>
__global__ void __launch_bounds__(256)
split_kernel(KArgs a, int item0, int nitems, const R* __restrict__ U, const double* __restrict__ Tguess,
             double* __restrict__ oT, double* __restrict__ o1, double* __restrict__ o2) {
  using S = Shape<K, D>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NP = S::NP, NV = V::NV;
  const ItemWalk walk(nitems);
  for (int k = 0;; ++k) {
  const int it_ = walk.item(k);
  if (it_ < 0) break;
  const int t = threadIdx.x;
  const Item item = a.items[item0 + it_];
  const MemberDesc& md = a.mem[item.member];
  const int le = t / NP, n = t - le * NP;
  const int e = item.e0 + le;
  const bool active = e < md.ne;
  int iters = 0, bad = 0;
  if (active) {
    const unsigned N = a.nnodes;
    const unsigned g = (unsigned)(md.eoff + e) * NP + n;
    const ElemCoord<D> ec = item_coord<D>(md, item, le);
    const int l = (D == 2) ? n / P1 : n / (P1 * P1);
    const int iz = md.hoff + ec.c[D - 1] * P1 + l;
    R Uq[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Uq[v] = (U + (size_t)v * N)[g];
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
      // the stored rho_vs(T) must be a fresh evaluation: it anchors later splits
      o1[g] = (s.iters > 0 && s.bad == 0) ? rho_vs(a, s.T) : s.rvs;
    }
  }
  record_stats(a, iters, bad);
  }
}

// ---------------------------------------------------------------------------
// right-hand side / stage kernel
// ---------------------------------------------------------------------------
// MODE 0: out = dU/dt
// MODE 1: out = c0 U0 + c1 U + c2 dt_member dU/dt  (a Shu-Osher stage)
// MODE 2: as MODE 1, then the split of the new state at every node, written
//         to (oT, oS); Newton is warm-started and anchored at the input
//         state's (T, rho_vs).  With `refresh` the stored rho_vs is a fresh
//         evaluation at the new T (once per step), otherwise the anchored one.
template <typename R, int D, int RAIN>
struct Nb {
  R U[Vars<D, RAIN>::NV];
  double T, rvs;
};

template <typename R, int K, int D, int RAIN, int J>
__device__ __forceinline__ void gather_nb(const MemberDesc& md, const ElemCoord<D>& ec, int e, int n,
                                          int ij, const R* __restrict__ U,
                                          const double* __restrict__ auxT,
                                          const double* __restrict__ auxS, unsigned N,
                                          Nb<R, D, RAIN>& nb, bool& wall, int& izn_off) {
  using S = Shape<K, D>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NV = V::NV;
  constexpr int STR = (J == 0) ? 1 : (J == 1 ? P1 : P1 * P1);
  const bool plus = (ij == K);
  const int c = ec.c[J];
  const bool at_end = plus ? (c == md.n[J] - 1) : (c == 0);
  wall = at_end && md.bc[J] == 1;
  if (wall) return;
  int cn = plus ? c + 1 : c - 1;
  if (cn < 0) cn += md.n[J];
  if (cn >= md.n[J]) cn -= md.n[J];
  const int en = e + (cn - c) * elem_stride(md, J);
  const int nn = plus ? n - K * STR : n + K * STR;
  const unsigned gn = (unsigned)(md.eoff + en) * S::NP + nn;
#pragma unroll
  for (int v = 0; v < NV; ++v) nb.U[v] = (U + (size_t)v * N)[gn];
  nb.T = auxT[gn];
  nb.rvs = auxS[gn];
  izn_off = (J == D - 1) ? (cn * P1 + (plus ? 0 : K)) : -1;
}

// Volume term (Section 3.2 weak form, Lobatto collocation): for direction J,
// R += (2/h_J) sum_b Dhat[i_J][b] F_J(node b on this node's J-line).  The
// fluxes of all directions are staged in LDS behind one barrier.
template <typename R, int K, int D, int RAIN, int J>
__device__ __forceinline__ void volume_dir(const MemberDesc& md, int ij, const R* sFJ, R* Rv,
                                           const R* sD) {
  using S = Shape<K, D>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NV = V::NV;
  constexpr int STR = (J == 0) ? 1 : (J == 1 ? P1 : P1 * P1);
  const int t = threadIdx.x;
  const int NT = blockDim.x;
  const R s = (R)md.two_over_h[J];
  const int base = t - ij * STR;
  R d[P1];
#pragma unroll
  for (int b = 0; b < P1; ++b) d[b] = sD[ij * P1 + b];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    R acc = R(0);
#pragma unroll
    for (int b = 0; b < P1; ++b) acc += d[b] * sFJ[v * NT + base + b * STR];
    Rv[v] += s * acc;
  }
}

template <typename R, int K, int D, int RAIN, int J>
__device__ __forceinline__ void stage_flux(const Pt<R, D, RAIN>& q, R* sFJ) {
  using V = Vars<D, RAIN>;
  constexpr int NV = V::NV;
  const int NT = blockDim.x;
  R F[NV];
  flux<R, D, RAIN, J>(q, F);
#pragma unroll
  for (int v = 0; v < NV; ++v) sFJ[v * NT + threadIdx.x] = F[v];
}

template <typename R, int K, int D, int RAIN, int J>
__device__ __forceinline__ void face_dir(const KArgs& a, const MemberDesc& md, int ij, int iz,
                                         const R* Uq, const Pt<R, D, RAIN>& q, const Nb<R, D, RAIN>& nb,
                                         bool wall, int izn_off, R* Rv) {
  using V = Vars<D, RAIN>;
  constexpr int NV = V::NV;
  const bool plus = (ij == K);
  R Un[NV];
  Pt<R, D, RAIN> qn;
  if (wall) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[v] = Uq[v];
    Un[V::M0 + J] = -Uq[V::M0 + J];
    qn = q;
    reflect<R, D, RAIN, J>(qn);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[v] = nb.U[v];
    const int izn = (J == D - 1) ? md.hoff + izn_off : iz;
    eval_point<R, D, RAIN>(a, Un, nb.T, nb.rvs, izn, qn);
  }
  R F[NV], Fn[NV];
  flux<R, D, RAIN, J>(q, F);
  flux<R, D, RAIN, J>(qn, Fn);
  const R lo = wave_speed<R, D, RAIN, J>(q);
  const R ln = wave_speed<R, D, RAIN, J>(qn);
  // Lambda = max over the two sides, ties to the minus side
  const R Lam = plus ? ((lo >= ln) ? lo : ln) : ((ln >= lo) ? ln : lo);
  const R half = R(0.5);
  if (plus) {
    const R lift = (R)(md.two_over_h[J] / a.w[K]);
#pragma unroll
    for (int v = 0; v < NV; ++v) Rv[v] -= lift * (half * (F[v] + Fn[v]) + half * Lam * (Uq[v] - Un[v]));
  } else {
    const R lift = (R)(md.two_over_h[J] / a.w[0]);
#pragma unroll
    for (int v = 0; v < NV; ++v) Rv[v] += lift * (half * (Fn[v] + F[v]) + half * Lam * (Un[v] - Uq[v]));
  }
}

template <typename R, int K, int D, int RAIN, int MODE>
__device__ __forceinline__ void rhs_item(const KArgs& a, int it_, R (*sF)[Vars<D, RAIN>::NV * Shape<K, D>::NT],
                                         const R* sD, const R* __restrict__ U,
                                         const double* __restrict__ auxT,
                                         const double* __restrict__ auxS, R* __restrict__ out,
                                         const R* __restrict__ U0, const double* __restrict__ dt_m,
                                         double c0, double c1, double c2, double* __restrict__ oT,
                                         double* __restrict__ oS, int refresh) {
  using S = Shape<K, D>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NP = S::NP, NV = V::NV;
  const int t = threadIdx.x;
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
  R Uq[NV];
  double T = 300.0, rvs = 0.0;
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Uq[v] = (U + (size_t)v * N)[g];
    T = auxT[g];
    rvs = auxS[g];
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) Uq[v] = R(0);
  }
  // neighbour traces: issue every gather before any arithmetic
  Nb<R, D, RAIN> nb0, nb1, nb2;
  bool w0 = false, w1 = false, w2 = false;
  int z0 = -1, z1 = -1, z2 = -1;
  const bool f0 = active && (idx[0] == 0 || idx[0] == K);
  const bool f1 = active && (idx[1] == 0 || idx[1] == K);
  const bool f2 = (D == 3) && active && (idx[2] == 0 || idx[2] == K);
  if (f0) gather_nb<R, K, D, RAIN, 0>(md, ec, e, n, idx[0], U, auxT, auxS, N, nb0, w0, z0);
  if (f1) gather_nb<R, K, D, RAIN, 1>(md, ec, e, n, idx[1], U, auxT, auxS, N, nb1, w1, z1);
  if constexpr (D == 3) {
    if (f2) gather_nb<R, K, D, RAIN, 2>(md, ec, e, n, idx[2], U, auxT, auxS, N, nb2, w2, z2);
  }
  Pt<R, D, RAIN> q;
  eval_point<R, D, RAIN>(a, Uq, T, rvs, active ? iz : md.hoff, q);
  R Rv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Rv[v] = R(0);
  stage_flux<R, K, D, RAIN, 0>(q, sF[0]);
  stage_flux<R, K, D, RAIN, 1>(q, sF[1]);
  if constexpr (D == 3) stage_flux<R, K, D, RAIN, 2>(q, sF[2]);
  __syncthreads();
  if (active) {
    volume_dir<R, K, D, RAIN, 0>(md, idx[0], sF[0], Rv, sD);
    volume_dir<R, K, D, RAIN, 1>(md, idx[1], sF[1], Rv, sD);
    if constexpr (D == 3) volume_dir<R, K, D, RAIN, 2>(md, idx[2], sF[2], Rv, sD);
  }
  if (f0) face_dir<R, K, D, RAIN, 0>(a, md, idx[0], iz, Uq, q, nb0, w0, z0, Rv);
  if (f1) face_dir<R, K, D, RAIN, 1>(a, md, idx[1], iz, Uq, q, nb1, w1, z1, Rv);
  if constexpr (D == 3) {
    if (f2) face_dir<R, K, D, RAIN, 2>(a, md, idx[2], iz, Uq, q, nb2, w2, z2, Rv);
  }
  int iters = 0, bad = 0;
  if (active) {
    sources<R, D, RAIN>(a, Uq, q, Rv);
    if (MODE == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) (out + (size_t)v * N)[g] = Rv[v];
    } else {
      const R k2 = (R)(c2 * dt_m[item.member]);
      const R k1 = (R)c1;
      R Un[NV];
      if (c0 != 0.0) {
        const R k0 = (R)c0;
#pragma unroll
        for (int v = 0; v < NV; ++v) Un[v] = k0 * (U0 + (size_t)v * N)[g] + k1 * Uq[v] + k2 * Rv[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) Un[v] = k1 * Uq[v] + k2 * Rv[v];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) (out + (size_t)v * N)[g] = Un[v];
      if (MODE == 2) {
        // split of the new state (FP64), warm-started at this node's (T, rho_vs)
        const double rd = a.bg_rd[iz] + (double)Un[V::RD];
        const double rm = a.bg_rm[iz] + (double)Un[V::RM];
        const double rr = RAIN ? a.bg_rr[iz] + (double)Un[V::RR] : 0.0;
        double ke = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
          const double mi = (double)Un[V::M0 + i];
          ke += mi * mi;
        }
        const double re = a.bg_E[iz] + (double)Un[V::E] - 0.5 * ke * rcp64(rd + rm + rr);
        Anchor A;
        A.T0 = 0.0; A.r0 = 0.0; A.inv0 = 0.0;
        if (T > 150.0 && T < 600.0 && rvs > 0.0) {
          A.T0 = T; A.r0 = rvs; A.inv0 = rcp64(T);
        }
        // the branch that held at this node before is tried first
        const SplitOut s = split_point_anchor(a, rd, rm, rr, re, T, A, rvs < rm);
        iters = s.iters;
        bad = s.bad;
        oT[g] = s.T;
        oS[g] = (refresh && s.bad == 0) ? rho_vs(a, s.T) : s.rvs;
      }
    }
  }
  if (MODE == 2) record_stats(a, iters, bad);
}

// one work item per block
template <typename R, int K, int D, int RAIN, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
rhs_kernel(KArgs a, const R* __restrict__ U, const double* __restrict__ auxT,
           const double* __restrict__ auxS, R* __restrict__ out, const R* __restrict__ U0,
           const double* __restrict__ dt_m, double c0, double c1, double c2,
           double* __restrict__ oT, double* __restrict__ oS, int refresh) {
  using S = Shape<K, D>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1;
  __shared__ R sF[D][V::NV * S::NT];
  __shared__ R sD[P1 * P1];
  if (threadIdx.x < P1 * P1) sD[threadIdx.x] = (R)a.Dhat[threadIdx.x];
  const ItemWalk walk(a.nitems);
  const int it_ = walk.item(0);
  if (it_ < 0) return;
  rhs_item<R, K, D, RAIN, MODE>(a, it_, sF, sD, U, auxT, auxS, out, U0, dt_m, c0, c1, c2, oT, oS, refresh);
}

// persistent: a grid smaller than the item count walks the items
template <typename R, int K, int D, int RAIN, int MODE>
__global__ void __launch_bounds__(256)
rhs_kernel_persistent(KArgs a, const R* __restrict__ U, const double* __restrict__ auxT,
                      const double* __restrict__ auxS, R* __restrict__ out, const R* __restrict__ U0,
                      const double* __restrict__ dt_m, double c0, double c1, double c2,
                      double* __restrict__ oT, double* __restrict__ oS, int refresh) {
  using S = Shape<K, D>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1;
  __shared__ R sF[D][V::NV * S::NT];
  __shared__ R sD[P1 * P1];
  if (threadIdx.x < P1 * P1) sD[threadIdx.x] = (R)a.Dhat[threadIdx.x];
  const ItemWalk walk(a.nitems);
  for (int kk = 0;; ++kk) {
    const int it_ = walk.item(kk);
    if (it_ < 0) break;
    rhs_item<R, K, D, RAIN, MODE>(a, it_, sF, sD, U, auxT, auxS, out, U0, dt_m, c0, c1, c2, oT, oS, refresh);
    __syncthreads();   // sF is reused by the next item
  }
}



// ---------------------------------------------------------------------------
// conservation diagnostics: per-block FP64 partial sums in a fixed order
// ---------------------------------------------------------------------------
template <typename R, int K, int D, int RAIN>
__global__ void __launch_bounds__(256)
mass_kernel(KArgs a, int item0, const R* __restrict__ U, double* __restrict__ partial) {
  // (blocks map to items in order here: partials are summed in a fixed order)
  using S = Shape<K, D>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NP = S::NP;
  __shared__ double sm[3][S::NT];
  const int NT = blockDim.x;
  const int t = threadIdx.x;
  const Item item = a.items[item0 + blockIdx.x];
  const MemberDesc& md = a.mem[item.member];
  const int le = t / NP, n = t - le * NP;
  const int e = item.e0 + le;
  double md_ = 0.0, mw = 0.0, fl = 0.0;
  if (e < md.ne) {
    const size_t N = a.nnodes;
    const size_t g = (size_t)(md.eoff + e) * NP + n;
    int idx[3] = {n % P1, (n / P1) % P1, (D == 3) ? n / (P1 * P1) : 0};
    double w = md.J;
#pragma unroll
    for (int j = 0; j < D; ++j) w *= a.w[idx[j]];
    md_ = w * (double)U[V::RD * N + g];
    mw = w * ((double)U[V::RM * N + g] + (RAIN ? (double)U[V::RR * N + g] : 0.0));
    if (RAIN && md.bc[D - 1] == 1) {
      const ElemCoord<D> ec = item_coord<D>(md, item, le);
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
