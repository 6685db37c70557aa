// Right-hand side / stage kernel of the Gauss basis: nodes at the k+1
// Gauss-Legendre points per axis.  That nodal basis spans the same Q^k as the
// paper's Legendre modes, its quadrature at the nodes is the paper's Gauss
// rule, the mass matrix is diagonal and exact, and the L2 projection of the
// split results onto Q^k (Section 3.4) is their nodal value.  What changes
// against the Lobatto kernels is the face: no node lies on it, so every face
// quadrature point takes the traces of U', T and rho_v along its normal line
// (k+1 nodes per side), and the face flux is lifted back to every node of
// that line.
//
// A block owns a work item of EPB elements, one thread per node:
//   1. node pass: the point state, its fluxes (LDS) and the perturbation, T
//      and rho_v (LDS), then the volume term and the sources;
//   2. face pass: the block's EPB * 2D * (k+1)^(D-1) face points, each with
//      its own trace interpolated from LDS and the neighbour's read from the
//      trace buffer of the stage state, the Lax-Friedrichs flux with normal
//      +e_J into LDS;
//   3. lifting, the stage update and the split of the new state;
//   4. (MODE 2) the new state back into LDS and its face traces to the
//      output trace buffer, for the next stage.
// gauss_trace_kernel writes the traces of a state that no stage produced
// (the first stage of a call, dg_rhs).
#pragma once
#include "dg_kernels.h"

namespace dgm {

template <int K, int D>
struct GaussShape {
  static constexpr int P1 = K + 1;
  static constexpr int NF = (D == 2) ? P1 : P1 * P1;   // quadrature points of one face
  static constexpr int NFE = 2 * D * NF;                // face points of one element
};

// Node of an element on the J-line through face point fp at position a along J.
// The face point enumerates the other axes, the lower axis fastest.
template <int K, int D, int J>
__device__ __forceinline__ int line_node(int fp, int a) {
  constexpr int P1 = K + 1;
  if constexpr (D == 2) {
    return J == 0 ? a + P1 * fp : fp + P1 * a;
  } else {
    const int u = fp % P1, w = fp / P1;
    if constexpr (J == 0) return a + P1 * (u + P1 * w);
    else if constexpr (J == 1) return u + P1 * (a + P1 * w);
    else return u + P1 * (w + P1 * a);
  }
}

// vertical node index (within the element) of face point fp of a face normal
// to a horizontal axis J < D-1
template <int K, int D, int J>
__device__ __forceinline__ int face_level(int fp) {
  return D == 2 ? fp : fp / (K + 1);
}

// Trace of U', T and rho_v at face point fp on side `side` (0: xi_J = -1,
// 1: xi_J = +1) of element le of the block, from the block's LDS tiles.
// The face pass (own side) and the trace writer share this code, so both
// sides of a face see the same bits.
template <typename R, int K, int D, int RAIN, int J>
__device__ __forceinline__ void gauss_trace(int le, int side, int fp, const R* sU, const double* sT,
                                            const double* sRv, const double (*sL)[kMaxP1], R* Ut,
                                            double& Tt, double& Rvt) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NP = S::NP, NV = V::NV, NT = S::NT;
#pragma unroll
  for (int v = 0; v < NV; ++v) Ut[v] = R(0);
  Tt = 0.0;
  Rvt = 0.0;
#pragma unroll
  for (int i = 0; i < P1; ++i) {
    const int nd = le * NP + line_node<K, D, J>(fp, i);
    const double w = sL[side][i];
#pragma unroll
    for (int v = 0; v < NV; ++v) Ut[v] += (R)w * sU[v * NT + nd];
    Tt += w * sT[nd];
    Rvt += w * sRv[nd];
  }
}

// Every face-point trace of the block's elements, from the tiles, to the
// output trace buffers.
template <typename R, int K, int D, int RAIN>
__device__ __forceinline__ void write_traces(const KArgs& a, const MemberDesc& md, const Item& item, int epb,
                                             const R* sU, const double* sT, const double* sRv,
                                             const double (*sL)[kMaxP1]) {
  using V = Vars<D, RAIN>;
  using G = GaussShape<K, D>;
  constexpr int NV = V::NV, NF = G::NF, NFE = G::NFE;
  R* tu = (R*)a.tr_u_out;
  for (int task = threadIdx.x; task < epb * NFE; task += (int)blockDim.x) {
    const int fle = task / NFE;
    const int r = task - fle * NFE;
    if (item.e0 + fle >= md.ne) continue;
    const int f = r / NF;
    const int fp = r - f * NF;
    const int J = f >> 1, side = f & 1;
    R Ut[NV];
    double Tt, Rvt;
    if (J == 0) gauss_trace<R, K, D, RAIN, 0>(fle, side, fp, sU, sT, sRv, sL, Ut, Tt, Rvt);
    else if (J == 1 || D == 2) gauss_trace<R, K, D, RAIN, 1>(fle, side, fp, sU, sT, sRv, sL, Ut, Tt, Rvt);
    else if constexpr (D == 3) gauss_trace<R, K, D, RAIN, 2>(fle, side, fp, sU, sT, sRv, sL, Ut, Tt, Rvt);
    const size_t eg = (size_t)(md.eoff + item.e0 + fle);
    const size_t et = (size_t)a.etot;
#pragma unroll
    for (int v = 0; v < NV; ++v) tu[((size_t)v * et + eg) * NFE + r] = Ut[v];
    a.tr_a_out[eg * NFE + r] = Tt;
    a.tr_a_out[(et + eg) * NFE + r] = Rvt;
  }
}

// LF flux with normal +e_J at face point fp on side `side` of element le of
// the item: the own trace from the tiles, the neighbour's from the input
// trace buffer (its face point on the opposite side), or the slip-wall ghost.
template <typename R, int K, int D, int RAIN, int J>
__device__ __forceinline__ void gauss_face(const KArgs& a, const MemberDesc& md, const Item& item, int le,
                                           int side, int fp, const R* sU, const double* sT,
                                           const double* sRv, const double (*sL)[kMaxP1], R* Fs) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  using G = GaussShape<K, D>;
  constexpr int P1 = S::P1, NV = V::NV, NF = G::NF, NFE = G::NFE;
  R Uo[NV];
  double To, Rvo;
  gauss_trace<R, K, D, RAIN, J>(le, side, fp, sU, sT, sRv, sL, Uo, To, Rvo);
  const ElemCoord<D> ec = item_coord<D>(md, item, le);
  const int e = item.e0 + le;
  const int c = ec.c[J];
  const bool at_end = side ? (c == md.n[J] - 1) : (c == 0);
  const bool wall = at_end && md.bc[J] == 1;
  int cn = side ? c + 1 : c - 1;
  if (cn < 0) cn += md.n[J];
  if (cn >= md.n[J]) cn -= md.n[J];
  // background at the face point, own and neighbour side
  double bo[5], bn[5];
  if constexpr (J == D - 1) {
    const int r0 = md.hoff / P1;
#pragma unroll
    for (int f = 0; f < 5; ++f) {
      bo[f] = a.bgf[f * a.bgf_n + 2 * (r0 + c) + side];
      bn[f] = a.bgf[f * a.bgf_n + 2 * (r0 + cn) + 1 - side];
    }
  } else {
    const int izf = md.hoff + ec.c[D - 1] * P1 + face_level<K, D, J>(fp);
    bo[0] = a.bg_rd[izf]; bo[1] = a.bg_rm[izf]; bo[2] = RAIN ? a.bg_rr[izf] : 0.0;
    bo[3] = a.bg_E[izf]; bo[4] = a.bg_p[izf];
#pragma unroll
    for (int f = 0; f < 5; ++f) bn[f] = bo[f];
  }
  R Un[NV];
  double Tn, Rvn;
  if (wall) {
    // the ghost keeps the own background (cn wrapped to the far end of the column)
#pragma unroll
    for (int f = 0; f < 5; ++f) bn[f] = bo[f];
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[v] = Uo[v];
    Un[V::M0 + J] = -Uo[V::M0 + J];
    Tn = To;
    Rvn = Rvo;
  } else {
    const size_t en = (size_t)(md.eoff + e + (cn - c) * elem_stride(md, J));
    const size_t et = (size_t)a.etot;
    const int rn = (2 * J + 1 - side) * NF + fp;
    const R* tu = (const R*)a.tr_u_in;
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[v] = tu[((size_t)v * et + en) * NFE + rn];
    Tn = a.tr_a_in[en * NFE + rn];
    Rvn = a.tr_a_in[(et + en) * NFE + rn];
  }
  Pt<R, D, RAIN> qo, qn;
  eval_core<R, D, RAIN>(a, Uo, To, Rvo, Rvo, bo[0], bo[1], bo[2], bo[3], bo[4], qo);
  eval_core<R, D, RAIN>(a, Un, Tn, Rvn, Rvn, bn[0], bn[1], bn[2], bn[3], bn[4], qn);
  // minus side = lower coordinate along J
  const Pt<R, D, RAIN>& qm = side ? qo : qn;
  const Pt<R, D, RAIN>& qp = side ? qn : qo;
  const R* Um = side ? Uo : Un;
  const R* Up = side ? Un : Uo;
  R Fm[NV], Fp[NV];
  flux<R, D, RAIN, J>(qm, Fm);
  flux<R, D, RAIN, J>(qp, Fp);
  const R lm = wave_speed<R, D, RAIN, J>(qm), lp = wave_speed<R, D, RAIN, J>(qp);
  const R Lam = lm >= lp ? lm : lp;
  const R half = R(0.5);
#pragma unroll
  for (int v = 0; v < NV; ++v) Fs[v] = half * (Fm[v] + Fp[v]) + half * Lam * (Um[v] - Up[v]);
}

// Node pass shared by the stage and trace kernels: the node's perturbation,
// T and rho_v = min(rho_vs, rho_m) into the tiles.
template <typename R, int K, int D, int RAIN>
__device__ __forceinline__ void stage_node_tiles(const KArgs& a, bool active, int iz, unsigned g, const R* Uq,
                                                 double T, double rvs, R* sU, double* sT, double* sRv) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  constexpr int NV = V::NV, NT = S::NT;
  const int t = threadIdx.x;
#pragma unroll
  for (int v = 0; v < NV; ++v) sU[v * NT + t] = Uq[v];
  sT[t] = T;
  sRv[t] = active ? fmin(rvs, a.bg_rm[iz] + (double)Uq[V::RM]) : 0.0;
}

// Face traces of a state and its split (T, rho_vs): the first stage of a
// call, and dg_rhs, read them.
template <typename R, int K, int D, int RAIN>
__global__ void __launch_bounds__(256)
gauss_trace_kernel(KArgs a, const R* __restrict__ U, const double* __restrict__ auxT,
                   const double* __restrict__ auxS) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NP = S::NP, NV = V::NV, NT = S::NT;
  __shared__ R sU[NV * NT];
  __shared__ double sT[NT], sRv[NT];
  __shared__ double sL[2][kMaxP1];
  const int t = threadIdx.x;
  if (t < P1) {
    sL[0][t] = a.gl_m[t];
    sL[1][t] = a.gl_p[t];
  }
  const int epb = (int)blockDim.x / NP;
  const ItemWalk walk(a.nitems);
#pragma clang loop unroll(disable)
  for (int kk = 0;; ++kk) {
    const int it_ = walk.item(kk);
    if (it_ < 0) break;
    const Item item = a.items[it_];
    const MemberDesc& md = a.mem[item.member];
    const int le = t / NP, n = t - le * NP;
    const int e = item.e0 + le;
    const bool active = e < md.ne;
    const unsigned N = a.nnodes;
    const unsigned g = (unsigned)(md.eoff + (active ? e : 0)) * NP + n;
    const ElemCoord<D> ec = item_coord<D>(md, item, active ? le : 0);
    const int l = (D == 2) ? n / P1 : n / (P1 * P1);
    const int iz = md.hoff + ec.c[D - 1] * P1 + l;
    R Uq[NV];
    double T = 300.0, rvs = 0.0;
    if (active) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Uq[v] = ld(U, N, v, g);
      T = ld(auxT, N, 0, g);
      rvs = ld(auxS, N, 0, g);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) Uq[v] = R(0);
    }
    stage_node_tiles<R, K, D, RAIN>(a, active, iz, g, Uq, T, rvs, sU, sT, sRv);
    __syncthreads();
    write_traces<R, K, D, RAIN>(a, md, item, epb, sU, sT, sRv, sL);
    __syncthreads();   // the tiles are reused by the next item
  }
}

// FP32 up to Q3 in 3D and Q5 in 2D: 4 wavefronts per SIMD (128 VGPRs; with
// the face fluxes in the flux tile, four blocks fit a CU's LDS). FP64 up to
// Q3 in 3D and Q6 in 2D: 2 wavefronts per SIMD, i.e. no more than 256
// registers in all (left free, the compiler parks a few values in AGPRs
// beyond the 256 VGPRs, which halves the occupancy). Higher orders would
// spill under these bounds and are left to the compiler.
template <typename R, int K, int D>
constexpr int gauss_min_waves() {
  if (sizeof(R) == 4) return K <= (D == 3 ? 3 : 5) ? 4 : 1;
  return K <= (D == 3 ? 3 : 6) ? 2 : 1;
}

template <typename R, int K, int D, int RAIN, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(gauss_min_waves<R, K, D>())))
rhs_gauss_kernel(KArgs a, const R* __restrict__ U, const double* __restrict__ auxT,
                 const double* __restrict__ auxS, R* __restrict__ out, const R* __restrict__ U0,
                 const double* __restrict__ dt_m, double c0, double c1, double c2,
                 double* __restrict__ oT, double* __restrict__ oS, int flags) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  using G = GaussShape<K, D>;
  constexpr int P1 = S::P1, NP = S::NP, NV = V::NV, NT = S::NT;
  constexpr int NF = G::NF, NFE = G::NFE, NFB = S::EPB * NFE;
  __shared__ R sF[D * NV * NT];
  __shared__ R sU[NV * NT];
  __shared__ double sT[NT], sRv[NT];
  R* const sFs = sF;   // the face fluxes reuse the flux tile once the volume term has read it
  __shared__ R sD[P1 * P1];
  __shared__ double sL[2][kMaxP1];
  const int t = threadIdx.x;
  if (t < P1 * P1) sD[t] = (R)a.Dhat[t];
  if (t < P1) {
    sL[0][t] = a.gl_m[t];
    sL[1][t] = a.gl_p[t];
  }
  const int epb = (int)blockDim.x / NP;
  // one work item per block: a loop over items lets the compiler keep
  // loop-invariant values live across the whole body, which about doubles the
  // registers (and halves the occupancy)
  const int it_ = ItemWalk(a.nitems, a.walk_rev).item(0);
  if (it_ < 0) return;
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
  // 1. node pass
  R Uq[NV];
  double T = 300.0, rvs = 0.0;
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Uq[v] = ld(U, N, v, g);
    T = ld(auxT, N, 0, g);
    rvs = ld(auxS, N, 0, g);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) Uq[v] = R(0);
  }
  Pt<R, D, RAIN> q;
  eval_point<R, D, RAIN>(a, Uq, T, rvs, active ? iz : md.hoff, q);
  stage_flux<R, K, D, RAIN, 0>(q, sF);
  stage_flux<R, K, D, RAIN, 1>(q, sF + NV * NT);
  if constexpr (D == 3) stage_flux<R, K, D, RAIN, 2>(q, sF + 2 * NV * NT);
  stage_node_tiles<R, K, D, RAIN>(a, active, iz, g, Uq, T, rvs, sU, sT, sRv);
  __syncthreads();
  R Rv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Rv[v] = R(0);
  if (active) {
    volume_dir<R, K, D, RAIN, 0>(md, idx[0], sF, Rv, sD, t);
    volume_dir<R, K, D, RAIN, 1>(md, idx[1], sF + NV * NT, Rv, sD, t);
    if constexpr (D == 3) volume_dir<R, K, D, RAIN, 2>(md, idx[2], sF + 2 * NV * NT, Rv, sD, t);
    sources<R, D, RAIN>(a, Uq, q, Rv);
  }
  __syncthreads();   // the volume term's reads of sF are over
  // 2. face pass
  for (int task = t; task < epb * NFE; task += (int)blockDim.x) {
    const int fle = task / NFE;
    const int r = task - fle * NFE;
    const int f = r / NF;
    const int fp = r - f * NF;
    const int J = f >> 1, side = f & 1;
    R Fs[NV];
    if (item.e0 + fle < md.ne) {
      if (J == 0) gauss_face<R, K, D, RAIN, 0>(a, md, item, fle, side, fp, sU, sT, sRv, sL, Fs);
      else if (J == 1 || D == 2) gauss_face<R, K, D, RAIN, 1>(a, md, item, fle, side, fp, sU, sT, sRv, sL, Fs);
      else if constexpr (D == 3) gauss_face<R, K, D, RAIN, 2>(a, md, item, fle, side, fp, sU, sT, sRv, sL, Fs);
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) Fs[v] = R(0);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) sFs[v * NFB + task] = Fs[v];
  }
  __syncthreads();
  // 3. lifting: + l_i(-1)/w_i F*(minus face) - l_i(+1)/w_i F*(plus face),
  // then the stage update and the split
  int iters = 0, bad = 0;
  if (active) {
#pragma unroll
    for (int J = 0; J < D; ++J) {
      const int i = idx[J];
      int fpJ;
      if (D == 2) fpJ = (J == 0) ? idx[1] : idx[0];
      else fpJ = (J == 0) ? idx[1] + P1 * idx[2] : (J == 1 ? idx[0] + P1 * idx[2] : idx[0] + P1 * idx[1]);
      const int base = le * NFE + 2 * J * NF + fpJ;
      const R km = (R)(md.two_over_h[J] * a.lift_m[i]);
      const R kp = (R)(md.two_over_h[J] * a.lift_p[i]);
#pragma unroll
      for (int v = 0; v < NV; ++v) Rv[v] += km * sFs[v * NFB + base] - kp * sFs[v * NFB + base + NF];
    }
    R U0q[NV];
    const double dtm = (MODE != 0) ? dt_m[item.member] : 0.0;
    if (MODE != 0 && c0 != 0.0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) U0q[v] = ld(U0, N, v, g);
    }
    double bg[4] = {a.bg_rd[iz], a.bg_rm[iz], RAIN ? a.bg_rr[iz] : 0.0, a.bg_E[iz]};
    if (MODE == 2) {
      // the new state and its split go back to the tiles: every face-pass
      // read of them ended at the barrier above
      R Unew[NV];
      double Tnew = 300.0, Snew = 0.0;
      stage_epilogue<R, D, RAIN, MODE>(a, bg, iz, g, N, Uq, U0q, Rv, T, rvs, out, dtm, c0, c1, c2, oT, oS,
                                       flags, iters, bad, Unew, &Tnew, &Snew);
      stage_node_tiles<R, K, D, RAIN>(a, true, iz, g, Unew, Tnew, Snew, sU, sT, sRv);
    } else {
      stage_epilogue<R, D, RAIN, MODE>(a, bg, iz, g, N, Uq, U0q, Rv, T, rvs, out, dtm, c0, c1, c2, oT, oS,
                                       flags, iters, bad);
    }
  }
  if (MODE == 2) {
    record_stats(a, iters, bad);
    __syncthreads();
    // 4. the traces of the new state for the next stage
    write_traces<R, K, D, RAIN>(a, md, item, epb, sU, sT, sRv, sL);
  }
}

}  // namespace dgm
