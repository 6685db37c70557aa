// Stage kernel for Q3 hexahedra (Lobatto basis): one wavefront per element.
//
// A Q3 hexahedron has (3+1)^3 = 64 nodes, so lane n of a wavefront owns node
// n = i + 4 j + 16 l of one element.  Everything that depends on the element
// alone (its coordinates, neighbours, wall flags, offsets) is wave-uniform and
// lives in scalar registers; per-lane indices are bit fields of the lane id.
// Each wavefront works in its own LDS tiles, so the kernel has no block-wide
// barrier: a wavefront only orders its own LDS writes before its reads.
//
// Per element and RK stage (Section 3.2 weak form, Section 3.3 mass and
// update, Section 3.4 split):
//   1. load U, (T, rho_vs) of every node, and the background at the
//      element's heights and the neighbours' face heights into a small LDS
//      table; issue the loads of the neighbour traces of the first face pass
//      at once (their addresses depend on the element only), and those of the
//      second pass before the first pass's arithmetic;
//   2. evaluate the point state (FP64 reconstruction of p' and rho e), stage
//      F_x, F_y, F_z, U and the wave speeds in LDS;
//   3. volume term from the LDS lines, slip walls and sources by each node;
//   4. face passes: the element's 96 face nodes (16 per face) are tasks; pass
//      0 takes the x and y faces (64 lanes), pass 1 the z faces (32 lanes).
//      A task evaluates the neighbour's trace, forms the Lax-Friedrichs flux
//      with the own trace from LDS, and leaves the lifted correction in LDS;
//   5. every node adds the corrections of its faces, then the stage update,
//      the sponge, the store and the split of the new state (stage_epilogue).
#pragma once
#include "dg_kernels.h"

namespace dgm {

// Order LDS traffic of one wavefront: its earlier LDS writes are visible to
// its later reads (LDS operations of a wavefront complete in order; the fences
// keep the compiler from moving memory operations across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Physical flux in a horizontal direction chosen per lane (jx: x, else y);
// the vertical direction keeps its compile-time form (flux<.., D-1>).
template <typename R, int RAIN>
__device__ __forceinline__ void flux_h(const Pt<R, 3, RAIN>& q, bool jx, R* F) {
  using V = Vars<3, RAIN>;
  const R uj = jx ? q.u[0] : q.u[1];
  F[V::RD] = q.rd * uj;
  F[V::RM] = q.rm * uj;
  if (RAIN) F[V::RR] = q.rr * uj;
  F[V::M0 + 0] = q.m[0] * uj + (jx ? q.pp : R(0));
  F[V::M0 + 1] = q.m[1] * uj + (jx ? R(0) : q.pp);
  F[V::M0 + 2] = q.m[2] * uj;
  F[V::E] = q.H * uj;
}

// Volume term from this wavefront's flux tiles (rows of 64 nodes), variable
// by variable: R_v += sum_J (2/h_J) sum_b Dhat[i_J][b] F_J,v(node b on the
// lane's J-line).  The scheduling barrier after each variable keeps the
// compiler from issuing all 84 LDS reads at once (their results would need
// more registers than the kernel has).
template <typename R, int RAIN>
__device__ __forceinline__ void volume_q3(const MemberDesc& md, int li, int lj, int ll, int lane,
                                          const R (*sF)[Vars<3, RAIN>::NV][64], R* Rv, const R* sD) {
  constexpr int NV = Vars<3, RAIN>::NV;
  const R sx = (R)md.two_over_h[0], sy = (R)md.two_over_h[1], sz = (R)md.two_over_h[2];
  const int bx = lane - li, by = lane - 4 * lj, bz = lane - 16 * ll;
  R dx[4], dy[4], dz[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    dx[b] = sD[li * 4 + b];
    dy[b] = sD[lj * 4 + b];
    dz[b] = sD[ll * 4 + b];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    R ax = dx[0] * sF[0][v][bx], ay = dy[0] * sF[1][v][by], az = dz[0] * sF[2][v][bz];
#pragma unroll
    for (int b = 1; b < 4; ++b) {
      ax += dx[b] * sF[0][v][bx + b];
      ay += dy[b] * sF[1][v][by + 4 * b];
      az += dz[b] * sF[2][v][bz + 16 * b];
    }
    Rv[v] += sx * ax;
    Rv[v] += sy * ay;
    Rv[v] += sz * az;
    __builtin_amdgcn_sched_barrier(0);
  }
}

// eval_point with the background taken from a wavefront's LDS table
// (fields rho_d, rho_m, rho_r, E, p; column h)
template <typename R, int D, int RAIN>
__device__ __forceinline__ void eval_tab(const KArgs& a, const R* Uq, double T, double rvs, const double (*sB)[6],
                                         int h, Pt<R, D, RAIN>& q) {
  using V = Vars<D, RAIN>;
  const double bm = sB[1][h];
  const double rv = fmin(rvs, bm + (double)Uq[V::RM]);
  eval_core<R, D, RAIN>(a, Uq, T, rv, rvs, sB[0][h], bm, RAIN ? sB[2][h] : 0.0, sB[3][h], sB[4][h], q);
}

template <typename R, int RAIN, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(min_waves<R>())))
rhs_q3_kernel(KArgs a, const R* __restrict__ U, const double* __restrict__ auxT,
              const double* __restrict__ auxS, R* __restrict__ out, const R* __restrict__ U0,
              const double* __restrict__ dt_m, double c0, double c1, double c2, double* __restrict__ oT,
              double* __restrict__ oS, int flags) {
  constexpr int K = 3, P1 = 4, NP = 64, D = 3;
  using V = Vars<D, RAIN>;
  constexpr int NV = V::NV;
  constexpr int WPB = block_threads<R>() / NP;   // wavefronts (elements) per block
  // per-wavefront LDS tiles: fluxes of the three directions (later the face
  // corrections), the state, the wave speeds
  __shared__ R sF_all[WPB][D][NV][NP];
  __shared__ R sU_all[WPB][NV][NP];
  __shared__ R sL_all[WPB][D][NP];
  // background (rho_d, rho_m, rho_r, E, p) at the element's four heights and
  // at the face heights of the neighbours below and above
  __shared__ double sB_all[WPB][5][6];
  __shared__ R sD[P1 * P1];
  if (threadIdx.x < P1 * P1) sD[threadIdx.x] = (R)a.Dhat[threadIdx.x];
  __syncthreads();   // the only block-wide barrier: the shared D-hat table

  const ItemWalk walk(a.nitems, a.walk_rev);
  const int it_ = walk.item(0);
  if (it_ < 0) return;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int lane = (int)(threadIdx.x & 63);
  const Item item = a.items[it_];
  const MemberDesc& md = a.mem[item.member];
  const int e = item.e0 + w;
  if (e >= md.ne) return;                  // wave-uniform
  R(*sF)[NV][NP] = sF_all[w];
  R(*sU)[NP] = sU_all[w];
  R(*sL)[NP] = sL_all[w];
  double(*sB)[6] = sB_all[w];

  // element (scalar): coordinates, neighbours per (direction, side), walls
  const ElemCoord<D> ec = item_coord<D>(md, item, w);
  int nbe[3][2];
  bool wall[3][2];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const int c = ec.c[j], n = md.n[j], st = elem_stride(md, j);
    wall[j][0] = (c == 0) && md.bc[j] == 1;
    wall[j][1] = (c == n - 1) && md.bc[j] == 1;
    nbe[j][0] = e + ((c == 0) ? (n - 1) * st : -st);
    nbe[j][1] = e + ((c == n - 1) ? -(n - 1) * st : st);
  }
  const unsigned N = a.nnodes;
  const unsigned gbase = (unsigned)(md.eoff + e) * NP;   // first node of the element
  const unsigned g = gbase + lane;
  const int li = lane & 3, lj = (lane >> 2) & 3, ll = lane >> 4;
  // this node on a slip wall (wx, wy, wz) or on a face with a neighbour (fx, fy, fz)
  const bool ox0 = li == 0, ox1 = li == K, oy0 = lj == 0, oy1 = lj == K, oz0 = ll == 0, oz1 = ll == K;
  const bool wx = (ox0 & wall[0][0]) | (ox1 & wall[0][1]);
  const bool wy = (oy0 & wall[1][0]) | (oy1 & wall[1][1]);
  const bool wz = (oz0 & wall[2][0]) | (oz1 & wall[2][1]);
  const bool fx = (ox0 | ox1) & !wx, fy = (oy0 | oy1) & !wy, fz = (oz0 | oz1) & !wz;
  const int izb = md.hoff + ec.c[2] * P1;                // first height index of the element
  const int iz = izb + ll;
  // height index of the neighbours' face layers below and above (periodic wrap)
  const int izn_lo = md.hoff + (ec.c[2] == 0 ? md.n[2] - 1 : ec.c[2] - 1) * P1 + K;
  const int izn_hi = md.hoff + (ec.c[2] == md.n[2] - 1 ? 0 : ec.c[2] + 1) * P1;

  // face task of pass 0 (x and y faces): direction jx/jy, side, face node
  const bool t0x = lane < 32;
  const int t0s = (lane >> 4) & 1;
  const int t0a = lane & 3, t0b = (lane >> 2) & 3;
  // own node of the task and the matching node of the neighbour
  const int n0 = t0x ? (t0s * K + P1 * t0a + P1 * P1 * t0b) : (t0a + P1 * t0s * K + P1 * P1 * t0b);
  const int nn0 = t0x ? (n0 + (t0s ? -K : K)) : (n0 + (t0s ? -K * P1 : K * P1));
  const int en0 = t0x ? (t0s ? nbe[0][1] : nbe[0][0]) : (t0s ? nbe[1][1] : nbe[1][0]);
  const bool w0 = t0x ? (t0s ? wall[0][1] : wall[0][0]) : (t0s ? wall[1][1] : wall[1][0]);
  // (wall tasks read their own node: in range, unused)
  const unsigned gn0 = w0 ? g : (unsigned)(md.eoff + en0) * NP + nn0;
  // face task of pass 1 (z faces, lanes 0..31)
  const int t1s = (lane >> 4) & 1;
  const int n1 = (lane & 15) + P1 * P1 * K * t1s;
  const int nn1 = n1 + (t1s ? -K * P1 * P1 : K * P1 * P1);
  const bool a1 = lane < 32;
  const bool w1 = t1s ? wall[2][1] : wall[2][0];
  const int en1 = t1s ? nbe[2][1] : nbe[2][0];
  const unsigned gn1 = (!a1 || w1) ? g : (unsigned)(md.eoff + en1) * NP + nn1;

  // background table: lane 6 f + h loads field f at height h (issued with the
  // own loads, stored after the evaluation)
  double bgt = 0.0;
  {
    const int f = lane / 6, h = lane - 6 * (lane / 6);
    const int izt = h < 4 ? izb + h : (h == 4 ? izn_lo : izn_hi);
    const double* src = f == 0 ? a.bg_rd : (f == 1 ? a.bg_rm : (f == 2 ? a.bg_rr : (f == 3 ? a.bg_E : a.bg_p)));
    if (lane < 30 && (RAIN || f != 2)) bgt = src[izt];
  }
  // 1. own state
  R Uq[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Uq[v] = ld(U, N, v, g);
  const double T = ld(auxT, N, 0, g), rvs = ld(auxS, N, 0, g);

  // 2. point state, fluxes, wave speeds to LDS
  Pt<R, D, RAIN> q;
  eval_point<R, D, RAIN>(a, Uq, T, rvs, iz, q);
  {
    R F[NV];
    flux<R, D, RAIN, 0>(q, F);
#pragma unroll
    for (int v = 0; v < NV; ++v) sF[0][v][lane] = F[v];
    flux<R, D, RAIN, 1>(q, F);
#pragma unroll
    for (int v = 0; v < NV; ++v) sF[1][v][lane] = F[v];
    flux<R, D, RAIN, 2>(q, F);
#pragma unroll
    for (int v = 0; v < NV; ++v) sF[2][v][lane] = F[v];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) sU[v][lane] = Uq[v];
  sL[0][lane] = wave_speed<R, D, RAIN, 0>(q);
  sL[1][lane] = wave_speed<R, D, RAIN, 1>(q);
  sL[2][lane] = wave_speed<R, D, RAIN, 2>(q);
  if (lane < 30) (&sB[0][0])[lane] = bgt;
  // the neighbour traces of the first face pass: in flight during the volume term
  R Un0[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Un0[v] = ld(U, N, v, gn0);
  const double Tn0 = ld(auxT, N, 0, gn0), rvsn0 = ld(auxS, N, 0, gn0);
  wave_lds_sync();

  // 3. volume term, slip walls, sources
  R Rv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Rv[v] = R(0);
  volume_q3<R, RAIN>(md, li, lj, ll, lane, sF, Rv, sD);
  {
    Nb<R, D, RAIN> none;
    if (wx) face_dir<R, K, D, RAIN, 0>(a, md, li, iz, Uq, q, none, true, -1, Rv);
    if (wy) face_dir<R, K, D, RAIN, 1>(a, md, lj, iz, Uq, q, none, true, -1, Rv);
    if (wz) face_dir<R, K, D, RAIN, 2>(a, md, ll, iz, Uq, q, none, true, -1, Rv);
  }
  sources<R, D, RAIN>(a, Uq, q, Rv);
  wave_lds_sync();   // the volume term has read sF before the faces overwrite it

  // the neighbour traces of the second face pass: in flight during the first
  R Un1[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Un1[v] = ld(U, N, v, gn1);
  const double Tn1 = ld(auxT, N, 0, gn1), rvsn1 = ld(auxS, N, 0, gn1);
  // 4. face passes: the lifted Lax-Friedrichs correction replaces F_J at the
  // own node: +-(lift/2)(F + F_n) + (lift/2) Lambda (U_n - U), + on the minus face
  const R half = R(0.5);
  if (!w0) {
    Pt<R, D, RAIN> qn;
    eval_tab<R, D, RAIN>(a, Un0, Tn0, rvsn0, sB, t0b, qn);
    R Fn[NV];
    flux_h<R, RAIN>(qn, t0x, Fn);
    const R ln = fabs(t0x ? qn.u[0] : qn.u[1]) + qn.cm;
    const int J = t0x ? 0 : 1;
    const R lo = sL[J][n0];
    const bool own = t0s ? (lo >= ln) : !(ln >= lo);
    const R Lam = own ? lo : ln;
    const double l00 = md.lift[0][0], l01 = md.lift[0][1], l10 = md.lift[1][0], l11 = md.lift[1][1];
    const R lift = (R)(t0x ? (t0s ? l01 : l00) : (t0s ? l11 : l10));
    const R hl = half * lift;
    const R kf = t0s ? -hl : hl;
    const R kj = hl * Lam;
#pragma unroll
    for (int v = 0; v < NV; ++v) sF[J][v][n0] = fma(kf, sF[J][v][n0] + Fn[v], kj * (Un0[v] - sU[v][n0]));
  }
  {
    if (a1 && !w1) {
      Pt<R, D, RAIN> qn;
      eval_tab<R, D, RAIN>(a, Un1, Tn1, rvsn1, sB, t1s ? 5 : 4, qn);
      R Fn[NV];
      flux<R, D, RAIN, 2>(qn, Fn);
      const R ln = wave_speed<R, D, RAIN, 2>(qn);
      const R lo = sL[2][n1];
      const bool own = t1s ? (lo >= ln) : !(ln >= lo);
      const R Lam = own ? lo : ln;
      const double l20 = md.lift[2][0], l21 = md.lift[2][1];
      const R hl = half * (R)(t1s ? l21 : l20);
      const R kf = t1s ? -hl : hl;
      const R kj = hl * Lam;
#pragma unroll
      for (int v = 0; v < NV; ++v) sF[2][v][n1] = fma(kf, sF[2][v][n1] + Fn[v], kj * (Un1[v] - sU[v][n1]));
    }
  }
  // operands of the update and the split, fetched while the faces finish
  R U0q[NV];
  double bg[4] = {0.0, 0.0, 0.0, 0.0};
  if (MODE != 0 && c0 != 0.0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) U0q[v] = ld(U0, N, v, g);
  }
  if (MODE == 2) {
    bg[0] = sB[0][ll];
    bg[1] = sB[1][ll];
    if (RAIN) bg[2] = sB[2][ll];
    bg[3] = sB[3][ll];
  }
  wave_lds_sync();

  // 5. face corrections of this node, then the stage epilogue
  if (fx) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Rv[v] += sF[0][v][lane];
  }
  if (fy) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Rv[v] += sF[1][v][lane];
  }
  if (fz) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Rv[v] += sF[2][v][lane];
  }
  if (flags & kSip) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Rv[v] += ld((const R*)a.sip_out, N, v, g);
  }
  const double dtm = (MODE != 0) ? dt_m[item.member] : 0.0;
  int iters = 0, bad = 0;
#pragma unroll
  for (int v = 0; v < NV; ++v) Uq[v] = sU[v][lane];
  // with kSipAlpha, the new state's element viscosity (Section 3.5) for the
  // next stage's diffusion: the node shares, then the pairwise sum over the
  // wavefront in the order of sip_alpha_kernel's tree
  double at[2] = {0.0, 0.0};
  const double wq = md.J * a.w[li] * a.w[lj] * a.w[ll];
  stage_epilogue<R, D, RAIN, MODE>(a, bg, iz, g, N, Uq, U0q, Rv, T, rvs, out, dtm, c0, c1, c2, oT, oS, flags,
                                   iters, bad, nullptr, nullptr, nullptr, wq, at);
  if (MODE == 2) record_stats(a, iters, bad);
  if (MODE == 2 && (flags & kSipAlpha)) {
#pragma unroll
    for (int h = 1; h < NP; h <<= 1) {
      at[0] += __shfl_down(at[0], h);
      at[1] += __shfl_down(at[1], h);
    }
    if (lane == 0) {
      a.sip_aK[md.eoff + e] = md.sip_pre * sqrt(at[0]);
      a.sip_aK[a.etot + md.eoff + e] = md.sip_pre * sqrt(at[1]);
    }
  }
}

}  // namespace dgm
