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

// The constant address space (read-only global memory; scalar loads) in the
// device pass.
#if defined(__HIP_DEVICE_COMPILE__)
#define DGM_AS_CONST __attribute__((address_space(4)))
#else
#define DGM_AS_CONST
#endif

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
// with stride gridDim/8.  gridDim.x is always a multiple of 8.  A reversed
// walk (rev) runs each XCD's range from the top down: every XCD keeps its
// own items (and so what its L2 holds of them) and starts on the ones it
// wrote last.
struct ItemWalk {
  int per, g8, x, l, nitems, rev;
  __device__ __forceinline__ explicit ItemWalk(int n, int reverse = 0) {
    nitems = n;
    rev = reverse;
    per = (n + 7) >> 3;
    g8 = gridDim.x >> 3;
    x = blockIdx.x & 7;
    l = blockIdx.x >> 3;
  }
  // item of the k-th iteration, or -1 when the walk is over (uniform per block)
  __device__ __forceinline__ int item(int k) const {
    const int li = l + k * g8;
    if (li >= per) return -1;
    const int it = x * per + (rev ? per - 1 - li : li);
    return it < nitems ? it : -1;
  }
};

__host__ __device__ inline int grid_for_items(int nitems) { return ((nitems + 7) >> 3) << 3; }

// flags of a stage launch
constexpr int kRefreshRvs = 1;   // store a fresh rho_vs(T) evaluation (anchors later splits)
constexpr int kSponge = 2;       // the stage ends a time step: apply the sponge
// the diffusive tendency in a.sip_out is added to the right-hand side
constexpr int kSip = 4;
// (Q3 stage kernel) the element viscosity alpha_K of the new state is written
// to a.sip_aK, so the next stage's diffusion need not compute it
constexpr int kSipAlpha = 8;

// One node's share of the element viscosity of Section 3.5: with quadrature
// weight w, w |u|^2 and w |u - v_r e_z|^2 (full densities rd, rm, rr, momentum
// m).  sip_alpha_kernel and the Q3 stage epilogue both call this, and both
// sum the shares over the element in the same pairwise order, so alpha_K has
// the same bits whichever kernel formed it.
template <int D, int RAIN>
__device__ __forceinline__ void sip_alpha_terms(const KArgs& a, double w, double rd, double rm, double rr,
                                                const double* m, double& s0, double& s1) {
  const double irho = 1.0 / (rd + rm + rr);
  double vr = 0.0;
  if (RAIN) vr = a.vr_mode == 0 ? a.vr_const : (rr > 0.0 ? a.vr_pref * pow(rr, 0.125) : 0.0);
  s0 = 0.0;
  s1 = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double ui = m[i] * irho;
    const double ur = (i == D - 1) ? ui - vr : ui;
    s0 += w * ui * ui;
    s1 += w * ur * ur;
  }
}

// The sponge at the end of a step (Section 3.6):
// (rho_m', rho_r', m, E') <- (1 - delta) (rho_m', rho_r', m, E') with the
// far field at rest, and the moist mass removed goes to rho_d' at the node.
template <typename R, int D, int RAIN>
__device__ __forceinline__ void sponge_point(const KArgs& a, int iz, R* Un) {
  using V = Vars<D, RAIN>;
  const R dl = (R)a.sponge[iz];
  if (dl == R(0)) return;
  R lost = Un[V::RM] * dl;
  if (RAIN) lost = lost + Un[V::RR] * dl;
  const R keep = R(1) - dl;
#pragma unroll
  for (int v = 1; v < V::NV; ++v) Un[v] = Un[v] * keep;
  Un[V::RD] = Un[V::RD] + lost;
}

// ---------------------------------------------------------------------------
// split kernel: (T, rho_vs) per node, or the API outputs (T, rho_v, rho_c)
// ---------------------------------------------------------------------------
template <typename R, int K, int D, int RAIN, int API>
__global__ void __launch_bounds__(256)
split_kernel(KArgs a, int item0, int nitems, const R* __restrict__ U, const double* __restrict__ Tguess,
             double* __restrict__ oT, double* __restrict__ o1, double* __restrict__ o2) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NP = S::NP, NV = V::NV;
  // one work item per block (no item loop: loop-invariant values would stay
  // live across the body)
  const int it_ = ItemWalk(nitems).item(0);
  if (it_ < 0) return;
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

// ---------------------------------------------------------------------------
// right-hand side / stage kernel
// ---------------------------------------------------------------------------
// MODE 0: out = dU/dt
// MODE 1: out = c0 U0 + c1 U + c2 dt_member dU/dt  (a Shu-Osher stage)
// MODE 2: as MODE 1, then the split of the new state at every node, written
//         to (oT, oS); Newton is warm-started and anchored at the input
//         state's (T, rho_vs).  With kRefreshRvs the stored rho_vs is a fresh
//         evaluation at the new T (once per step), otherwise the anchored one.
// With kSponge (MODE 1, 2) the new state is the end of a step: the sponge
// acts on it before it is stored and split.
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
  using S = Shape<K, D, block_threads<R>()>;
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
                                           const R* sD, int t = threadIdx.x) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NV = V::NV;
  constexpr int STR = (J == 0) ? 1 : (J == 1 ? P1 : P1 * P1);
    constexpr int NT = S::NT;   // LDS row stride (the largest block)
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
  constexpr int NT = Shape<K, D, block_threads<R>()>::NT;   // LDS row stride (the largest block)
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
    const R lift = (R)md.lift[J][1];
#pragma unroll
    for (int v = 0; v < NV; ++v) Rv[v] -= lift * (half * (F[v] + Fn[v]) + half * Lam * (Uq[v] - Un[v]));
  } else {
    const R lift = (R)md.lift[J][0];
#pragma unroll
    for (int v = 0; v < NV; ++v) Rv[v] += lift * (half * (Fn[v] + F[v]) + half * Lam * (Un[v] - Uq[v]));
  }
}

// Face work of a block as (element, direction J, side, face node) pairs, PE =
// 2 (K+1)^(D-1) per element and direction.  The pairs of one direction are cut
// into slot-waves of WL = min(64, NT) lanes; full wavefronts take the
// slot-waves in turn, so every lane of a pass holds one face node (a
// node-per-thread face loop leaves the lanes of interior nodes idle in each
// of the D directions) and J is uniform across a wavefront.
template <int K, int D>
struct FaceShape {
  static constexpr int P1 = K + 1;
  static constexpr int FN = (D == 2) ? P1 : P1 * P1;  // nodes per face
  static constexpr int NP = Shape<K, D>::NP;
};

struct SlotPlan {
  int wl, pj, swj, sw, nfull, wave, lane;
  __device__ __forceinline__ SlotPlan(int NT, int NP, int FN, int dim, int t) {
    wl = NT < 64 ? NT : 64;
    pj = (NT / NP) * 2 * FN;
    swj = (pj + wl - 1) / wl;
    sw = dim * swj;
    nfull = NT / wl;
    wave = t / wl;
    lane = t - wave * wl;
  }
  // slot-wave of pass k for this thread's wavefront, or -1
  __device__ __forceinline__ int slot_wave(int k) const {
    if (wave >= nfull) return -1;
    const int s = wave + k * nfull;
    return s < sw ? __builtin_amdgcn_readfirstlane(s) : -1;
  }
};

template <typename R, int D, int RAIN>
struct Pair {
  Nb<R, D, RAIN> nb;
  int slot;   // block slot (le * NP + n) of the own node; -1: nothing to do
  int side, izn;
};

// Pair q of direction J: decode the own node and gather the neighbour's trace.
// Inactive elements and wall faces get slot = -1 (the node's own thread handles
// walls: the ghost is its own reflected point state).
template <typename R, int K, int D, int RAIN, int J>
__device__ __forceinline__ void pair_gather(const MemberDesc& md, const Item& item, int q, int pj,
                                            const R* __restrict__ U, const double* __restrict__ auxT,
                                            const double* __restrict__ auxS, unsigned N,
                                            Pair<R, D, RAIN>& pr) {
  using FS = FaceShape<K, D>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = FS::P1, FN = FS::FN, NP = FS::NP, NV = V::NV;
  constexpr int STR = (J == 0) ? 1 : (J == 1 ? P1 : P1 * P1);
  pr.slot = -1;
  pr.side = 0;
  pr.izn = 0;
  if (q >= pj) return;
  const int le = q / (2 * FN);
  const int r = q - le * (2 * FN);
  const int side = r / FN;
  const int f = r - side * FN;
  const int e = item.e0 + le;
  if (e >= md.ne) return;
  // own node: index K*side along J, the face node f over the other axes
  const int fa = f % P1, fb = f / P1;
  int n;
  if (J == 0) n = side * K + P1 * fa + P1 * P1 * fb;
  else if (J == 1) n = fa + P1 * side * K + P1 * P1 * fb;
  else n = fa + P1 * fb + P1 * P1 * side * K;
  const ElemCoord<D> ec = item_coord<D>(md, item, le);
  const int c = ec.c[J];
  const bool at_end = side ? (c == md.n[J] - 1) : (c == 0);
  if (at_end && md.bc[J] == 1) return;
  int cn = side ? c + 1 : c - 1;
  if (cn < 0) cn += md.n[J];
  if (cn >= md.n[J]) cn -= md.n[J];
  const int en = e + (cn - c) * elem_stride(md, J);
  const int nn = side ? n - K * STR : n + K * STR;
  const unsigned gn = (unsigned)(md.eoff + en) * NP + nn;
#pragma unroll
  for (int v = 0; v < NV; ++v) pr.nb.U[v] = ld(U, N, v, gn);
  pr.nb.T = ld(auxT, N, 0, gn);
  pr.nb.rvs = ld(auxS, N, 0, gn);
  const int lz = (D == 2) ? (J == 0 ? fa : side * K) : (J == 2 ? side * K : fb);
  pr.izn = md.hoff + ((J == D - 1) ? cn * P1 + (side ? 0 : K) : ec.c[D - 1] * P1 + lz);
  pr.slot = le * NP + n;
  pr.side = side;
}

template <typename R, int K, int D, int RAIN>
__device__ __forceinline__ void pair_gather_rt(int J, const MemberDesc& md, const Item& item, int q, int pj,
                                               const R* __restrict__ U, const double* __restrict__ auxT,
                                               const double* __restrict__ auxS, unsigned N,
                                               Pair<R, D, RAIN>& pr) {
  if (J == 0) pair_gather<R, K, D, RAIN, 0>(md, item, q, pj, U, auxT, auxS, N, pr);
  else if (D == 2 || J == 1) pair_gather<R, K, D, RAIN, 1>(md, item, q, pj, U, auxT, auxS, N, pr);
  else pair_gather<R, K, D, RAIN, (D == 3 ? 2 : 1)>(md, item, q, pj, U, auxT, auxS, N, pr);
}

// Lax-Friedrichs flux of one pair (Section 3.2): the own trace (U, F_J,
// lambda_J) comes from the block's LDS tiles, the neighbour's is evaluated
// here.  The lifted correction replaces F_J at the own slot of sF:
// +-(lift/2)(F + F_n) + (lift/2) Lambda (U_n - U), + on the minus face.
template <typename R, int K, int D, int RAIN, int J>
__device__ __forceinline__ void pair_flux(const KArgs& a, const MemberDesc& md, const Pair<R, D, RAIN>& pr,
                                          R* sF, const R* sU, const R* sL) {
  using V = Vars<D, RAIN>;
  constexpr int NV = V::NV;
  constexpr int NT = Shape<K, D, block_threads<R>()>::NT;
  if (pr.slot < 0) return;
  Pt<R, D, RAIN> qn;
  eval_point<R, D, RAIN>(a, pr.nb.U, pr.nb.T, pr.nb.rvs, pr.izn, qn);
  R Fn[NV];
  flux<R, D, RAIN, J>(qn, Fn);
  const R ln = wave_speed<R, D, RAIN, J>(qn);
  R* F = sF + J * (NV * NT) + pr.slot;
  const R* Uo = sU + pr.slot;
  const R lo = sL[J * NT + pr.slot];
  // Lambda = max over the two sides, ties to the minus side
  const bool own = pr.side ? (lo >= ln) : !(ln >= lo);
  const R Lam = own ? lo : ln;
  const R hl = R(0.5) * (pr.side ? (R)md.lift[J][1] : (R)md.lift[J][0]);
  const R kf = pr.side ? -hl : hl;
  const R kj = hl * Lam;
#pragma unroll
  for (int v = 0; v < NV; ++v) F[v * NT] = fma(kf, F[v * NT] + Fn[v], kj * (pr.nb.U[v] - Uo[v * NT]));
}

template <typename R, int K, int D, int RAIN>
__device__ __forceinline__ void pair_flux_rt(int J, const KArgs& a, const MemberDesc& md,
                                             const Pair<R, D, RAIN>& pr, R* sF, const R* sU, const R* sL) {
  if (J == 0) pair_flux<R, K, D, RAIN, 0>(a, md, pr, sF, sU, sL);
  else if (D == 2 || J == 1) pair_flux<R, K, D, RAIN, 1>(a, md, pr, sF, sU, sL);
  else pair_flux<R, K, D, RAIN, (D == 3 ? 2 : 1)>(a, md, pr, sF, sU, sL);
}

// Stage update and the split epilogue shared by both face schemes.
template <typename R, int D, int RAIN, int MODE>
__device__ __forceinline__ void stage_epilogue(const KArgs& a, const double* bg, int iz, unsigned g, unsigned N,
                                               const R* Uq, const R* U0q, const R* Rv, double T, double rvs,
                                               R* __restrict__ out, double dtm, double c0, double c1,
                                               double c2, double* __restrict__ oT,
                                               double* __restrict__ oS, int flags, int& iters, int& bad,
                                               R* Unew = nullptr, double* Tnew = nullptr,
                                               double* Snew = nullptr, double wq = 0.0,
                                               double* alpha_terms = nullptr) {
  // (Unew, Tnew, Snew), when given, receive the stored new state and its
  // stored (T, rho_vs); alpha_terms, when given with kSipAlpha, the node's
  // shares of the new state's element viscosity (weight wq)
  using V = Vars<D, RAIN>;
  constexpr int NV = V::NV;
  if (MODE == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) st(out, N, v, g, Rv[v]);
    return;
  }
  const R k2 = (R)(c2 * dtm);
  const R k1 = (R)c1;
  R Un[NV];
  if (c0 != 0.0) {
    const R k0 = (R)c0;
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[v] = k0 * U0q[v] + k1 * Uq[v] + k2 * Rv[v];
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[v] = k1 * Uq[v] + k2 * Rv[v];
  }
  if (flags & kSponge) sponge_point<R, D, RAIN>(a, iz, Un);
#pragma unroll
  for (int v = 0; v < NV; ++v) st(out, N, v, g, Un[v]);
  if (alpha_terms && (flags & kSipAlpha)) {
    double m[D];
#pragma unroll
    for (int i = 0; i < D; ++i) m[i] = (double)Un[V::M0 + i];
    sip_alpha_terms<D, RAIN>(a, wq, bg[0] + (double)Un[V::RD], bg[1] + (double)Un[V::RM],
                             RAIN ? bg[2] + (double)Un[V::RR] : 0.0, m, alpha_terms[0], alpha_terms[1]);
  }
  if (Unew) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Unew[v] = Un[v];
  }
  if (MODE == 2) {
    // split of the new state (FP64), warm-started at this node's (T, rho_vs);
    // bg = (rho_d, rho_m, rho_r, E) of the background at this node
    const double rd = bg[0] + (double)Un[V::RD];
    const double rm = bg[1] + (double)Un[V::RM];
    const double rr = RAIN ? bg[2] + (double)Un[V::RR] : 0.0;
    double ke = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double mi = (double)Un[V::M0 + i];
      ke += mi * mi;
    }
    const double re = bg[3] + (double)Un[V::E] - 0.5 * ke * rcp64(rd + rm + rr);
    Anchor A;
    A.T0 = 0.0; A.r0 = 0.0; A.inv0 = 0.0;
    if (T > 150.0 && T < 600.0 && rvs > 0.0) {
      A.T0 = T; A.r0 = rvs; A.inv0 = rcp64(T);
    }
    // the branch that held at this node before is tried first
    const SplitOut s = split_point_anchor(a, rd, rm, rr, re, T, A, rvs < rm);
    iters = s.iters;
    bad = s.bad;
    const double rvs_st = ((flags & kRefreshRvs) && s.bad == 0) ? rho_vs(a, s.T) : s.rvs;
    st(oT, N, 0, g, s.T);
    st(oS, N, 0, g, rvs_st);
    if (Tnew) *Tnew = s.T;
    if (Snew) *Snew = rvs_st;
  }
}

// Right-hand side / stage of one work item with the lane-dense face pass
// (K >= 2, where a node lies on at most one face per direction).  LDS tiles
// use the compile-time stride NT of the largest block; smaller blocks use a
// prefix of each row.
template <typename R, int K, int D, int RAIN, int MODE>
__device__ __forceinline__ void rhs_item_pairs(const KArgs& a, int t, int it_, R* sF, R* sU, R* sL,
                                               const R* sD, const R* __restrict__ U,
                                               const double* __restrict__ auxT,
                                               const double* __restrict__ auxS, R* __restrict__ out,
                                               const R* __restrict__ U0, const double* __restrict__ dt_m,
                                               double c0, double c1, double c2, double* __restrict__ oT,
                                               double* __restrict__ oS, int flags) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  using FS = FaceShape<K, D>;
  constexpr int P1 = S::P1, NP = S::NP, NV = V::NV, NT = S::NT;
  static_assert(K >= 2, "pair face pass needs K >= 2");
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
    for (int v = 0; v < NV; ++v) Uq[v] = ld(U, N, v, g);
    T = ld(auxT, N, 0, g);
    rvs = ld(auxS, N, 0, g);
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) Uq[v] = R(0);
  }
  const SlotPlan sp((int)blockDim.x, NP, FS::FN, D, t);

  Pt<R, D, RAIN> q;
  eval_point<R, D, RAIN>(a, Uq, T, rvs, active ? iz : md.hoff, q);
  {
    R F[NV];
    flux<R, D, RAIN, 0>(q, F);
#pragma unroll
    for (int v = 0; v < NV; ++v) sF[v * NT + t] = F[v];
    flux<R, D, RAIN, 1>(q, F);
#pragma unroll
    for (int v = 0; v < NV; ++v) sF[(NV + v) * NT + t] = F[v];
    if constexpr (D == 3) {
      flux<R, D, RAIN, 2>(q, F);
#pragma unroll
      for (int v = 0; v < NV; ++v) sF[(2 * NV + v) * NT + t] = F[v];
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) sU[v * NT + t] = Uq[v];
  sL[t] = wave_speed<R, D, RAIN, 0>(q);
  sL[NT + t] = wave_speed<R, D, RAIN, 1>(q);
  if constexpr (D == 3) sL[2 * NT + t] = wave_speed<R, D, RAIN, 2>(q);
  __syncthreads();
  R U0q[NV];
  double bg[4] = {0.0, 0.0, 0.0, 0.0};
  const double dtm = (MODE != 0) ? dt_m[item.member] : 0.0;
  R Rv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Rv[v] = R(0);
  bool fa[3], wl[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    fa[j] = j < D && active && (idx[j] == 0 || idx[j] == K);
    const bool at_end = (idx[j] == K) ? (ec.c[j] == md.n[j] - 1) : (ec.c[j] == 0);
    wl[j] = fa[j] && at_end && md.bc[j] == 1;
  }
  // 2D: the first face pass's neighbour traces are in flight during the
  // volume term (in 3D the registers they hold would cost a wavefront per
  // SIMD at some orders)
  Pair<R, D, RAIN> p0;
  const int s0 = sp.slot_wave(0);
  const int J0 = s0 >= 0 ? s0 / sp.swj : 0;
  if (D == 2 && s0 >= 0)
    pair_gather_rt<R, K, D, RAIN>(J0, md, item, (s0 - J0 * sp.swj) * sp.wl + sp.lane, sp.pj, U, auxT, auxS, N, p0);
  if (active) {
    volume_dir<R, K, D, RAIN, 0>(md, idx[0], sF, Rv, sD, t);
    volume_dir<R, K, D, RAIN, 1>(md, idx[1], sF + NV * NT, Rv, sD, t);
    if constexpr (D == 3) volume_dir<R, K, D, RAIN, 2>(md, idx[2], sF + 2 * NV * NT, Rv, sD, t);
    // slip walls: the ghost is this node's own reflected state
    Nb<R, D, RAIN> none;
    if (wl[0]) face_dir<R, K, D, RAIN, 0>(a, md, idx[0], iz, Uq, q, none, true, -1, Rv);
    if (wl[1]) face_dir<R, K, D, RAIN, 1>(a, md, idx[1], iz, Uq, q, none, true, -1, Rv);
    if constexpr (D == 3) {
      if (wl[2]) face_dir<R, K, D, RAIN, 2>(a, md, idx[2], iz, Uq, q, none, true, -1, Rv);
    }
    sources<R, D, RAIN>(a, Uq, q, Rv);
  }
  __syncthreads();   // the volume term has read sF
  // face passes: in 3D the neighbour traces are gathered here, not ahead of
  // the volume term, and every pass runs the same code, so the rounding of a
  // face flux does not depend on the pass (the launch geometry) that
  // computes it
  if (D == 2 && s0 >= 0) pair_flux_rt<R, K, D, RAIN>(J0, a, md, p0, sF, sU, sL);
#pragma clang loop unroll(disable)
  for (int k = (D == 2 ? 1 : 0); s0 >= 0; ++k) {
    const int s = sp.slot_wave(k);
    if (s < 0) break;
    const int J = s / sp.swj;
    Pair<R, D, RAIN> p1;
    pair_gather_rt<R, K, D, RAIN>(J, md, item, (s - J * sp.swj) * sp.wl + sp.lane, sp.pj, U, auxT, auxS, N,
                                  p1);
    pair_flux_rt<R, K, D, RAIN>(J, a, md, p1, sF, sU, sL);
  }
  // operands of the stage update and the split, fetched while the faces of
  // the other wavefronts finish
  if (MODE != 0 && active && c0 != 0.0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) U0q[v] = ld(U0, N, v, g);
  }
  if (MODE == 2 && active) {
    bg[0] = a.bg_rd[iz];
    bg[1] = a.bg_rm[iz];
    if (RAIN) bg[2] = a.bg_rr[iz];
    bg[3] = a.bg_E[iz];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < D; ++j)
    if (fa[j] && !wl[j]) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Rv[v] += sF[(j * NV + v) * NT + t];
    }
  int iters = 0, bad = 0;
  if (active) {
    R Us[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Us[v] = sU[v * NT + t];
    if (flags & kSip) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Rv[v] += ld((const R*)a.sip_out, N, v, g);
    }
    stage_epilogue<R, D, RAIN, MODE>(a, bg, iz, g, N, Us, U0q, Rv, T, rvs, out, dtm, c0, c1, c2, oT, oS, flags,
                                     iters, bad);
  }
  if (MODE == 2) record_stats(a, iters, bad);
}

template <typename R, int K, int D, int RAIN, int MODE>
__device__ __forceinline__ void rhs_item(const KArgs& a, int it_, R (*sF)[Vars<D, RAIN>::NV * Shape<K, D, block_threads<R>()>::NT],
                                         const R* sD, const R* __restrict__ U,
                                         const double* __restrict__ auxT,
                                         const double* __restrict__ auxS, R* __restrict__ out,
                                         const R* __restrict__ U0, const double* __restrict__ dt_m,
                                         double c0, double c1, double c2, double* __restrict__ oT,
                                         double* __restrict__ oS, int flags) {
  using S = Shape<K, D, block_threads<R>()>;
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
    if (flags & kSip) {
#pragma unroll
      for (int v = 0; v < NV; ++v) Rv[v] += (((const R*)a.sip_out) + (size_t)v * N)[g];
    }
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
      if (MODE != 0 && (flags & kSponge)) sponge_point<R, D, RAIN>(a, iz, Un);
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
        oS[g] = ((flags & kRefreshRvs) && s.bad == 0) ? rho_vs(a, s.T) : s.rvs;
      }
    }
  }
  if (MODE == 2) record_stats(a, iters, bad);
}

// one work item per block
// FP32: at least 4 wavefronts per SIMD (the register budget the kernel fits
// without spills); FP64 kernels need more registers than that and are left to
// the compiler (spills cost far more than the occupancy they buy).
template <typename R>
constexpr int min_waves() { return sizeof(R) == 4 ? 4 : 1; }

template <typename R, int K, int D, int RAIN, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(min_waves<R>())))
rhs_kernel(KArgs a, const R* __restrict__ U, const double* __restrict__ auxT,
           const double* __restrict__ auxS, R* __restrict__ out, const R* __restrict__ U0,
           const double* __restrict__ dt_m, double c0, double c1, double c2,
           double* __restrict__ oT, double* __restrict__ oS, int flags) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1;
  constexpr bool PAIRS = K >= 2;
  __shared__ R sF[D][V::NV * S::NT];
  __shared__ R sD[P1 * P1];
  __shared__ R sU[PAIRS ? V::NV * S::NT : 1];
  __shared__ R sL[PAIRS ? D * S::NT : 1];
  if (threadIdx.x < P1 * P1) sD[threadIdx.x] = (R)a.Dhat[threadIdx.x];
  const ItemWalk walk(a.nitems, a.walk_rev);
  const int it_ = walk.item(0);
  if (it_ < 0) return;
  if constexpr (PAIRS)
    rhs_item_pairs<R, K, D, RAIN, MODE>(
        a, threadIdx.x, it_, &sF[0][0], sU, sL, sD, U, auxT, auxS, out, U0, dt_m, c0, c1, c2, oT, oS, flags);
  else
    rhs_item<R, K, D, RAIN, MODE>(a, it_, sF, sD, U, auxT, auxS, out, U0, dt_m, c0, c1, c2, oT, oS, flags);
}

// persistent: a grid smaller than the item count walks the items
template <typename R, int K, int D, int RAIN, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(min_waves<R>())))
rhs_kernel_persistent(KArgs a, const KArgs* __restrict__ a_dev, const R* __restrict__ U,
                      const double* __restrict__ auxT,
                      const double* __restrict__ auxS, R* __restrict__ out, const R* __restrict__ U0,
                      const double* __restrict__ dt_m, double c0, double c1, double c2,
                      double* __restrict__ oT, double* __restrict__ oS, int flags) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1;
  constexpr bool PAIRS = K >= 2;
  __shared__ R sF[D][V::NV * S::NT];
  __shared__ R sD[P1 * P1];
  __shared__ R sU[PAIRS ? V::NV * S::NT : 1];
  __shared__ R sL[PAIRS ? D * S::NT : 1];
  if (threadIdx.x < P1 * P1) sD[threadIdx.x] = (R)a.Dhat[threadIdx.x];
  const ItemWalk walk(a.nitems);
#pragma clang loop unroll(disable)
  for (int kk = 0;; ++kk) {
    const int it_ = walk.item(kk);
    if (it_ < 0) break;
    // The argument block (its device copy a_dev) and the thread index pass
    // through opaque copies in every iteration: constants and per-thread
    // values hoisted out of the loop would stay live across it and exhaust
    // the registers.
    unsigned long long apv = (unsigned long long)a_dev;
    asm volatile("" : "+s"(apv));
    // constant address space: the block is read-only during the launch, so
    // its fields are scalar loads
    const KArgs DGM_AS_CONST* ap = (const KArgs DGM_AS_CONST*)apv;
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    if constexpr (PAIRS)
      rhs_item_pairs<R, K, D, RAIN, MODE>(*ap, t, it_, &sF[0][0], sU, sL, sD, U, auxT, auxS, out, U0, dt_m,
                                          c0, c1, c2, oT, oS, flags);
    else
      rhs_item<R, K, D, RAIN, MODE>(a, it_, sF, sD, U, auxT, auxS, out, U0, dt_m, c0, c1, c2, oT, oS, flags);
    __syncthreads();   // the LDS tiles are reused by the next item
  }
}



// ---------------------------------------------------------------------------
// conservation diagnostics: per-block FP64 partial sums in a fixed order
// ---------------------------------------------------------------------------
template <typename R, int K, int D, int RAIN>
__global__ void __launch_bounds__(256)
mass_kernel(KArgs a, int item0, const R* __restrict__ U, double* __restrict__ partial) {
  // (blocks map to items in order here: partials are summed in a fixed order)
  using S = Shape<K, D, block_threads<R>()>;
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
    // rain through the slip walls: with Lobatto nodes the wall is a node
    // layer; with Gauss nodes the thread of the lowest (highest) node of each
    // vertical line takes the trace of rho_r' along it at the floor (lid),
    // plus the background's face trace
    if (RAIN && md.bc[D - 1] == 1) {
      const ElemCoord<D> ec = item_coord<D>(md, item, le);
      const int l = idx[D - 1];
      const bool bottom = ec.c[D - 1] == 0 && l == 0;
      const bool top = ec.c[D - 1] == md.n[D - 1] - 1 && l == K;
      if (bottom || top) {
        double rr;
        if (a.basis == 0) {
          rr = a.bg_rr[md.hoff + ec.c[D - 1] * P1 + l] + (double)U[V::RR * N + g];
        } else {
          constexpr int ZS = (D == 2) ? P1 : P1 * P1;   // node stride along the vertical
          const double* Lt = bottom ? a.gl_m : a.gl_p;
          const size_t g0 = g - (size_t)l * ZS;
          double tr = 0.0;
          for (int m = 0; m < P1; ++m) tr += Lt[m] * (double)U[V::RR * N + g0 + (size_t)m * ZS];
          const int row = md.hoff / P1 + ec.c[D - 1];
          rr = a.bgf[2 * a.bgf_n + 2 * row + (bottom ? 0 : 1)] + tr;
        }
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

// ---------------------------------------------------------------------------
// transpose of the end-of-step sponge (the adjoint of dg_rk_step)
// ---------------------------------------------------------------------------
// Wp = S^T W for the pointwise sponge map S of sponge_point:
//   Wp[rho_d] = W[rho_d],  Wp[rho_m] = (1 - delta) W[rho_m] + delta W[rho_d],
//   Wp[rho_r] = (1 - delta) W[rho_r] + delta W[rho_d],  Wp[v] = (1 - delta) W[v]
//   for the momentum and E'.
template <typename R, int K, int D, int RAIN>
__global__ void __launch_bounds__(256)
sponge_vjp_kernel(KArgs a, const R* __restrict__ W, R* __restrict__ Wp) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NP = S::NP, NV = V::NV;
  const ItemWalk walk(a.nitems);
  for (int k = 0;; ++k) {
    const int it_ = walk.item(k);
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
    const R dl = (R)a.sponge[md.hoff + ec.c[D - 1] * P1 + l];
    const R keep = R(1) - dl;
    const R wd = ld(W, N, V::RD, g);
    st(Wp, N, V::RD, g, wd);
    st(Wp, N, V::RM, g, keep * ld(W, N, V::RM, g) + dl * wd);
    if (RAIN) st(Wp, N, V::RR, g, keep * ld(W, N, V::RR, g) + dl * wd);
#pragma unroll
    for (int v = V::M0; v < NV; ++v) st(Wp, N, v, g, keep * ld(W, N, v, g));
  }
}

}  // namespace dgm
