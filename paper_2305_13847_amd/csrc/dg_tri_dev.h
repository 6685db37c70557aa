// Device code on triangulations: the space P^k of Section 3.1 on a conforming
// triangulation of the vertical plane.
//
// A block holds a few elements with one thread per volume point of each
// (Duffy-mapped rule of the footnote in Section 3.4); coefficients and
// per-point results are exchanged through LDS, and a face point's thread
// gathers the neighbour's coefficients through the neighbour table to form
// the neighbour's trace at the shared point (Section 3.2).  The reference
// tables sit in constant memory.
//
// Precision as on the box meshes: the state, fluxes and accumulation in R,
// the reconstruction of full densities and p', the split and the projected T
// and rho_v in FP64.
#pragma once
#include <type_traits>

#include "dg_device.h"

namespace dgm {

template <int K>
struct TriShape {
  static constexpr int NP = (K + 1) * (K + 2) / 2;   // modes
  static constexpr int NQ = (K + 1) * (K + 2);       // volume points
  static constexpr int NF = K + 1;                   // points per face
};

// Reference tables of order K (filled on the host at handle creation).
template <typename R, int K>
struct TriTab {
  static constexpr int NP = TriShape<K>::NP, NQ = TriShape<K>::NQ, NF = TriShape<K>::NF;
  R psi[NQ][NP], dr[NQ][NP], ds[NQ][NP];   // basis and reference gradient at the volume points
  R w[NQ];                                  // volume weights (sum 1/2)
  double psid[NQ][NP];                      // the basis in FP64 (T, rho_v, split, projection)
  double wd[NQ];
  double rq[NQ], sq[NQ];                    // volume points
  R psif[3][NF][NP];                        // basis at the face points
  double psifd[3][NF][NP];
  R wf[NF];                                 // half the face Gauss weights
  double rf[3][NF], sf[3][NF];              // face points
  double xg[NF], lagd[NF];                  // layer Gauss heights on [-1, 1], 1 / prod_{j != i} (x_i - x_j)
};

__constant__ TriTab<float, 1> c_tri_f1;
__constant__ TriTab<float, 2> c_tri_f2;
__constant__ TriTab<float, 3> c_tri_f3;
__constant__ TriTab<float, 4> c_tri_f4;
__constant__ TriTab<double, 1> c_tri_d1;
__constant__ TriTab<double, 2> c_tri_d2;
__constant__ TriTab<double, 3> c_tri_d3;
__constant__ TriTab<double, 4> c_tri_d4;

template <typename R, int K>
__device__ __forceinline__ const TriTab<R, K>& ttab() {
  if constexpr (sizeof(R) == 4) {
    if constexpr (K == 1) return c_tri_f1;
    else if constexpr (K == 2) return c_tri_f2;
    else if constexpr (K == 3) return c_tri_f3;
    else return c_tri_f4;
  } else {
    if constexpr (K == 1) return c_tri_d1;
    else if constexpr (K == 2) return c_tri_d2;
    else if constexpr (K == 3) return c_tri_d3;
    else return c_tri_d4;
  }
}

struct TriArgs {
  const double* xy;   // ne x 3 x (x, z)
  const int* nbr;     // ne x 3: neighbour * 4 + its face; -1 slip wall
  const double* bgl;  // background [layer][height i][field]: rho_d, rho_m, rho_r, E, p
  double z0, inv_dz;
  int nz, ne;
};

// Vertex heights and layer of element e; the layer is the one holding the
// centroid.
struct TriZ {
  double z0, dz1, dz2;
  int layer;
};

__device__ __forceinline__ TriZ tri_z(const TriArgs& t, int e) {
  const double* v = t.xy + (size_t)e * 6;
  TriZ g;
  g.z0 = v[1];
  g.dz1 = v[3] - v[1];
  g.dz2 = v[5] - v[1];
  const double zc = (v[1] + v[3] + v[5]) * (1.0 / 3.0);
  int l = (int)floor((zc - t.z0) * t.inv_dz);
  g.layer = l < 0 ? 0 : (l >= t.nz ? t.nz - 1 : l);
  return g;
}

// Background (rho_d, rho_m, rho_r, E, p) at height z from layer l's
// degree-K interpolant through its Gauss heights.
template <typename R, int K>
__device__ __forceinline__ void tri_bg(const TriArgs& t, const TriTab<R, K>& T, int l, double z, double* b) {
  const double xi = 2.0 * ((z - t.z0) * t.inv_dz - (double)l) - 1.0;
  double ell[K + 1];
#pragma unroll
  for (int i = 0; i <= K; ++i) {
    double p = T.lagd[i];
#pragma unroll
    for (int j = 0; j <= K; ++j)
      if (j != i) p *= xi - T.xg[j];
    ell[i] = p;
  }
  const double* B = t.bgl + (size_t)l * (K + 1) * 5;
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    double v = 0.0;
#pragma unroll
    for (int i = 0; i <= K; ++i) v += ell[i] * B[i * 5 + f];
    b[f] = v;
  }
}

// The flux of Section 2.3 along the direction (nx, nz): F(q) . n for every
// variable (n need not be a unit vector).
template <typename R, int RAIN>
__device__ __forceinline__ void flux_dir(const Pt<R, 2, RAIN>& q, R nx, R nz, R* Fn) {
  using V = Vars<2, RAIN>;
  const R un = q.u[0] * nx + q.u[1] * nz;
  Fn[V::RD] = q.rd * un;
  Fn[V::RM] = q.rm * un;
  R f0 = q.m[0] * un + q.pp * nx, f1 = q.m[1] * un + q.pp * nz, fe = q.H * un;
  if (RAIN) {
    const R fall = q.rrvr * nz;
    Fn[V::RR] = q.rr * un - fall;
    f0 -= fall * q.u[0];
    f1 -= fall * q.u[1];
    fe -= q.rain_e * nz;
  }
  Fn[V::M0] = f0;
  Fn[V::M0 + 1] = f1;
  Fn[V::E] = fe;
}

// wave speed along the unit normal (Section 3.2): |u.n| + |v_r n_z| + c_m
template <typename R, int RAIN>
__device__ __forceinline__ R speed_dir(const Pt<R, 2, RAIN>& q, R nx, R nz) {
  R l = fabs(q.u[0] * nx + q.u[1] * nz) + q.cm;
  if (RAIN) l += fabs(q.vr * nz);
  return l;
}

// Split (Section 2.2) of the state with perturbation Uq (FP64) over background
// b at one point, from the guess Tg: T and rho_v = min(rho_vs(T), rho_m).
template <int RAIN>
__device__ __forceinline__ SplitOut tri_split_point(const KArgs& a, const double* Uq, const double* b, double Tg,
                                                    double* rv) {
  using V = Vars<2, RAIN>;
  const double rd = b[0] + Uq[V::RD];
  const double rm = b[1] + Uq[V::RM];
  const double rr = RAIN ? b[2] + Uq[V::RR] : 0.0;
  const double rho = rd + rm + rr;
  const double m0 = Uq[V::M0], m1 = Uq[V::M0 + 1];
  const double re = (b[3] + Uq[V::E]) - 0.5 * (m0 * m0 + m1 * m1) / rho;
  const SplitOut s = split_point(a, rd, rm, rr, re, Tg);
  *rv = fmin(s.rvs, rm);
  return s;
}

// Work layout: a block of 256 threads holds EPB elements, one thread per
// volume point of each (EPB NQ threads; the rest idle).  The elements'
// coefficients, their projected T and rho_v and the per-point results sit in
// LDS; the contractions between modes and points read them from there:
//   points:  thread (element, q) evaluates the state at volume point q, its
//            flux along the two columns of A^{-T} and its sources;
//   modes:   thread (element, m), m < NP, sums the volume point results and
//            the weighted face fluxes against psi_m, and forms the update;
//   faces:   thread (element, j), j < 3 NF, handles face point j: its own
//            trace from LDS, the neighbour's from global memory.
template <int K>
struct TriBlock {
  static constexpr int NQ = TriShape<K>::NQ;
  static constexpr int EPB = 256 / NQ;
  static constexpr int NT = EPB * NQ;
};

template <typename R, int K, int RAIN>
struct TriLds {
  static constexpr int NV = Vars<2, RAIN>::NV, NP = TriShape<K>::NP, NQ = TriShape<K>::NQ;
  static constexpr int NF = TriShape<K>::NF, EPB = TriBlock<K>::EPB;
  static constexpr bool HAS_AUX = true;
  // the reference tables (FP32; in FP64 they would halve the blocks per CU and
  // stay in constant memory)
  struct Empty {};
  std::conditional_t<sizeof(R) == 4, TriTab<R, K>, Empty> tab;
  double aux[EPB][2][NP];   // projected T and rho_v of the stage input
  double ts[EPB][NQ][2];    // the split of the updated state at the volume points
  R c[EPB][NV][NP];         // coefficients of the stage input, then of its update
  union {
    R pf[EPB][NQ][3 * NV];  // per volume point: w F.G0, w F.G1, w G
    struct {                // then the neighbours across the three faces
      double aux[EPB][3][2][NP];
      R c[EPB][3][NV][NP];
    } nb;
  } u;
  R ff[EPB][3 * NF][NV];    // per face point: the weighted normal flux
  TriZ fz[EPB];             // heights of the vertices and background layer
  R fn[EPB][3][3];          // per face: n_x, n_z, |e_f| / det A
};

// First element of this block.  Consecutive blocks go round-robin to the 8
// XCDs; XCD x takes the contiguous block range [x per, (x+1) per), so an
// element and its neighbours in the rows above and below share an L2.  The
// grid is 8 per blocks; a block past the end returns -1 (uniformly).
template <int K>
__device__ __forceinline__ long long tri_first_element(int ne) {
  constexpr int EPB = TriBlock<K>::EPB;
  const int nblocks = (ne + EPB - 1) / EPB;
  const int per = (nblocks + 7) >> 3;
  const int b = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  return b < nblocks ? (long long)b * EPB : -1;
}

// LDS of the split kernel: coefficients and the split values only
template <typename R, int K, int RAIN>
struct TriLdsSplit {
  static constexpr int NV = Vars<2, RAIN>::NV, NP = TriShape<K>::NP, NQ = TriShape<K>::NQ;
  static constexpr int EPB = TriBlock<K>::EPB;
  static constexpr bool HAS_AUX = false;
  struct Empty {};
  std::conditional_t<sizeof(R) == 4, TriTab<R, K>, Empty> tab;
  double ts[EPB][NQ][2];
  R c[EPB][NV][NP];
};

// Copy the reference tables (a plain struct) from constant memory into LDS
// (FP32 kernels), and the tables a kernel reads: the LDS copy or constant memory.
template <typename R, int K, typename L>
__device__ __forceinline__ void tri_copy_tab(L& S) {
  if constexpr (sizeof(R) == 4) {
    static_assert(sizeof(TriTab<R, K>) % 4 == 0, "tables are whole words");
    const unsigned* s = reinterpret_cast<const unsigned*>(&ttab<R, K>());
    unsigned* d = reinterpret_cast<unsigned*>(&S.tab);
    for (int i = threadIdx.x; i < (int)(sizeof(TriTab<R, K>) / 4); i += blockDim.x) d[i] = s[i];
  }
}

template <typename R, int K, typename L>
__device__ __forceinline__ const TriTab<R, K>& tri_tab(const L& S) {
  if constexpr (sizeof(R) == 4) return S.tab;
  else return ttab<R, K>();
}

// Load the block's coefficients (and aux) into LDS with coalesced reads;
// elements past the end repeat the last one (their results are never stored).
template <typename R, int K, int RAIN, typename L>
__device__ __forceinline__ void tri_load_block(L& S, const TriArgs& t, long long e0, const R* __restrict__ U,
                                               const double* __restrict__ aux) {
  constexpr int NV = Vars<2, RAIN>::NV, NP = TriShape<K>::NP, EPB = TriBlock<K>::EPB;
  const size_t N = (size_t)t.ne * NP;
  for (int idx = threadIdx.x; idx < NV * EPB * NP; idx += blockDim.x) {
    const int v = idx / (EPB * NP), r = idx - v * (EPB * NP);
    const int le = r / NP, m = r - le * NP;
    const long long e = min(e0 + le, (long long)t.ne - 1);
    S.c[le][v][m] = U[v * N + (size_t)e * NP + m];
  }
  if constexpr (L::HAS_AUX)
    for (int idx = threadIdx.x; idx < 2 * EPB * NP; idx += blockDim.x) {
      const int v = idx / (EPB * NP), r = idx - v * (EPB * NP);
      const int le = r / NP, m = r - le * NP;
      const long long e = min(e0 + le, (long long)t.ne - 1);
      S.aux[le][v][m] = aux[v * N + (size_t)e * NP + m];
    }
}

// The split of the block's state S.c at volume point q of element slot el
// (thread (el, q)), written to S.ts; Tguess (optional) from S.aux.
template <typename R, int K, int RAIN, typename L>
__device__ __forceinline__ void tri_split_at(const KArgs& a, const TriArgs& t, L& S, int el, int q, const TriZ& g,
                                             int* iters, int* bad) {
  constexpr int NV = Vars<2, RAIN>::NV, NP = TriShape<K>::NP;
  const auto& T = tri_tab<R, K>(S);
  double X[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < NP; ++m) s += (double)S.c[el][v][m] * T.psid[q][m];
    X[v] = s;
  }
  double Tg = 0.0;
  if constexpr (L::HAS_AUX) {
#pragma unroll
    for (int m = 0; m < NP; ++m) Tg += S.aux[el][0][m] * T.psid[q][m];
  }
  double b[5];
  tri_bg<R, K>(t, T, g.layer, g.z0 + g.dz1 * T.rq[q] + g.dz2 * T.sq[q], b);
  double rv;
  const SplitOut o = tri_split_point<RAIN>(a, X, b, Tg, &rv);
  S.ts[el][q][0] = o.T;
  S.ts[el][q][1] = rv;
  *iters = o.iters;
  *bad = o.bad;
}

// The L2 projections of the split values S.ts onto P^k, by thread (el, j),
// j < 2 NP (j < NP: T, else rho_v), stored to Tn / Rn.
template <typename R, int K, int RAIN, typename L>
__device__ __forceinline__ void tri_project_split(const L& S, int el, int j, long long e, bool act,
                                                  double* __restrict__ Tn, double* __restrict__ Rn) {
  constexpr int NP = TriShape<K>::NP, NQ = TriShape<K>::NQ;
  const auto& T = tri_tab<R, K>(S);
  if (j >= 2 * NP) return;
  const int c = j >= NP ? 1 : 0, m = j - c * NP;
  double s = 0.0;
#pragma unroll 4
  for (int qq = 0; qq < NQ; ++qq) s += T.wd[qq] * T.psid[qq][m] * S.ts[el][qq][c];
  if (act) (c ? Rn : Tn)[(size_t)e * NP + m] = s;
}

// Split kernel: (Tn, Rn) = the projected T and rho_v of U.
template <typename R, int K, int RAIN>
__global__ void __launch_bounds__(256) tri_split_kernel(KArgs a, TriArgs t, const R* __restrict__ U,
                                                        double* __restrict__ Tn, double* __restrict__ Rn) {
  constexpr int NQ = TriShape<K>::NQ, EPB = TriBlock<K>::EPB, NT = TriBlock<K>::NT;
  __shared__ TriLdsSplit<R, K, RAIN> S;
  const int tid = threadIdx.x;
  const bool lane = tid < NT;
  const int el = lane ? tid / NQ : 0, q = lane ? tid - el * NQ : 0;
  const long long e0 = tri_first_element<K>(t.ne);
  if (e0 < 0) return;
  const bool act = lane && e0 + el < t.ne;
  const long long e = min(e0 + el, (long long)t.ne - 1);
  tri_copy_tab<R, K>(S);
  tri_load_block<R, K, RAIN>(S, t, e0, U, nullptr);
  __syncthreads();
  int it = 0, bd = 0;
  if (lane) tri_split_at<R, K, RAIN>(a, t, S, el, q, tri_z(t, (int)e), &it, &bd);
  __syncthreads();
  if (lane) tri_project_split<R, K, RAIN>(S, el, q, e, act, Tn, Rn);
  record_stats(a, act ? it : 0, act ? bd : 0);
}

// Stage kernel.  MODE 0: out = dC/dt.  MODE 2: out = c0 U0 + c1 U + c2 dt dC/dt
// and the split of out into (Tn, Rn) for the next stage.  aux holds the
// projected T and rho_v of U: aux[0 .. N) and aux[N .. 2N), N = ne NP.
template <typename R, int K, int RAIN, int MODE>
__global__ void __launch_bounds__(256) tri_stage_kernel(KArgs a, TriArgs t, const R* __restrict__ U,
                                                        const double* __restrict__ aux, R* __restrict__ out,
                                                        const R* __restrict__ U0, double c0, double c1, double c2dt,
                                                        double* __restrict__ Tn, double* __restrict__ Rn) {
  using V = Vars<2, RAIN>;
  constexpr int NV = V::NV, NP = TriShape<K>::NP, NQ = TriShape<K>::NQ, NF = TriShape<K>::NF;
  constexpr int EPB = TriBlock<K>::EPB, NT = TriBlock<K>::NT;
  __shared__ TriLds<R, K, RAIN> S;
  const auto& T = tri_tab<R, K>(S);
  const int tid = threadIdx.x;
  const bool lane = tid < NT;
  const int el = lane ? tid / NQ : 0, q = lane ? tid - el * NQ : 0;
  const long long e0 = tri_first_element<K>(t.ne);
  if (e0 < 0) return;
  const bool act = lane && e0 + el < t.ne;
  const int e = (int)min(e0 + el, (long long)t.ne - 1);
  const size_t N = (size_t)t.ne * NP;

  // the neighbours' coefficients across the three faces of the block's
  // elements, read now (coalesced runs of NP values) and parked in LDS once
  // the volume phase has released its storage
  constexpr int NNC = (EPB * 3 * NV * NP + 255) / 256, NNA = (EPB * 3 * 2 * NP + 255) / 256;
  R nreg[NNC];
  double areg[NNA];
#pragma unroll
  for (int k = 0; k < NNC; ++k) {
    const int idx = tid + 256 * k;
    nreg[k] = R(0);
    if (idx < EPB * 3 * NV * NP) {
      const int m = idx % NP, r = idx / NP, v = r % NV, r2 = r / NV, f = r2 % 3, le = r2 / 3;
      const long long ee = min(e0 + le, (long long)t.ne - 1);
      const int nb = t.nbr[(size_t)ee * 3 + f];
      if (nb >= 0) nreg[k] = U[v * N + (size_t)(nb >> 2) * NP + m];
    }
  }
#pragma unroll
  for (int k = 0; k < NNA; ++k) {
    const int idx = tid + 256 * k;
    areg[k] = 0.0;
    if (idx < EPB * 3 * 2 * NP) {
      const int m = idx % NP, r = idx / NP, v = r % 2, r2 = r / 2, f = r2 % 3, le = r2 / 3;
      const long long ee = min(e0 + le, (long long)t.ne - 1);
      const int nb = t.nbr[(size_t)ee * 3 + f];
      if (nb >= 0) areg[k] = aux[v * N + (size_t)(nb >> 2) * NP + m];
    }
  }
  tri_copy_tab<R, K>(S);
  tri_load_block<R, K, RAIN>(S, t, e0, U, aux);

  // geometry: A = [V1 - V0, V2 - V0], G = A^{-T}
  const double* xv = t.xy + (size_t)e * 6;
  const TriZ g = tri_z(t, e);
  const double a00 = xv[2] - xv[0], a01 = xv[4] - xv[0], a10 = g.dz1, a11 = g.dz2;
  const double det = a00 * a11 - a01 * a10;
  const double idet = 1.0 / det;
  // the face geometry, for whichever threads take the element's face points
  if (lane && q < 3) {
    const double ex = q == 0 ? a00 : (q == 1 ? a01 - a00 : -a01);
    const double ez = q == 0 ? a10 : (q == 1 ? a11 - a10 : -a11);
    const double len = sqrt(ex * ex + ez * ez);
    S.fn[el][q][0] = (R)(ez / len);
    S.fn[el][q][1] = (R)(-ex / len);
    S.fn[el][q][2] = (R)(len * idet);
    if (q == 0) S.fz[el] = g;
  }
  __syncthreads();

  // volume point q: flux along the columns of A^{-T} and sources, weighted
  if (lane) {
    R Uq[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      R s = R(0);
#pragma unroll
      for (int m = 0; m < NP; ++m) s += S.c[el][v][m] * T.psi[q][m];
      Uq[v] = s;
    }
    double Tq = 0.0, Rq = 0.0;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      Tq += S.aux[el][0][m] * T.psid[q][m];
      Rq += S.aux[el][1][m] * T.psid[q][m];
    }
    double b[5];
    tri_bg<R, K>(t, T, g.layer, g.z0 + g.dz1 * T.rq[q] + g.dz2 * T.sq[q], b);
    Pt<R, 2, RAIN> p;
    eval_core<R, 2, RAIN>(a, Uq, Tq, Rq, RAIN ? rho_vs(a, Tq) : 0.0, b[0], b[1], b[2], b[3], b[4], p);
    const R wq = T.w[q];
    R Fr[NV], Fs[NV], Gs[NV];
    flux_dir<R, RAIN>(p, wq * (R)(a11 * idet), wq * (R)(-a01 * idet), Fr);
    flux_dir<R, RAIN>(p, wq * (R)(-a10 * idet), wq * (R)(a00 * idet), Fs);
#pragma unroll
    for (int v = 0; v < NV; ++v) Gs[v] = R(0);
    sources<R, 2, RAIN>(a, Uq, p, Gs);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      S.u.pf[el][q][v] = Fr[v];
      S.u.pf[el][q][NV + v] = Fs[v];
      S.u.pf[el][q][2 * NV + v] = wq * Gs[v];
    }
  }
  __syncthreads();

  // modes: (F, grad psi_m) + (G, psi_m) over the volume points.  NQ = 2 NP,
  // so thread (el, q) takes mode m = q mod NP for the variables v = par,
  // par + 2, ... with par = q / NP.
  static_assert(NQ == 2 * NP, "the Duffy rule has twice as many points as P^k has modes");
  constexpr int NH = (NV + 1) / 2;
  const int m = q % NP, par = q / NP;
  R acc[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) acc[h] = R(0);
  if (lane) {
#pragma unroll 2
    for (int qq = 0; qq < NQ; ++qq) {
      const R dr = T.dr[qq][m], ds = T.ds[qq][m], ps = T.psi[qq][m];
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int v = par + 2 * h;
        if (v < NV)
          acc[h] += S.u.pf[el][qq][v] * dr + S.u.pf[el][qq][NV + v] * ds + S.u.pf[el][qq][2 * NV + v] * ps;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NNC; ++k) {
    const int idx = tid + 256 * k;
    if (idx < EPB * 3 * NV * NP) (&S.u.nb.c[0][0][0][0])[idx] = nreg[k];
  }
#pragma unroll
  for (int k = 0; k < NNA; ++k) {
    const int idx = tid + 256 * k;
    if (idx < EPB * 3 * 2 * NP) (&S.u.nb.aux[0][0][0][0])[idx] = areg[k];
  }
  __syncthreads();

  // face point j = f NF + i of element slot fe: the Lax-Friedrichs flux
  // against the neighbour's trace (or the slip-wall ghost), weighted by
  // |e_f| / det A and w_i / 2.  The EPB 3 NF face tasks go to the block's
  // first threads, so whole wavefronts skip this phase instead of every
  // wavefront running it with idle lanes.
  static_assert(EPB * 3 * NF <= 256, "face tasks exceed the block");
  if (tid < EPB * 3 * NF) {
    const int fe = tid / (3 * NF), j = tid - fe * (3 * NF);
    const int f = j / NF, i = j - f * NF;
    const int ef = (int)min(e0 + fe, (long long)t.ne - 1);
    const TriZ gf = S.fz[fe];
    const R nx = S.fn[fe][f][0], nz = S.fn[fe][f][1];
    const int nb = t.nbr[(size_t)ef * 3 + f];
    const bool wall = nb < 0;
    const double z = gf.z0 + gf.dz1 * T.rf[f][i] + gf.dz2 * T.sf[f][i];
    R Um[NV], Up[NV], Fm[NV], Fp[NV], lm, lp;
    double Tm = 0.0, Rm = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      R s = R(0);
#pragma unroll
      for (int m = 0; m < NP; ++m) s += S.c[fe][v][m] * T.psif[f][i][m];
      Um[v] = s;
    }
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      Tm += S.aux[fe][0][m] * T.psifd[f][i][m];
      Rm += S.aux[fe][1][m] * T.psifd[f][i][m];
    }
    double b[5];
    tri_bg<R, K>(t, T, gf.layer, z, b);
    const double rvsm = RAIN ? rho_vs(a, Tm) : 0.0;
    {
      Pt<R, 2, RAIN> pm;
      eval_core<R, 2, RAIN>(a, Um, Tm, Rm, rvsm, b[0], b[1], b[2], b[3], b[4], pm);
      flux_dir<R, RAIN>(pm, nx, nz, Fm);
      lm = speed_dir<R, RAIN>(pm, nx, nz);
    }
    {
      Pt<R, 2, RAIN> pp;
      if (wall) {
        // slip wall: m+ = m- - 2 (m-.n) n, everything else copied
#pragma unroll
        for (int v = 0; v < NV; ++v) Up[v] = Um[v];
        const R mn = Um[V::M0] * nx + Um[V::M0 + 1] * nz;
        Up[V::M0] = Um[V::M0] - R(2) * mn * nx;
        Up[V::M0 + 1] = Um[V::M0 + 1] - R(2) * mn * nz;
        eval_core<R, 2, RAIN>(a, Up, Tm, Rm, rvsm, b[0], b[1], b[2], b[3], b[4], pp);
      } else {
        // the neighbour's trace at its face point K - i (the same physical point)
        const int e2 = nb >> 2, f2 = nb & 3, i2 = K - i;
        double Tp = 0.0, Rp = 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          R s = R(0);
#pragma unroll
          for (int m = 0; m < NP; ++m) s += S.u.nb.c[fe][f][v][m] * T.psif[f2][i2][m];
          Up[v] = s;
        }
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          Tp += S.u.nb.aux[fe][f][0][m] * T.psifd[f2][i2][m];
          Rp += S.u.nb.aux[fe][f][1][m] * T.psifd[f2][i2][m];
        }
        double b2[5];
        tri_bg<R, K>(t, T, tri_z(t, e2).layer, z, b2);
        eval_core<R, 2, RAIN>(a, Up, Tp, Rp, RAIN ? rho_vs(a, Tp) : 0.0, b2[0], b2[1], b2[2], b2[3], b2[4], pp);
      }
      flux_dir<R, RAIN>(pp, nx, nz, Fp);
      lp = speed_dir<R, RAIN>(pp, nx, nz);
    }
    const R L = lm >= lp ? lm : lp;
    const R wgt = S.fn[fe][f][2] * T.wf[i];
#pragma unroll
    for (int v = 0; v < NV; ++v)
      S.ff[fe][j][v] = wgt * (R(0.5) * (Fm[v] + Fp[v]) + R(0.5) * L * (Um[v] - Up[v]));
  }
  __syncthreads();

  // modes: minus the face integrals, then the update
  if (lane) {
#pragma unroll
    for (int j = 0; j < 3 * NF; ++j) {
      const R ps = T.psif[j / NF][j % NF][m];
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int v = par + 2 * h;
        if (v < NV) acc[h] -= S.ff[el][j][v] * ps;
      }
    }
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int v = par + 2 * h;
      if (v < NV) {
        R x = acc[h];
        if (MODE != 0) {
          x = (R)c1 * S.c[el][v][m] + (R)c2dt * acc[h];
          if (c0 != 0.0) x += (R)c0 * U0[v * N + (size_t)e * NP + m];
        }
        S.c[el][v][m] = x;
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < NV * EPB * NP; idx += blockDim.x) {
    const int v = idx / (EPB * NP), r = idx - v * (EPB * NP);
    const int le = r / NP, m = r - le * NP;
    if (e0 + le < t.ne) out[v * N + (size_t)(e0 + le) * NP + m] = S.c[le][v][m];
  }
  if constexpr (MODE == 2) {
    // the split of the updated state for the next stage (Section 3.4)
    int it = 0, bd = 0;
    if (lane) tri_split_at<R, K, RAIN>(a, t, S, el, q, g, &it, &bd);
    __syncthreads();
    if (lane) tri_project_split<R, K, RAIN>(S, el, q, e, act, Tn, Rn);
    record_stats(a, act ? it : 0, act ? bd : 0);
  }
}

// Projection onto P^k of fields given at the volume points: one thread per
// (field, element).
template <typename R, int K>
__global__ void __launch_bounds__(64) tri_project_kernel(TriArgs t, const double* __restrict__ vals, int nfields,
                                                         R* __restrict__ C) {
  constexpr int NP = TriShape<K>::NP, NQ = TriShape<K>::NQ;
  const auto& T = ttab<R, K>();
  const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= (long long)nfields * t.ne) return;
  double s[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) s[m] = 0.0;
#pragma unroll 1
  for (int q = 0; q < NQ; ++q) {
    const double wv = T.wd[q] * vals[b * NQ + q];
#pragma unroll
    for (int m = 0; m < NP; ++m) s[m] += wv * T.psid[q][m];
  }
#pragma unroll
  for (int m = 0; m < NP; ++m) C[b * NP + m] = (R)s[m];
}

// Background pressure at every layer height: the equation of state of the
// split background.
__global__ void tri_bg_pressure_kernel(KArgs a, double* bgl, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double* b = bgl + (size_t)i * 5;
  const double rd = b[0], rm = b[1], rr = a.rain ? b[2] : 0.0;
  const SplitOut s = split_point(a, rd, rm, rr, b[3], 0.0);
  const double rv = fmin(s.rvs, rm);
  b[4] = s.bad ? __builtin_nan("") : (rd * a.Rd + rv * a.Rv) * s.T;
}

}  // namespace dgm
