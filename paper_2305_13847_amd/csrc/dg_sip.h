// Artificial diffusion (Section 3.5) on the Lobatto basis: the symmetric
// interior penalty form on interior faces, acting on the perturbation
// unknowns, with the element-wise viscosity
//   alpha_K = gamma 0.5 h^(1-d/2) ||u||_{0,K}   (||u - v_r e_z||_{0,K} for rho_r)
// carried to a continuous Q1 field by the mean over the elements that share
// each vertex.  Three kernels per right-hand side:
//   1. sip_alpha_kernel: alpha_K of every element (two fields), an LDS
//      reduction over the element's nodes (the Q3 stage kernel forms the same
//      values for the state it writes, and then this launch is skipped);
//   2. sip_vertex_kernel: the vertex means (all members in one launch);
//   3. sip_kernel: the tendency S = -M^{-1} A_h(U, .) at every node, written
//      in the state layout; the stage kernels add it to the right-hand side.
// With nodes at the Lobatto points, S at node i reads (d_j = 2/h_j, D the
// collocation derivative matrix, Dhat its weak form, G_j = d_j D U along the
// j-line, alpha continuous):
//   S_i = - sum_j d_j sum_a Dhat[i_j][a] (alpha G_j)_a
//         + sum_j sum_{sides s} d_j / w_{i_j} alpha_f ( d_j/2 D[f_j][i_j] [U]_f
//                                  + [i_j = f_j] s ({G_j}_f - tau_j [U]_f) )
// where f is the face node of i's j-line on side s (s = -1 at xi_j = -1,
// +1 at xi_j = +1), [U] = U(lower element) - U(upper element) across the
// face, {G_j} the mean of both sides' gradients, tau_j = sigma k^2 / h_j.
// Faces on slip walls contribute nothing.
#pragma once
#include "dg_kernels.h"

namespace dgm {

template <typename R, int K, int D, int RAIN>
__global__ void __launch_bounds__(256)
sip_alpha_kernel(KArgs a, const R* __restrict__ U) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NP = S::NP, NT = S::NT;
  __shared__ double sm[2][NT];
  // one work item per block (no item loop: loop-invariant values would stay
  // live across the body)
  const int it_ = ItemWalk(a.nitems).item(0);
  if (it_ < 0) return;
  const int t = threadIdx.x;
  const Item item = a.items[it_];
  const MemberDesc& md = a.mem[item.member];
  const int le = t / NP, n = t - le * NP;
  const int e = item.e0 + le;
  double s0 = 0.0, s1 = 0.0;
  if (e < md.ne) {
    const unsigned N = a.nnodes;
    const unsigned g = (unsigned)(md.eoff + e) * NP + n;
    const ElemCoord<D> ec = item_coord<D>(md, item, le);
    const int idx[3] = {n % P1, (n / P1) % P1, D == 3 ? n / (P1 * P1) : 0};
    const int iz = md.hoff + ec.c[D - 1] * P1 + idx[D - 1];
    const double rd = a.bg_rd[iz] + (double)ld(U, N, V::RD, g);
    const double rm = a.bg_rm[iz] + (double)ld(U, N, V::RM, g);
    const double rr = RAIN ? a.bg_rr[iz] + (double)ld(U, N, V::RR, g) : 0.0;
    double w = md.J;
#pragma unroll
    for (int j = 0; j < D; ++j) w *= a.w[idx[j]];
    double m[D];
#pragma unroll
    for (int i = 0; i < D; ++i) m[i] = (double)ld(U, N, V::M0 + i, g);
    sip_alpha_terms<D, RAIN>(a, w, rd, rm, rr, m, s0, s1);
  }
  sm[0][t] = s0;
  sm[1][t] = s1;
  __syncthreads();
  // fixed-order tree over the element's nodes
  for (int h = 1; h < NP; h <<= 1) {
    if ((n % (2 * h)) == 0 && n + h < NP) {
      sm[0][t] += sm[0][t + h];
      sm[1][t] += sm[1][t + h];
    }
    __syncthreads();
  }
  if (n == 0 && e < md.ne) {
    a.sip_aK[md.eoff + e] = md.sip_pre * sqrt(sm[0][t]);
    a.sip_aK[a.etot + md.eoff + e] = md.sip_pre * sqrt(sm[1][t]);
  }
}

// one thread per vertex of every member (one launch for an ensemble): the
// mean of alpha_K over the elements that share it (a periodic axis wraps, a
// walled one has n + 1 vertices); the member is found by bisection over the
// members' first vertices
template <int D>
__global__ void sip_vertex_kernel(KArgs a) {
  const long long gi = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= a.nvert) return;
  int lo = 0, hi = a.nmembers - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.mem[mid].voff <= gi) lo = mid;
    else hi = mid - 1;
  }
  const MemberDesc& md = a.mem[lo];
  const long long i = gi - md.voff;
  int v[3] = {(int)(i % md.nvx[0]), (int)((i / md.nvx[0]) % md.nvx[1]), (int)(i / ((long long)md.nvx[0] * md.nvx[1]))};
  double s0 = 0.0, s1 = 0.0;
  int cnt = 0;
  for (int corner = 0; corner < (1 << D); ++corner) {
    int c[3] = {0, 0, 0};
    bool ok = true;
    for (int ax = 0; ax < D; ++ax) {
      int ca = v[ax] - ((corner >> ax) & 1);
      if (md.bc[ax] == 0) {
        if (ca < 0) ca += md.n[ax];
      } else if (ca < 0 || ca >= md.n[ax]) {
        ok = false;
      }
      c[ax] = ca;
    }
    if (!ok) continue;
    const long long e = c[0] + (long long)md.n[0] * (c[1] + (long long)md.n[1] * c[2]);
    s0 += a.sip_aK[md.eoff + e];
    s1 += a.sip_aK[a.etot + md.eoff + e];
    ++cnt;
  }
  a.sip_av[md.voff + i] = s0 / cnt;
  a.sip_av[a.nvert + md.voff + i] = s1 / cnt;
}

template <typename R, int K, int D, int RAIN>
__global__ void __launch_bounds__(256)
sip_kernel(KArgs a, const R* __restrict__ U) {
  using S = Shape<K, D, block_threads<R>()>;
  using V = Vars<D, RAIN>;
  constexpr int P1 = S::P1, NP = S::NP, NV = V::NV, NT = S::NT;
  constexpr int NF = (D == 2) ? P1 : P1 * P1;          // nodes of one face
  constexpr int NFBJ = S::EPB * 2 * NF;                 // face points of one direction in a block
  __shared__ R sU[NV * NT];
  __shared__ R sG[NV * NT];                  // one direction's gradients
  __shared__ R sA[2 * NT];
  __shared__ R sJ[NV * NFBJ];                // one direction's jumps [U]
  __shared__ R sM[NV * NFBJ];                // and mean gradients {G_j}
  __shared__ R sDm[P1 * P1];
  __shared__ R sDh[P1 * P1];
  __shared__ double sV[2][S::EPB][1 << D];   // the viscosity at each element's corners
  const int t = threadIdx.x;
  if (t < P1 * P1) {
    sDm[t] = (R)a.Dm[t];
    sDh[t] = (R)a.Dhat[t];
  }
  R* out = (R*)a.sip_out;
  const int epb = (int)blockDim.x / NP;
  // one work item per block (no item loop: loop-invariant values would stay
  // live across the body)
  const int it_ = ItemWalk(a.nitems).item(0);
  if (it_ < 0) return;
  const Item item = a.items[it_];
  const MemberDesc& md = a.mem[item.member];
  const unsigned N = a.nnodes;
  const int le = t / NP, n = t - le * NP;
  const int e = item.e0 + le;
  const bool active = e < md.ne;
  const unsigned g = (unsigned)(md.eoff + (active ? e : 0)) * NP + n;
  const ElemCoord<D> ec = item_coord<D>(md, item, active ? le : 0);
  const int idx[3] = {n % P1, (n / P1) % P1, D == 3 ? n / (P1 * P1) : 0};
  // A. the state, and the viscosity at the element's corners (vertex means)
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) sU[v * NT + t] = ld(U, N, v, g);
    if (n < (1 << D)) {
      long long vid = 0, stride = 1;
#pragma unroll
      for (int ax = 0; ax < D; ++ax) {
        int va = ec.c[ax] + ((n >> ax) & 1);
        if (md.bc[ax] == 0 && va == md.n[ax]) va = 0;
        vid += va * stride;
        stride *= md.nvx[ax];
      }
      sV[0][le][n] = a.sip_av[md.voff + vid];
      sV[1][le][n] = a.sip_av[a.nvert + md.voff + vid];
    }
  } else {
#pragma unroll
    for (int v = 0; v < NV; ++v) sU[v * NT + t] = R(0);
  }
  __syncthreads();
  // the Q1 viscosity at the node
  {
    double a0 = 0.0, a1 = 0.0;
    if (active) {
#pragma unroll
      for (int corner = 0; corner < (1 << D); ++corner) {
        double wq = 1.0;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
          const double xi = a.xn[idx[ax]];
          wq *= ((corner >> ax) & 1) ? 0.5 * (1.0 + xi) : 0.5 * (1.0 - xi);
        }
        a0 += wq * sV[0][le][corner];
        a1 += wq * sV[1][le][corner];
      }
    }
    sA[t] = (R)a0;
    sA[NT + t] = (R)a1;
  }
  // B-D, one direction j at a time (the tiles hold one direction's
  // gradients and face values, so a block needs a third of the LDS):
  //   B. the gradient G_j of every variable at every node;
  //   C. face points of the j-faces: [U] and {G_j}; the own side's gradient
  //      from the state tile, the neighbour's from its normal line in HBM;
  //   D. the volume and face terms of direction j at every node, added to
  //      the tendency in the order j, volume, minus face, plus face.
  R Sv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Sv[v] = R(0);
  constexpr int NFJ = 2 * NF;              // face points of one element's two j-faces
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const int str = j == 0 ? 1 : (j == 1 ? P1 : P1 * P1);
    const R dj = (R)md.two_over_h[j];
    if (j > 0) __syncthreads();            // the previous direction's tiles are read
    // B.
    {
      const int base = t - idx[j] * str;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        R acc = R(0);
#pragma unroll
        for (int b = 0; b < P1; ++b) acc += sDm[idx[j] * P1 + b] * sU[v * NT + base + b * str];
        sG[v * NT + t] = dj * acc;
      }
    }
    // C.  A face point's variables are split over two threads (the first
    // half and the rest), so the block's 2 EPB NF face points occupy every
    // thread (each reads k+1 neighbour values per variable).
    constexpr int VH = (NV + 1) / 2;
    for (int tv = t; tv < 2 * epb * NFJ; tv += (int)blockDim.x) {
      const int half = tv >= epb * NFJ;
      const int task = tv - half * epb * NFJ;
      const int fle = task / NFJ;
      const int r = task - fle * NFJ;
      const int side = r / NF;
      const int fp = r - side * NF;
      const int fe = item.e0 + fle;
      bool live = fe < md.ne;
      int en = 0;
      if (live) {
        const ElemCoord<D> fc = item_coord<D>(md, item, fle);
        const int c = j == 0 ? fc.c[0] : (j == 1 ? fc.c[1] : fc.c[D - 1]);
        const bool at_end = side ? (c == md.n[j] - 1) : (c == 0);
        live = !(at_end && md.bc[j] == 1);
        int cn = side ? c + 1 : c - 1;
        if (cn < 0) cn += md.n[j];
        if (cn >= md.n[j]) cn -= md.n[j];
        en = fe + (cn - c) * elem_stride(md, j);
      }
      // node of the line through face point fp at position 0 along j
      // (fp enumerates the other axes, the lower one fastest)
      int nf0;
      if (D == 2) {
        nf0 = (j == 0) ? fp * P1 : fp;
      } else {
        const int u = fp % P1, w2 = fp / P1;
        nf0 = (j == 0) ? P1 * (u + P1 * w2) : (j == 1 ? u + P1 * P1 * w2 : u + P1 * w2);
      }
      const int fo = side ? K : 0;                              // the own face node, along j
      const int l0 = fle * NP + nf0;                            // the own line (LDS index)
      const int fnb = side ? 0 : K;                             // the neighbour's, along j
      const unsigned gn0 = (unsigned)(md.eoff + en) * NP + nf0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if ((v < VH) == (half != 0)) continue;
        R ju = R(0), mg = R(0);
        if (live) {
          R gnb = R(0), unb = R(0), gow = R(0);
#pragma unroll
          for (int b = 0; b < P1; ++b) {
            const R ub = ld(U, N, v, gn0 + b * str);
            gnb += sDm[fnb * P1 + b] * ub;
            if (b == fnb) unb = ub;
            gow += sDm[fo * P1 + b] * sU[v * NT + l0 + b * str];
          }
          gnb *= dj;
          gow *= dj;
          const R uo = sU[v * NT + l0 + fo * str];
          ju = side ? uo - unb : unb - uo;
          mg = R(0.5) * (gow + gnb);
        }
        sJ[v * NFBJ + task] = ju;
        sM[v * NFBJ + task] = mg;
      }
    }
    __syncthreads();
    // D.  The line coefficients d_j Dhat[i_j][a] alpha_a and the face
    // coefficients depend on the viscosity field, not on the variable: they
    // are formed once, then each variable reads only its gradients and face
    // values.
    if (active) {
      constexpr int NA = RAIN ? 2 : 1;     // viscosity fields in use
      R cw[NA][P1];                        // volume: d_j Dhat[i_j][a] alpha(line node a)
      R cl[NA][2];                         // faces: d_j / w_{i_j} alpha_f, per side
      R cd[2];                             // d_j / 2 D[f_j][i_j]
      const int base = t - idx[j] * str;
      const R kw = dj / (R)a.w[idx[j]];
      const R ct = (R)md.sip_tau[j];
#pragma unroll
      for (int b = 0; b < P1; ++b) {
        const R db = dj * sDh[idx[j] * P1 + b];
#pragma unroll
        for (int f = 0; f < NA; ++f) cw[f][b] = db * sA[f * NT + base + b * str];
      }
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int fj = side ? K : 0;
        cd[side] = R(0.5) * dj * sDm[fj * P1 + idx[j]];
#pragma unroll
        for (int f = 0; f < NA; ++f) cl[f][side] = kw * sA[f * NT + base + fj * str];
      }
      int fpj;
      if (D == 2) fpj = (j == 0) ? idx[1] : idx[0];
      else fpj = (j == 0) ? idx[1] + P1 * idx[2] : (j == 1 ? idx[0] + P1 * idx[2] : idx[0] + P1 * idx[1]);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const bool rr = RAIN && v == V::RR;
        // volume
        R acc = R(0);
#pragma unroll
        for (int b = 0; b < P1; ++b) acc += (rr ? cw[NA - 1][b] : cw[0][b]) * sG[v * NT + base + b * str];
        R sv = Sv[v] - acc;
        // faces: this node's line meets the minus face (side 0) and the plus face (side 1)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          const int fj = side ? K : 0;
          const int task = le * NFJ + side * NF + fpj;
          const R ju = sJ[v * NFBJ + task];
          R term = cd[side] * ju;
          if (idx[j] == fj) term += (side ? R(1) : R(-1)) * (sM[v * NFBJ + task] - ct * ju);
          sv += (rr ? cl[NA - 1][side] : cl[0][side]) * term;
        }
        Sv[v] = sv;
      }
    }
  }
  if (active) {
#pragma unroll
    for (int v = 0; v < NV; ++v) st(out, N, v, g, Sv[v]);
  }
}

}  // namespace dgm
