// Shared host/device definitions of libdgmoist: kernel argument blocks and the
// per-member mesh descriptors of a (possibly batched) handle.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgm {

constexpr int kMaxOrder = 7;     // 2D; 3D kernels are instantiated up to 4
constexpr int kMaxP1 = kMaxOrder + 1;

// One ensemble member: a structured box.  Elements of all members are
// concatenated; eoff is this member's first global element.
struct MemberDesc {
  int n[3];             // elements per axis (n[2] = 1 in 2D)
  int bc[3];            // 0 periodic, 1 slip wall
  double two_over_h[3]; // 2 / h_j
  double J;             // element Jacobian prod_j h_j / 2
  double face_J[3];     // face Jacobian for a face normal to axis j
  double lift[3][2];    // (2 / h_j) / w_0 and (2 / h_j) / w_K: face-to-node lifting
  long long eoff;       // first global element
  int ne;               // elements of this member
  int hoff;             // first background index (n_z (k+1) entries)
  // artificial diffusion: gamma 0.5 h^(1-d/2), the penalty sigma k^2 / h_j,
  // the vertices per axis and the first vertex of this member
  double sip_pre;
  double sip_tau[3];
  int nvx[3];
  long long voff;
};

// A work item: EPB consecutive elements of one member, starting at element e0
// with element coordinates (c0, c1, c2) packed as c12 = c1 + (c2 << 16).
struct Item {
  int member;
  int e0;
  int c0;
  int c12;
};

// Everything the kernels need besides the state arrays.
struct KArgs {
  // thermodynamics (Section 2; appendix table)
  double g, cvd, cvv, cl, Rd, Rv, Tref;
  double Lp;                       // L_ref - R_v T_ref
  double am1, b, inv_Tref, C0;     // rho_vs(T) = C0 exp(am1 ln(T/T_ref) + b (1/T_ref - 1/T))
  double vr_const, vr_pref, q_au;  // terminal speed, COSMO prefactor, autoconversion threshold
  int rain, vr_mode;
  double rtol;
  int maxit;
  // nodal tables of the basis (Lobatto, or Gauss for basis 1):
  // Dhat[i*(k+1)+a] = w_a D_ai / w_i, weights w
  double Dhat[kMaxP1 * kMaxP1];
  double w[kMaxP1];
  // basis 1 (Gauss nodes): traces l_i(-1), l_i(+1) of the Lagrange basis and
  // the lifting weights l_i(-+1) / w_i
  int basis;
  double gl_m[kMaxP1], gl_p[kMaxP1];
  double lift_m[kMaxP1], lift_p[kMaxP1];
  // basis 1: background traces on the horizontal faces, bgf[f * bgf_n + 2 r + s]
  // for field f = (rho_d, rho_m, rho_r, E, p), element row r of the
  // concatenated columns (hoff / (k+1) + ez) and side s (0 bottom, 1 top)
  const double* bgf;
  int bgf_n;
  // basis 1: face traces of the stage state (read) and of the new state
  // (written by MODE 2): U' at tr_u[(v * etot + e) * NFE + f], T and rho_v at
  // tr_a[(c * etot + e) * NFE + f] for face point f of element e
  const void* tr_u_in;
  const double* tr_a_in;
  void* tr_u_out;
  double* tr_a_out;
  // artificial diffusion (Lobatto basis): collocation derivative matrix
  // Dm[a*(k+1)+i] = l_i'(x_a), Lobatto nodes, per-element viscosity aK[2][e],
  // vertex means av[2][vertex] and the diffusive tendency (state layout)
  double Dm[kMaxP1 * kMaxP1];
  double xn[kMaxP1];
  double* sip_aK;
  double* sip_av;
  void* sip_out;
  long long nvert;
  // members and work items (member, first element) of EPB elements each
  const MemberDesc* mem;
  const Item* items;
  int nitems;
  int nmembers;
  long long etot;                  // elements of all members
  unsigned nnodes;                 // nodes of all members: the stride between variables
  // background per vertical node index, concatenated over members
  const double* bg_rd;
  const double* bg_rm;
  const double* bg_rr;
  const double* bg_E;
  const double* bg_p;
  // sponge blending factor per vertical node index (nullptr: no sponge)
  const double* sponge;
  // status words: [0] max iterations, [1] non-converged, [2] invalid, [3] spare,
  // [4..5] split count (64-bit)
  unsigned* stats;
  // stage kernels: walk the work items from the last one (every other stage,
  // so a stage starts on the data the previous one wrote last)
  int walk_rev;
};

}  // namespace dgm
