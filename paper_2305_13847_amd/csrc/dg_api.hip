// Host side of libdgmoist: the C interface declared in include/dg.h.
//
// Validation, Lobatto tables, member/work-item tables, device buffers and the
// sequencing of kernels on the caller's stream.  Every step of the method runs
// in the kernels of dg_kernels.h / dg_vjp.h; the host only prepares tables and
// enqueues work.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>
#include <tuple>

#include "dg.h"
#include "dg_launch.h"

using namespace dgm;

namespace dgm {
extern template struct Launch<double>;
extern template struct Launch<float>;
}

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static dg_status fail(dg_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(DG_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

extern "C" const char* dg_last_error(void) { return g_err.c_str(); }

namespace dgm {
// error reporting and the thermodynamic part of the kernel arguments, shared
// with the triangle interface
dg_status api_fail(dg_status s, const char* msg) {
  g_err = msg;
  return s;
}

void fill_thermo(KArgs& a, const dg_params* p) {
  a.g = p->g; a.cvd = p->cvd; a.cvv = p->cvv; a.cl = p->cl; a.Rd = p->Rd; a.Rv = p->Rv;
  a.Tref = p->Tref;
  a.Lp = p->Lref - p->Rv * p->Tref;
  const double aa = (p->cpv - p->cl) / p->Rv;
  a.am1 = aa - 1.0;
  a.b = (p->Lref - (p->cpv - p->cl) * p->Tref) / p->Rv;
  a.inv_Tref = 1.0 / p->Tref;
  a.C0 = p->eref / (p->Rv * p->Tref);
  a.vr_const = p->vr_const;
  a.vr_pref = std::pow(M_PI * p->rho_w * p->N0r, -0.125) * p->v0r * std::tgamma(4.5) / 6.0;
  a.q_au = p->q_au;
  a.rain = p->rain; a.vr_mode = p->vr_mode;
  a.rtol = p->newton_rtol; a.maxit = p->newton_maxit;
}
}  // namespace dgm

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct dg_handle {
  int dim = 0, order = 0, nvars = 0, rain = 0, prec = 0, rk = 0, nmembers = 0;
  dg_params P{};
  std::vector<MemberDesc> mem;
  std::vector<Item> items;
  std::vector<int> item_off;     // first item of each member (+ total)
  std::vector<int> hoff;         // first background index of each member (+ total)
  std::vector<char> bg_set;
  long long etot = 0, nnodes = 0;
  int np = 0;
  size_t state_bytes = 0;
  // device
  MemberDesc* mem_d = nullptr;
  Item* items_d = nullptr;
  double* bg_d[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // rd, rm, rr, E, p
  void* stage[2] = {nullptr, nullptr};
  void* stage_x[4] = {nullptr, nullptr, nullptr, nullptr};          // adjoint workspace
  void* stage_w = nullptr;       // adjoint of the step's end state through the sponge
  double* sponge_d = nullptr;    // sponge blending factor per vertical node index
  double* bgf_d = nullptr;       // Gauss basis: background traces on horizontal faces
  void* tr_u[2] = {nullptr, nullptr};     // Gauss basis: face traces of U' (ping-pong like aux)
  double* tr_a[2] = {nullptr, nullptr};   // and of T, rho_v
  bool sip = false;              // artificial diffusion on
  double* sip_aK = nullptr;      // per-element viscosity, two fields
  double* sip_av = nullptr;      // vertex means, two fields
  void* sip_out = nullptr;       // diffusive tendency (state layout)
  std::vector<long long> nvert;  // vertices of each member
  bool sponge = false;
  double* auxT = nullptr;
  double* auxS = nullptr;
  double* auxT2 = nullptr;
  double* auxS2 = nullptr;
  double* auxT3 = nullptr;        // adjoint: splits of the recomputed stages
  double* auxS3 = nullptr;
  double* auxT4 = nullptr;
  double* auxS4 = nullptr;
  double* dt_d = nullptr;
  double* dt_h = nullptr;        // pinned staging for dt
  double* partial = nullptr;
  double* red_out = nullptr;
  unsigned* stats = nullptr;
  long long splits = 0;          // node splits enqueued since the last reset
  KArgs ka{};
  KArgs* ka_d = nullptr;         // device copy of ka (read by the persistent kernels)
  // launch geometry
  int epb = 1;                   // elements per block
  int persist = 0;               // persistent blocks per CU (0: one block per item)
  int item_order = 2;            // order of the work items (build_items); 2 measured fastest on Q3 3D
  int ncu = 256;
  long long items_cap = 0;       // device capacity of the item table
  // captured multi-step graph
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  const void* graph_U = nullptr;
  int graph_nsteps = -1, graph_epb = -1, graph_persist = -1;
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev;        // pairs (start, stop)
  std::vector<int> ev_class;         // class of each pending pair
  int ev_used = 0;
  double t_ms[4] = {0, 0, 0, 0};
  long long t_n[4] = {0, 0, 0, 0};
};

static const int kEvPairs = 2048;

static void timing_flush(dg_handle* h) {
  if (!h->timing || h->ev_used == 0) return;
  for (int i = 0; i < h->ev_used; ++i) {
    (void)hipEventSynchronize(h->ev[2 * i + 1]);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]) == hipSuccess) {
      h->t_ms[h->ev_class[i]] += ms;
      h->t_n[h->ev_class[i]] += 1;
    }
  }
  h->ev_used = 0;
}

// RAII bracket of one kernel launch with timing events
struct KTimer {
  dg_handle* h;
  int slot = -1;
  hipStream_t s;
  KTimer(dg_handle* hh, int cls, hipStream_t ss) : h(hh), s(ss) {
    if (!h->timing) return;
    if (h->ev_used == kEvPairs) timing_flush(h);
    slot = h->ev_used++;
    h->ev_class[slot] = cls;
    (void)hipEventRecord(h->ev[2 * slot], s);
  }
  ~KTimer() {
    if (slot >= 0) (void)hipEventRecord(h->ev[2 * slot + 1], s);
  }
};

extern "C" void dg_default_params(dg_params* p) {
  std::memset(p, 0, sizeof *p);
  // thermodynamic table of the paper's appendix; g is the usual 9.81
  p->cl = 4218.0; p->cpd = 1005.0; p->cpv = 1850.0; p->cvd = 718.0; p->cvv = 1390.0;
  p->eref = 610.7; p->Lref = 2.835e6; p->Rd = 287.05; p->Rv = 461.51; p->Tref = 273.15;
  p->pref = 1.0e5; p->g = 9.81;
  p->rain = 0; p->vr_mode = DG_VR_CONST; p->vr_const = 5.0;
  // COSMO warm-rain parameters (Section 2.1)
  p->rho_w = 1000.0; p->N0r = 8.0e6; p->v0r = 130.0; p->q_au = 0.0;
  p->precision = DG_FP64; p->rk = DG_SSPRK43;
  p->newton_rtol = 1e-14; p->newton_maxit = 30;
  p->basis = DG_BASIS_LOBATTO;
  p->sip_gamma = 0.0; p->sip_sigma = 10.0;
}

// Lobatto nodes in closed form (k <= 4), weights 2 / (k (k+1) P_k(x)^2) and the
// classical Legendre form of the collocation derivative matrix.
static double legendre_P(int k, double x) {
  double p0 = 1.0, p1 = x;
  if (k == 0) return 1.0;
  for (int m = 1; m < k; ++m) {
    double p2 = ((2 * m + 1) * x * p1 - m * p0) / (m + 1);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// P_n and P_n' at x (three-term recurrence; P_n' from (1 - x^2) P_n' = n (P_{n-1} - x P_n))
static void legendre_pd(int n, double x, double* P, double* dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int m = 1; m < n; ++m) {
    const double p2 = ((2 * m + 1) * x * p1 - m * p0) / (m + 1);
    p0 = p1;
    p1 = p2;
  }
  *P = p1;
  *dP = n * (p0 - x * p1) / (1.0 - x * x);
}

// Lobatto nodes: closed forms for k <= 4; above, the roots of P_k' by Newton
// (with P_k'' from Legendre's equation) from the Chebyshev-Lobatto points
static void lobatto_nodes(int k, double* x) {
  switch (k) {
    case 1: x[0] = -1; x[1] = 1; return;
    case 2: x[0] = -1; x[1] = 0; x[2] = 1; return;
    case 3: x[0] = -1; x[1] = -1 / std::sqrt(5.0); x[2] = -x[1]; x[3] = 1; return;
    case 4: x[0] = -1; x[1] = -std::sqrt(3.0 / 7.0); x[2] = 0; x[3] = -x[1]; x[4] = 1; return;
    default: break;
  }
  x[0] = -1.0;
  x[k] = 1.0;
  for (int i = 1; i < k; ++i) {
    double t = -std::cos(M_PI * i / k);
    for (int it = 0; it < 60; ++it) {
      double P, dP;
      legendre_pd(k, t, &P, &dP);
      const double d2P = (2.0 * t * dP - k * (k + 1.0) * P) / (1.0 - t * t);
      const double step = dP / d2P;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[i] = t;
  }
}

static void lobatto_tables(int k, double* w, double* Dhat, double* Dout = nullptr) {
  double x[kMaxP1];
  lobatto_nodes(k, x);
  const int p1 = k + 1;
  double P[kMaxP1];
  for (int i = 0; i < p1; ++i) {
    P[i] = legendre_P(k, x[i]);
    w[i] = 2.0 / (k * (k + 1.0) * P[i] * P[i]);
  }
  double Dm[kMaxP1][kMaxP1];   // Dm[a][i] = l_i'(x_a)
  for (int a = 0; a < p1; ++a)
    for (int i = 0; i < p1; ++i) {
      if (a != i) Dm[a][i] = P[a] / (P[i] * (x[a] - x[i]));
      else if (a == 0) Dm[a][i] = -k * (k + 1.0) / 4.0;
      else if (a == k) Dm[a][i] = k * (k + 1.0) / 4.0;
      else Dm[a][i] = 0.0;
    }
  for (int i = 0; i < p1; ++i)
    for (int a = 0; a < p1; ++a) Dhat[i * p1 + a] = w[a] * Dm[a][i] / w[i];
  if (Dout)
    for (int a = 0; a < p1; ++a)
      for (int i = 0; i < p1; ++i) Dout[a * p1 + i] = Dm[a][i];
}

// Gauss-Legendre nodes and weights of the (k+1)-point rule in closed form
// (k <= 4), the collocation derivative matrix on them from barycentric
// weights, the weak-form matrix Dhat[i][a] = w_a D_ai / w_i, and the values of
// the Lagrange basis at the element ends, l_i(-1) and l_i(+1).
static void gauss_tables(int k, double* x, double* w, double* Dhat, double* lm, double* lp) {
  const int p1 = k + 1;
  if (k > 4) {
    // the roots of P_{k+1} by Newton from the cosine guesses; w = 2 / ((1 - x^2) P'^2)
    for (int i = 0; i < p1; ++i) {
      double t = -std::cos(M_PI * (i + 0.75) / (p1 + 0.5));
      for (int it = 0; it < 60; ++it) {
        double P, dP;
        legendre_pd(p1, t, &P, &dP);
        const double step = P / dP;
        t -= step;
        if (std::fabs(step) < 1e-16) break;
      }
      double P, dP;
      legendre_pd(p1, t, &P, &dP);
      x[i] = t;
      w[i] = 2.0 / ((1.0 - t * t) * dP * dP);
    }
  } else switch (k) {
    case 1: x[1] = 1.0 / std::sqrt(3.0); w[0] = w[1] = 1.0; break;
    case 2: x[2] = std::sqrt(0.6); x[1] = 0.0; w[1] = 8.0 / 9.0; w[0] = w[2] = 5.0 / 9.0; break;
    case 3: {
      const double r = 2.0 / 7.0 * std::sqrt(6.0 / 5.0);
      x[2] = std::sqrt(3.0 / 7.0 - r); x[3] = std::sqrt(3.0 / 7.0 + r);
      w[1] = w[2] = (18.0 + std::sqrt(30.0)) / 36.0;
      w[0] = w[3] = (18.0 - std::sqrt(30.0)) / 36.0;
      break;
    }
    default: {
      const double r = 2.0 * std::sqrt(10.0 / 7.0);
      x[2] = 0.0; x[3] = std::sqrt(5.0 - r) / 3.0; x[4] = std::sqrt(5.0 + r) / 3.0;
      w[2] = 128.0 / 225.0;
      w[1] = w[3] = (322.0 + 13.0 * std::sqrt(70.0)) / 900.0;
      w[0] = w[4] = (322.0 - 13.0 * std::sqrt(70.0)) / 900.0;
      break;
    }
  }
  if (k <= 4)
    for (int i = 0; i < p1 / 2; ++i) x[i] = -x[k - i];
  double lam[kMaxP1];
  for (int i = 0; i < p1; ++i) {
    lam[i] = 1.0;
    for (int m = 0; m < p1; ++m)
      if (m != i) lam[i] /= (x[i] - x[m]);
  }
  double Dm[kMaxP1][kMaxP1];   // Dm[a][i] = l_i'(x_a)
  for (int a = 0; a < p1; ++a) {
    double diag = 0.0;
    for (int i = 0; i < p1; ++i) {
      if (i == a) continue;
      Dm[a][i] = lam[i] / lam[a] / (x[a] - x[i]);
      diag += 1.0 / (x[a] - x[i]);
    }
    Dm[a][a] = diag;
  }
  for (int i = 0; i < p1; ++i)
    for (int a = 0; a < p1; ++a) Dhat[i * p1 + a] = w[a] * Dm[a][i] / w[i];
  for (int i = 0; i < p1; ++i) {
    double vm = 1.0, vp = 1.0;
    for (int m = 0; m < p1; ++m)
      if (m != i) {
        vm *= (-1.0 - x[m]) / (x[i] - x[m]);
        vp *= (1.0 - x[m]) / (x[i] - x[m]);
      }
    lm[i] = vm;
    lp[i] = vp;
  }
}

static void free_all(dg_handle* h) {
  auto F = [](void* p) { if (p) (void)hipFree(p); };
  F(h->mem_d); F(h->items_d); F(h->ka_d);
  for (auto& b : h->bg_d) F(b);
  for (auto& b : h->stage) F(b);
  for (auto& b : h->stage_x) F(b);
  F(h->stage_w); F(h->sponge_d); F(h->bgf_d);
  F(h->sip_aK); F(h->sip_av); F(h->sip_out);
  for (int i = 0; i < 2; ++i) { F(h->tr_u[i]); F(h->tr_a[i]); }
  F(h->auxT); F(h->auxS); F(h->auxT2); F(h->auxS2);
  F(h->auxT3); F(h->auxS3); F(h->auxT4); F(h->auxS4);
  F(h->dt_d); F(h->partial); F(h->red_out); F(h->stats);
  if (h->dt_h) (void)hipHostFree(h->dt_h);
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
}

static dg_status validate_mesh(const dg_mesh* m, int dim) {
  if (m->dim != dim) return fail(DG_EINVAL, "all members must have the same dimension");
  for (int a = 0; a < dim; ++a) {
    if (m->n[a] < 1 || m->n[a] > (a == 0 ? (1 << 20) : 32767))
      return fail(DG_EINVAL, "mesh.n[%d] = %d out of range", a, m->n[a]);
    if (!(m->hi[a] > m->lo[a])) return fail(DG_EINVAL, "mesh.hi[%d] must exceed mesh.lo[%d]", a, a);
    if (m->bc[a] != DG_PERIODIC && m->bc[a] != DG_SLIPWALL)
      return fail(DG_EINVAL, "mesh.bc[%d] must be DG_PERIODIC or DG_SLIPWALL", a);
  }
  return DG_OK;
}

// (Re)build the work-item table for `epb` elements per block.
// Item orders (3D members; a 2D member's items are always in element order):
//   0: y-bands of `by` rows, z outside y inside a band (below);
//   1: plain element order (x, then y, then z);
//   2: y-bands twice as wide as in order 0.
static void build_items(dg_handle* h, int epb, int order = -1) {
  if (order < 0) order = h->item_order;
  h->items.clear();
  h->item_off.clear();
  for (int m = 0; m < h->nmembers; ++m) {
    h->item_off.push_back((int)h->items.size());
    const MemberDesc& md = h->mem[m];
    for (int e0 = 0; e0 < md.ne; e0 += epb) {
      Item it;
      it.member = m;
      it.e0 = e0;
      it.c0 = e0 % md.n[0];
      const int row = e0 / md.n[0];
      const int c1 = row % md.n[1];
      const int c2 = row / md.n[1];
      it.c12 = c1 + (c2 << 16);
      h->items.push_back(it);
    }
    if (h->dim == 3 && order != 1) {
      // Walk y-bands of `by` rows with z outside y inside a band, so the
      // elements above and below an item were visited at most ~64 items
      // earlier and are still in the XCD's L2 when their faces are read.
      const int per_row = (md.n[0] + epb - 1) / epb;
      const int span = order == 3 ? 256 : (order == 2 ? 128 : 64);
      const int by = std::max(1, std::min(md.n[1], span / std::max(1, per_row)));
      auto key = [&](const Item& it) {
        const int c1 = it.c12 & 0xffff, c2 = it.c12 >> 16;
        return std::make_tuple(c1 / by, c2, c1 % by, it.c0);
      };
      std::stable_sort(h->items.begin() + h->item_off[m], h->items.end(),
                       [&](const Item& x, const Item& y) { return key(x) < key(y); });
    }
  }
  h->item_off.push_back((int)h->items.size());
  h->epb = epb;
  h->item_order = order;
}

static LaunchCfg launch_cfg(const dg_handle* h) {
  LaunchCfg lc;
  lc.threads = h->epb * h->np;
  const int n = (int)h->items.size();
  lc.grid = grid_for_items(n);
  if (h->persist > 0) {
    const int pg = ((h->persist * h->ncu + 7) / 8) * 8;
    if (pg < lc.grid) lc.grid = pg;
  }
  return lc;
}

extern "C" dg_status dg_create_batch(const dg_mesh* meshes, int nmembers, int order, int nvars,
                                     const dg_params* p, dg_handle** out) {
  if (!meshes || !p || !out) return fail(DG_EINVAL, "null argument");
  *out = nullptr;
  if (nmembers < 1) return fail(DG_EINVAL, "nmembers must be >= 1");
  const int dim = meshes[0].dim;
  if (dim != 2 && dim != 3) return fail(DG_EINVAL, "dim must be 2 or 3 (got %d)", dim);
  if (order < 1 || order > (dim == 2 ? kMaxOrder : 4))
    return fail(DG_EINVAL, "order must be in 1..%d for dim %d (got %d)", dim == 2 ? kMaxOrder : 4, dim, order);
  if (p->rain != 0 && p->rain != 1) return fail(DG_EINVAL, "rain must be 0 or 1");
  if (nvars != (p->rain ? 4 : 3) + dim)
    return fail(DG_EINVAL, "nvars must be %d for dim=%d rain=%d (got %d)", (p->rain ? 4 : 3) + dim, dim, p->rain, nvars);
  if (p->precision != DG_FP64 && p->precision != DG_FP32_BULK) return fail(DG_EINVAL, "bad precision");
  if (p->rk != DG_SSPRK43 && p->rk != DG_SSPRK33) return fail(DG_EINVAL, "bad rk scheme");
  if (p->vr_mode != DG_VR_CONST && p->vr_mode != DG_VR_COSMO) return fail(DG_EINVAL, "bad vr_mode");
  if (!(p->newton_rtol > 0) || p->newton_maxit < 1) return fail(DG_EINVAL, "bad Newton settings");
  if (p->basis != DG_BASIS_LOBATTO && p->basis != DG_BASIS_GAUSS) return fail(DG_EINVAL, "bad basis");
  if (!(p->sip_gamma >= 0.0) || !std::isfinite(p->sip_gamma) || !(p->sip_sigma > 0.0) || !std::isfinite(p->sip_sigma))
    return fail(DG_EINVAL, "sip_gamma must be >= 0 and sip_sigma > 0");
  if (p->sip_gamma > 0.0 && p->basis != DG_BASIS_LOBATTO)
    return fail(DG_EUNSUPPORTED, "artificial diffusion exists for the Lobatto basis only");
  if (!(p->sponge_alpha >= 0.0 && p->sponge_alpha <= 1.0) || !std::isfinite(p->sponge_zD))
    return fail(DG_EINVAL, "sponge_alpha must lie in [0, 1] and sponge_zD be finite");
  if (p->sponge_alpha > 0.0)
    for (int m = 0; m < nmembers; ++m)
      if (!(p->sponge_zD < meshes[m].hi[dim - 1]))
        return fail(DG_EINVAL, "sponge_zD must lie below the top of member %d", m);
  for (int m = 0; m < nmembers; ++m) {
    dg_status s = validate_mesh(&meshes[m], dim);
    if (s != DG_OK) return s;
  }
  dg_handle* h = new dg_handle();
  h->dim = dim; h->order = order; h->nvars = nvars; h->rain = p->rain;
  h->prec = p->precision; h->rk = p->rk; h->nmembers = nmembers; h->P = *p;
  const int p1 = order + 1;
  h->np = dim == 2 ? p1 * p1 : p1 * p1 * p1;
  const int epb = elems_per_block(order, dim, p->precision == DG_FP64);
  long long eoff = 0;
  int hoff = 0;
  long long items_max = 0;
  double wq[kMaxP1], Dq[kMaxP1 * kMaxP1];
  lobatto_tables(order, wq, Dq);   // md.lift: Lobatto kernels only
  for (int m = 0; m < nmembers; ++m) {
    const dg_mesh& g = meshes[m];
    MemberDesc md{};
    long long ne = 1;
    md.J = 1.0;
    for (int a = 0; a < 3; ++a) {
      md.n[a] = a < dim ? g.n[a] : 1;
      md.bc[a] = a < dim ? g.bc[a] : 0;
      const double hh = a < dim ? (g.hi[a] - g.lo[a]) / g.n[a] : 2.0;
      md.two_over_h[a] = 2.0 / hh;
      md.lift[a][0] = md.two_over_h[a] / wq[0];
      md.lift[a][1] = md.two_over_h[a] / wq[order];
      if (a < dim) { ne *= g.n[a]; md.J *= 0.5 * hh; }
    }
    {
      double vol = 1.0;
      for (int a = 0; a < dim; ++a) vol *= (g.hi[a] - g.lo[a]) / g.n[a];
      const double hgeo = std::pow(vol, 1.0 / dim);
      md.sip_pre = p->sip_gamma * 0.5 * std::pow(hgeo, 1.0 - 0.5 * dim);
      long long nvm = 1;
      for (int a = 0; a < 3; ++a) {
        md.nvx[a] = a < dim ? g.n[a] + (g.bc[a] == DG_PERIODIC ? 0 : 1) : 1;
        md.sip_tau[a] = a < dim ? p->sip_sigma * order * order * g.n[a] / (g.hi[a] - g.lo[a]) : 0.0;
        nvm *= md.nvx[a];
      }
      md.voff = 0;   // set once every member's vertex count is known
      h->nvert.push_back(nvm);
    }
    for (int a = 0; a < dim; ++a) {
      md.face_J[a] = 1.0;
      for (int b = 0; b < dim; ++b)
        if (b != a) md.face_J[a] *= 0.5 * (g.hi[b] - g.lo[b]) / g.n[b];
    }
    if (ne > (1LL << 30)) { delete h; return fail(DG_EINVAL, "member %d too large", m); }
    md.ne = (int)ne;
    md.eoff = eoff;
    md.hoff = hoff;
    items_max += ne;
    h->hoff.push_back(hoff);
    eoff += ne;
    hoff += md.n[dim - 1] * p1;
    h->mem.push_back(md);
  }
  h->hoff.push_back(hoff);
  long long nvert_tot = 0;
  for (int m = 0; m < nmembers; ++m) {
    h->mem[m].voff = nvert_tot;
    nvert_tot += h->nvert[m];
  }
  build_items(h, epb);
  h->items_cap = items_max;
  {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      h->ncu = prop.multiProcessorCount;
  }
  h->bg_set.assign(nmembers, 0);
  h->etot = eoff;
  h->nnodes = eoff * h->np;
  // per-variable arrays are addressed with 32-bit byte offsets
  if (h->nnodes >= (p->precision == DG_FP64 ? (1LL << 29) : (1LL << 30))) {
    delete h;
    return fail(DG_EINVAL, "a handle holds fewer than 2^29 (FP64) or 2^30 (FP32 bulk) nodes");
  }
  const size_t rsz = h->prec == DG_FP64 ? sizeof(double) : sizeof(float);
  h->state_bytes = (size_t)nvars * h->nnodes * rsz;

  // device buffers
  auto A = [&](void** ptr, size_t bytes) -> bool { return hipMalloc(ptr, bytes) == hipSuccess; };
  bool ok = true;
  ok = ok && A((void**)&h->mem_d, sizeof(MemberDesc) * nmembers);
  ok = ok && A((void**)&h->items_d, sizeof(Item) * h->items_cap);
  ok = ok && A((void**)&h->ka_d, sizeof(KArgs));
  for (auto& b : h->bg_d) ok = ok && A((void**)&b, sizeof(double) * hoff);
  for (auto& b : h->stage) ok = ok && A(&b, h->state_bytes);
  ok = ok && A((void**)&h->auxT, sizeof(double) * h->nnodes);
  ok = ok && A((void**)&h->auxS, sizeof(double) * h->nnodes);
  ok = ok && A((void**)&h->auxT2, sizeof(double) * h->nnodes);
  ok = ok && A((void**)&h->auxS2, sizeof(double) * h->nnodes);
  ok = ok && A((void**)&h->auxT3, sizeof(double) * h->nnodes);
  ok = ok && A((void**)&h->auxS3, sizeof(double) * h->nnodes);
  ok = ok && A((void**)&h->auxT4, sizeof(double) * h->nnodes);
  ok = ok && A((void**)&h->auxS4, sizeof(double) * h->nnodes);
  for (auto& b : h->stage_x) ok = ok && A(&b, h->state_bytes);
  h->sponge = p->sponge_alpha > 0.0;
  if (h->sponge) {
    ok = ok && A(&h->stage_w, h->state_bytes);
    ok = ok && A((void**)&h->sponge_d, sizeof(double) * hoff);
  }
  if (p->basis == DG_BASIS_GAUSS) {
    ok = ok && A((void**)&h->bgf_d, sizeof(double) * 5 * 2 * (hoff / p1));
    // 2D faces of (k+1)^(d-1) quadrature points per element
    const size_t nfe = (size_t)2 * dim * (dim == 2 ? p1 : p1 * p1);
    for (int i = 0; i < 2; ++i) {
      ok = ok && A(&h->tr_u[i], (size_t)nvars * eoff * nfe * rsz);
      ok = ok && A((void**)&h->tr_a[i], (size_t)2 * eoff * nfe * sizeof(double));
    }
  }
  h->sip = p->sip_gamma > 0.0;
  if (h->sip) {
    ok = ok && A((void**)&h->sip_aK, sizeof(double) * 2 * eoff);
    ok = ok && A((void**)&h->sip_av, sizeof(double) * 2 * nvert_tot);
    ok = ok && A(&h->sip_out, h->state_bytes);
  }
  ok = ok && A((void**)&h->dt_d, sizeof(double) * nmembers);
  ok = ok && A((void**)&h->partial, sizeof(double) * 3 * h->items_cap);
  ok = ok && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) == hipSuccess;
  ok = ok && A((void**)&h->red_out, sizeof(double) * 4);
  ok = ok && A((void**)&h->stats, sizeof(unsigned) * 8);
  ok = ok && hipHostMalloc((void**)&h->dt_h, sizeof(double) * nmembers) == hipSuccess;
  if (!ok) {
    const size_t sb = h->state_bytes;
    free_all(h);
    delete h;
    return fail(DG_ENOMEM, "device allocation failed (state of %zu bytes)", sb);
  }
  if (hipMemcpy(h->mem_d, h->mem.data(), sizeof(MemberDesc) * nmembers, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->items_d, h->items.data(), sizeof(Item) * h->items.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(h->stats, 0, sizeof(unsigned) * 8) != hipSuccess ||
      hipMemset(h->auxT, 0, sizeof(double) * h->nnodes) != hipSuccess ||
      hipMemset(h->auxS, 0, sizeof(double) * h->nnodes) != hipSuccess) {
    free_all(h);
    delete h;
    return fail(DG_EHIP, "initial upload failed");
  }
  for (auto& b : h->bg_d) (void)hipMemset(b, 0, sizeof(double) * hoff);

  // kernel argument block
  KArgs& a = h->ka;
  fill_thermo(a, p);
  a.basis = p->basis;
  double xnode[kMaxP1];
  if (p->basis == DG_BASIS_GAUSS) {
    gauss_tables(order, xnode, a.w, a.Dhat, a.gl_m, a.gl_p);
    for (int i = 0; i <= order; ++i) {
      a.lift_m[i] = a.gl_m[i] / a.w[i];
      a.lift_p[i] = a.gl_p[i] / a.w[i];
    }
    a.bgf = h->bgf_d;
    a.bgf_n = 2 * (hoff / p1);
  } else {
    lobatto_tables(order, a.w, a.Dhat, a.Dm);
    lobatto_nodes(order, xnode);
    for (int i = 0; i <= order; ++i) a.xn[i] = xnode[i];
    a.bgf = nullptr;
    a.bgf_n = 0;
  }
  a.sip_aK = h->sip_aK;
  a.sip_av = h->sip_av;
  a.sip_out = h->sip_out;
  a.nvert = nvert_tot;
  a.mem = h->mem_d;
  a.items = h->items_d;
  a.nitems = (int)h->items.size();
  a.nmembers = nmembers;
  a.etot = h->etot;
  a.nnodes = (unsigned)h->nnodes;
  a.bg_rd = h->bg_d[0]; a.bg_rm = h->bg_d[1]; a.bg_rr = h->bg_d[2]; a.bg_E = h->bg_d[3];
  a.bg_p = h->bg_d[4];
  a.stats = h->stats;
  a.sponge = nullptr;
  if (h->sponge) {
    // blending factor at every node height of every member (the L2 projection
    // onto the nodal basis, Lobatto or Gauss, takes the nodal value)
    const double* xl = xnode;
    std::vector<double> dl(hoff, 0.0);
    for (int m = 0; m < nmembers; ++m) {
      const dg_mesh& g = meshes[m];
      const int az = dim - 1;
      const double hz = (g.hi[az] - g.lo[az]) / g.n[az];
      const double zD = p->sponge_zD, zT = g.hi[az];
      for (int c = 0; c < g.n[az]; ++c)
        for (int l = 0; l <= order; ++l) {
          const double z = g.lo[az] + hz * (c + 0.5 * (1.0 + xl[l]));
          dl[h->hoff[m] + c * (order + 1) + l] =
              z < zD ? 0.0 : 0.5 * p->sponge_alpha * (1.0 - std::cos(M_PI * (z - zD) / (zT - zD)));
        }
    }
    if (hipMemcpy(h->sponge_d, dl.data(), sizeof(double) * hoff, hipMemcpyHostToDevice) != hipSuccess) {
      free_all(h);
      delete h;
      return fail(DG_EHIP, "initial upload failed");
    }
    a.sponge = h->sponge_d;
  }
  if (hipMemcpy(h->ka_d, &h->ka, sizeof(KArgs), hipMemcpyHostToDevice) != hipSuccess) {
    free_all(h);
    delete h;
    return fail(DG_EHIP, "initial upload failed");
  }
  *out = h;
  return DG_OK;
}

extern "C" dg_status dg_create(const dg_mesh* mesh, int order, int nvars, const dg_params* p,
                               dg_handle** out) {
  return dg_create_batch(mesh, 1, order, nvars, p, out);
}

extern "C" dg_status dg_destroy(dg_handle* h) {
  if (!h) return DG_OK;
  (void)hipDeviceSynchronize();
  for (auto e : h->ev) (void)hipEventDestroy(e);
  free_all(h);
  delete h;
  return DG_OK;
}

extern "C" long long dg_state_size(const dg_handle* h) { return h ? (long long)h->nvars * h->nnodes : 0; }

extern "C" dg_status dg_member_offset(const dg_handle* h, int member, long long* eoff, long long* ne) {
  if (!h || member < 0 || member >= h->nmembers) return fail(DG_EINVAL, "bad member index");
  if (eoff) *eoff = h->mem[member].eoff;
  if (ne) *ne = h->mem[member].ne;
  return DG_OK;
}

// background pressure: equation of state of the split background (FP64)
__global__ void bg_pressure_kernel(KArgs a, int i0, int n, int rain) {
  const int i = i0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= i0 + n) return;
  const double rd = a.bg_rd[i], rm = a.bg_rm[i], rr = rain ? a.bg_rr[i] : 0.0;
  const SplitOut s = split_point(a, rd, rm, rr, a.bg_E[i], 0.0);
  const double rv = fmin(s.rvs, rm);
  const_cast<double*>(a.bg_p)[i] = (rd * a.Rd + rv * a.Rv) * s.T;
}

// Background traces on the horizontal faces of the Gauss basis, for the
// element rows [r0, r0 + nrows) of the concatenated columns: rho_d, rho_m,
// rho_r and E interpolated from the row's k+1 node heights to its bottom and
// top, and p the equation of state of the traced split background (T and
// rho_v traced as well), so that the unperturbed state has p' = 0 on faces.
__global__ void bg_face_kernel(KArgs a, int K, int r0, int nrows, int rain) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * nrows) return;
  const int r = r0 + i / 2, side = i % 2;
  const int P1 = K + 1;
  const double* L = side ? a.gl_p : a.gl_m;
  double t[6] = {0, 0, 0, 0, 0, 0};
  for (int l = 0; l < P1; ++l) {
    const int iz = r * P1 + l;
    const double rd = a.bg_rd[iz], rm = a.bg_rm[iz], rr = rain ? a.bg_rr[iz] : 0.0, E = a.bg_E[iz];
    const SplitOut s = split_point(a, rd, rm, rr, E, 0.0);
    const double w = L[l];
    t[0] += w * rd;
    t[1] += w * rm;
    t[2] += w * rr;
    t[3] += w * E;
    t[4] += w * s.T;
    t[5] += w * fmin(s.rvs, rm);
  }
  double* bgf = const_cast<double*>(a.bgf);
  const int at = 2 * r + side;
  for (int f = 0; f < 4; ++f) bgf[f * a.bgf_n + at] = t[f];
  bgf[4 * a.bgf_n + at] = (t[0] * a.Rd + t[5] * a.Rv) * t[4];
}

extern "C" dg_status dg_set_background(dg_handle* h, const double* rd, const double* rm, const double* rr,
                                       const double* E, int member) {
  if (!h) return fail(DG_EINVAL, "null handle");
  if (member < 0 || member >= h->nmembers) return fail(DG_EINVAL, "bad member index %d", member);
  if (!rd || !rm || !E) return fail(DG_EINVAL, "null background array");
  const int off = h->hoff[member];
  const int n = h->hoff[member + 1] - off;
  std::vector<double> z(n, 0.0);
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(rd[i]) || !std::isfinite(rm[i]) || !std::isfinite(E[i]) || (rr && !std::isfinite(rr[i])))
      return fail(DG_EINVAL, "non-finite background value at index %d", i);
  HIP_TRY(hipMemcpy(h->bg_d[0] + off, rd, n * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->bg_d[1] + off, rm, n * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->bg_d[2] + off, rr ? rr : z.data(), n * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->bg_d[3] + off, E, n * sizeof(double), hipMemcpyHostToDevice));
  hipLaunchKernelGGL(bg_pressure_kernel, dim3((n + 127) / 128), dim3(128), 0, 0, h->ka, off, n, h->rain);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipDeviceSynchronize());
  std::vector<double> pb(n);
  HIP_TRY(hipMemcpy(pb.data(), h->bg_d[4] + off, n * sizeof(double), hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(pb[i]) || !(pb[i] > 0))
      return fail(DG_EINVAL, "background state at index %d has no valid temperature", i);
  if (h->P.basis == DG_BASIS_GAUSS) {
    const int p1 = h->order + 1;
    const int nrows = n / p1;
    hipLaunchKernelGGL(bg_face_kernel, dim3((2 * nrows + 127) / 128), dim3(128), 0, 0, h->ka, h->order,
                       off / p1, nrows, h->rain);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipDeviceSynchronize());
  }
  h->bg_set[member] = 1;
  return DG_OK;
}

static dg_status ready(dg_handle* h) {
  if (!h) return fail(DG_EINVAL, "null handle");
  for (int m = 0; m < h->nmembers; ++m)
    if (!h->bg_set[m]) return fail(DG_EINVAL, "background of member %d not set", m);
  return DG_OK;
}

static bool do_split(dg_handle* h, const void* U, const double* guess, double* oT, double* o1,
                     double* o2, int api, hipStream_t s) {
  const int n = (int)h->items.size();
  KTimer kt(h, DG_K_SPLIT, s);
  h->splits += h->nnodes;
  const LaunchCfg lc = launch_cfg(h);
  if (h->prec == DG_FP64)
    return Launch<double>::split(h->ka, lc, h->order, h->dim, h->rain, 0, n, U, guess, oT, o1, o2, api, s);
  return Launch<float>::split(h->ka, lc, h->order, h->dim, h->rain, 0, n, U, guess, oT, o1, o2, api, s);
}

// tin / tout: the Gauss basis' trace buffers of the stage state (read) and of
// the new state (written in mode 2)
static bool do_rhs(dg_handle* h, int mode, const void* U, const double* aT, const double* aS, void* out,
                   const void* U0, double c0, double c1, double c2, hipStream_t s,
                   double* oT = nullptr, double* oS = nullptr, int flags = 0, int tin = 0, int tout = 1,
                   int rev = 0) {
  KTimer kt(h, DG_K_STAGE, s);
  if (mode == 2) h->splits += h->nnodes;
  const LaunchCfg lc = launch_cfg(h);
  KArgs ka = h->ka;
  ka.walk_rev = rev;
  if (h->P.basis == DG_BASIS_GAUSS) {
    ka.tr_u_in = h->tr_u[tin];
    ka.tr_a_in = h->tr_a[tin];
    ka.tr_u_out = h->tr_u[tout];
    ka.tr_a_out = h->tr_a[tout];
  }
  if (h->prec == DG_FP64)
    return Launch<double>::rhs(ka, h->ka_d, lc, h->order, h->dim, h->rain, mode, U, aT, aS, out, U0,
                               h->dt_d, c0, c1, c2, oT, oS, flags, s);
  return Launch<float>::rhs(ka, h->ka_d, lc, h->order, h->dim, h->rain, mode, U, aT, aS, out, U0, h->dt_d,
                            c0, c1, c2, oT, oS, flags, s);
}

// Gauss basis: face traces of U and its split (aT, aS) into trace buffer tout
static void do_gauss_trace(dg_handle* h, const void* U, const double* aT, const double* aS, int tout,
                           hipStream_t s) {
  if (h->P.basis != DG_BASIS_GAUSS) return;
  KTimer kt(h, DG_K_OTHER, s);
  const LaunchCfg lc = launch_cfg(h);
  KArgs ka = h->ka;
  ka.tr_u_out = h->tr_u[tout];
  ka.tr_a_out = h->tr_a[tout];
  if (h->prec == DG_FP64)
    Launch<double>::gauss_trace(ka, lc, h->order, h->dim, h->rain, U, aT, aS, s);
  else
    Launch<float>::gauss_trace(ka, lc, h->order, h->dim, h->rain, U, aT, aS, s);
}

// artificial diffusion of the state U into the handle's tendency buffer
// alpha = false: the stage that produced U already wrote its alpha_K
static void do_sip(dg_handle* h, const void* U, hipStream_t s, bool alpha = true) {
  KTimer kt(h, DG_K_OTHER, s);
  const LaunchCfg lc = launch_cfg(h);
  if (h->prec == DG_FP64)
    Launch<double>::sip(h->ka, lc, h->order, h->dim, h->rain, h->nmembers, h->nvert.data(), U, alpha, s);
  else
    Launch<float>::sip(h->ka, lc, h->order, h->dim, h->rain, h->nmembers, h->nvert.data(), U, alpha, s);
}

// The Q3 hexahedral stage kernel (Lobatto basis) can leave alpha_K of the
// state it writes for the next stage's diffusion (kSipAlpha).
static bool stage_writes_alpha(const dg_handle* h) {
  return h->sip && h->P.basis == DG_BASIS_LOBATTO && h->order == 3 && h->dim == 3;
}

extern "C" dg_status dg_rhs(dg_handle* h, const void* U, void* dUdt, hipStream_t s) {
  dg_status st = ready(h);
  if (st != DG_OK) return st;
  if (!U || !dUdt) return fail(DG_EINVAL, "null state pointer");
  if (U == dUdt) return fail(DG_EINVAL, "U and dUdt must not alias");
  if (!do_split(h, U, nullptr, h->auxT, h->auxS, nullptr, 0, s)) return fail(DG_EUNSUPPORTED, "no kernel for this shape");
  if (h->sip) do_sip(h, U, s);
  do_gauss_trace(h, U, h->auxT, h->auxS, 0, s);
  do_rhs(h, 0, U, h->auxT, h->auxS, dUdt, nullptr, 0, 0, 0, s, nullptr, nullptr, h->sip ? kSip : 0, 0, 1);
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

// ---------------------------------------------------------------------------
// right-hand side without allocation: the split scratch in a static array
// ---------------------------------------------------------------------------
// The split that precedes the right-hand side keeps (T, rho_vs(T)) per node
// (16 bytes) between its two kernels.  dg_rhs keeps them in the handle's
// buffers; dg_rhs_noalloc keeps them in this file-scope device array, of which
// every GPU the library runs on holds its own copy until the process ends.
// Host code never passes the array's name to a kernel (on the host it is only
// a stand-in): the device address comes from hipGetSymbolAddress, taken once
// per device with that device current.
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr long long kScratchNodes = (long long)(kScratchBytes / (2 * sizeof(double)));
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};

static dg_status scratch_for_current_device(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(DG_EINVAL, "device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(DG_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DG_OK;
}

extern "C" dg_status dg_rhs_noalloc(dg_handle* h, const void* U, void* dUdt, hipStream_t s) {
  dg_status st = ready(h);
  if (st != DG_OK) return st;
  if (!U || !dUdt) return fail(DG_EINVAL, "null state pointer");
  if (U == dUdt) return fail(DG_EINVAL, "U and dUdt must not alias");
  if (h->P.basis != DG_BASIS_LOBATTO || h->sip)
    return fail(DG_EUNSUPPORTED, "dg_rhs_noalloc covers the Lobatto basis without diffusion");
  if (h->nnodes > kScratchNodes)
    return fail(DG_EINVAL, "dg_rhs_noalloc holds at most %lld nodes in its %zu-byte scratch (handle has %lld)",
                kScratchNodes, kScratchBytes, h->nnodes);
  void* base = nullptr;
  st = scratch_for_current_device(&base);
  if (st != DG_OK) return st;
  double* sT = (double*)base;
  double* sS = sT + h->nnodes;
  if (!do_split(h, U, nullptr, sT, sS, nullptr, 0, s)) return fail(DG_EUNSUPPORTED, "no kernel for this shape");
  do_rhs(h, 0, U, sT, sS, dUdt, nullptr, 0, 0, 0, s);
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

extern "C" dg_status dg_saturation_split(dg_handle* h, const void* U, double* T, int use_guess,
                                         double* rho_v, double* rho_c, hipStream_t s) {
  dg_status st = ready(h);
  if (st != DG_OK) return st;
  if (!U || !T) return fail(DG_EINVAL, "null pointer");
  if (!do_split(h, U, use_guess ? T : nullptr, T, rho_v, rho_c, 1, s))
    return fail(DG_EUNSUPPORTED, "no kernel for this shape");
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

// Shu-Osher coefficients (c0, c1, c2) of out = c0 u0 + c1 u + c2 dt L(u)
struct Stage { double c0, c1, c2; };
static const Stage kSSP43[4] = {{0, 1, 0.5}, {0, 1, 0.5}, {2.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0}, {0, 1, 0.5}};
static const Stage kSSP33[3] = {{0, 1, 1}, {0.75, 0.25, 0.25}, {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0}};

static dg_status upload_dt(dg_handle* h, const double* dt, hipStream_t s) {
  for (int m = 0; m < h->nmembers; ++m) {
    if (!std::isfinite(dt[m]) || !(dt[m] > 0)) return fail(DG_EINVAL, "dt[%d] must be positive and finite", m);
    h->dt_h[m] = dt[m];
  }
  HIP_TRY(hipMemcpyAsync(h->dt_d, h->dt_h, sizeof(double) * h->nmembers, hipMemcpyHostToDevice, s));
  return DG_OK;
}

// One RK step in place on U; stage states go to the handle's buffers.  Each
// fused stage kernel also splits the state it writes, so the next stage reads
// (T, rho_vs) from the ping-pong aux buffers; only the first stage of a call
// runs the stand-alone split.  *cur is the aux buffer holding the split of U.
static dg_status rk_one(dg_handle* h, void* U, bool first, int* cur, hipStream_t s, int step = 0) {
  void* B1 = h->stage[0];
  void* B2 = h->stage[1];
  double* aT[2] = {h->auxT, h->auxT2};
  double* aS[2] = {h->auxS, h->auxS2};
  if (first) {
    *cur = 0;
    do_split(h, U, nullptr, aT[0], aS[0], nullptr, 0, s);
    do_gauss_trace(h, U, aT[0], aS[0], 0, s);
  }
  const int ns = h->rk == DG_SSPRK43 ? 4 : 3;
  const void* in43[4] = {U, B1, B2, B1};
  void* out43[4] = {B1, B2, B1, U};
  const void* in33[3] = {U, B1, B2};
  void* out33[3] = {B1, B2, U};
  for (int st = 0; st < ns; ++st) {
    const Stage& c = h->rk == DG_SSPRK43 ? kSSP43[st] : kSSP33[st];
    const void* in = h->rk == DG_SSPRK43 ? in43[st] : in33[st];
    void* outp = h->rk == DG_SSPRK43 ? out43[st] : out33[st];
    const int a = *cur, b = 1 - *cur;
    // the stored rho_vs(T) anchors the next split; it is evaluated afresh at
    // the last stage of every fourth step so series updates never chain long;
    // the last stage ends the step and applies the sponge
    const bool last = st == ns - 1;
    const int flags = (last && (step & 3) == 3 ? kRefreshRvs : 0) | (last && h->sponge ? kSponge : 0) |
                      (h->sip ? kSip : 0) | (stage_writes_alpha(h) ? kSipAlpha : 0);
    // alpha_K of the stage input: written by the previous stage kernel,
    // except at the first stage of a call
    if (h->sip) do_sip(h, in, s, !(stage_writes_alpha(h) && !(first && st == 0)));
    // every other stage walks its elements in reverse: it starts on what the
    // previous stage wrote last, which the last-level cache still holds.
    // Only states well beyond the L2s take this order (a small state, held
    // by the L2s, ran slower in it: 2D bubble Q4 in FP64, 15.8 -> 19.3 us)
    const bool rev = ((step * ns + st) & 1) && h->state_bytes > (64ull << 20);
    do_rhs(h, 2, in, aT[a], aS[a], outp, U, c.c0, c.c1, c.c2, s, aT[b], aS[b], flags, a, b, rev ? 1 : 0);
    *cur = b;
  }
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

extern "C" dg_status dg_rk_step(dg_handle* h, void* U, const double* dt, int nsteps, hipStream_t s) {
  dg_status st = ready(h);
  if (st != DG_OK) return st;
  if (!U || !dt) return fail(DG_EINVAL, "null pointer");
  if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
  st = upload_dt(h, dt, s);
  if (st != DG_OK) return st;
  int cur = 0;
  for (int i = 0; i < nsteps; ++i) {
    st = rk_one(h, U, i == 0, &cur, s, i);
    if (st != DG_OK) return st;
  }
  return DG_OK;
}

// fixed-order sum of the per-block partials (one block)
__global__ void reduce_partials_kernel(const double* partial, int n, double* out) {
  __shared__ double sm[3][256];
  const int t = threadIdx.x;
  double acc[3] = {0, 0, 0};
  for (int i = t; i < n; i += 256)
    for (int c = 0; c < 3; ++c) acc[c] += partial[3 * i + c];
  for (int c = 0; c < 3; ++c) sm[c][t] = acc[c];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st)
      for (int c = 0; c < 3; ++c) sm[c][t] += sm[c][t + st];
    __syncthreads();
  }
  if (t == 0)
    for (int c = 0; c < 3; ++c) out[c] = sm[c][0];
}

static dg_status reduce_mass(dg_handle* h, int member, const void* U, double* out3, hipStream_t s) {
  dg_status st = ready(h);
  if (st != DG_OK) return st;
  if (!U || !out3) return fail(DG_EINVAL, "null pointer");
  if (member >= h->nmembers) return fail(DG_EINVAL, "bad member index");
  const int i0 = member < 0 ? 0 : h->item_off[member];
  const int i1 = member < 0 ? (int)h->items.size() : h->item_off[member + 1];
  const int n = i1 - i0;
  const LaunchCfg lc = launch_cfg(h);
  if (h->prec == DG_FP64)
    Launch<double>::mass(h->ka, lc, h->order, h->dim, h->rain, i0, n, U, h->partial, s);
  else
    Launch<float>::mass(h->ka, lc, h->order, h->dim, h->rain, i0, n, U, h->partial, s);
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, s, h->partial, n, h->red_out);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(out3, h->red_out, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return DG_OK;
}

extern "C" dg_status dg_reduce_mass(dg_handle* h, const void* U, double* out3, hipStream_t s) {
  return reduce_mass(h, -1, U, out3, s);
}

extern "C" dg_status dg_reduce_mass_member(dg_handle* h, const void* U, double* out3, int member,
                                           hipStream_t s) {
  if (h && (member < 0 || member >= h->nmembers)) return fail(DG_EINVAL, "bad member index %d", member);
  return reduce_mass(h, member, U, out3, s);
}

extern "C" dg_status dg_get_stats(dg_handle* h, dg_stats* out) {
  if (!h || !out) return fail(DG_EINVAL, "null pointer");
  unsigned w[8];
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(w, h->stats, sizeof w, hipMemcpyDeviceToHost));
  out->max_iters = (int)w[0];
  out->nonconverged = w[1];
  out->nonfinite = w[2] ? 1 : 0;
  out->splits = h->splits;
  if (out->nonfinite) return fail(DG_ENONFINITE, "a state with no valid temperature was seen");
  if (out->nonconverged) return fail(DG_ENOCONV, "%lld Newton solves hit the iteration cap", out->nonconverged);
  return DG_OK;
}

extern "C" dg_status dg_reset_stats(dg_handle* h) {
  if (!h) return fail(DG_EINVAL, "null handle");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemset(h->stats, 0, sizeof(unsigned) * 8));
  h->splits = 0;
  return DG_OK;
}

static bool do_vjp(dg_handle* h, const void* U, const double* aT, const double* aS, const void* lam,
                   void* out, const void* X1, const void* X2, const double* dt, double cx1, double cx2,
                   double c1, double c2, hipStream_t s) {
  KTimer kt(h, DG_K_ADJOINT, s);
  const LaunchCfg lc = launch_cfg(h);
  if (h->prec == DG_FP64)
    return Launch<double>::rhs_vjp(h->ka, lc, h->order, h->dim, h->rain, U, aT, aS, lam, out, X1, X2, dt, cx1,
                                   cx2, c1, c2, s);
  return Launch<float>::rhs_vjp(h->ka, lc, h->order, h->dim, h->rain, U, aT, aS, lam, out, X1, X2, dt, cx1,
                                cx2, c1, c2, s);
}

extern "C" dg_status dg_rhs_vjp(dg_handle* h, const void* U, const void* lam, void* Ub, hipStream_t s) {
  dg_status st = ready(h);
  if (st != DG_OK) return st;
  if (h->P.basis != DG_BASIS_LOBATTO || h->sip)
    return fail(DG_EUNSUPPORTED, "adjoints exist for the Lobatto basis without diffusion only");
  if (!U || !lam || !Ub) return fail(DG_EINVAL, "null pointer");
  if (Ub == U || Ub == lam) return fail(DG_EINVAL, "U_bar must not alias U or dUdt_bar");
  if (!do_split(h, U, nullptr, h->auxT, h->auxS, nullptr, 0, s)) return fail(DG_EUNSUPPORTED, "no kernel for this shape");
  do_vjp(h, U, h->auxT, h->auxS, lam, Ub, nullptr, nullptr, nullptr, 0, 0, 0.0, 1.0, s);
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

extern "C" dg_status dg_saturation_split_vjp(dg_handle* h, const void* U, const double* Tb, const double* rvb,
                                             const double* rcb, void* Ub, hipStream_t s) {
  dg_status st = ready(h);
  if (st != DG_OK) return st;
  if (!U || !Ub) return fail(DG_EINVAL, "null pointer");
  if (Ub == U) return fail(DG_EINVAL, "U_bar must not alias U");
  if (!do_split(h, U, nullptr, h->auxT, h->auxS, nullptr, 0, s)) return fail(DG_EUNSUPPORTED, "no kernel for this shape");
  KTimer kt(h, DG_K_ADJOINT, s);
  bool ok;
  const LaunchCfg lc = launch_cfg(h);
  if (h->prec == DG_FP64)
    ok = Launch<double>::split_vjp(h->ka, lc, h->order, h->dim, h->rain, U, h->auxT, h->auxS, Tb, rvb, rcb, Ub, s);
  else
    ok = Launch<float>::split_vjp(h->ka, lc, h->order, h->dim, h->rain, U, h->auxT, h->auxS, Tb, rvb, rcb, Ub, s);
  if (!ok) return fail(DG_EUNSUPPORTED, "no kernel for this shape");
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

// Adjoint of one Shu-Osher step.  The stage states u1..u3 (and their splits)
// are recomputed from U_n with the forward stage kernels, then the stages are
// transposed in reverse order:
//   SSPRK(4,3): r3 = w + dt/2 J3^T w;  r2 = r3/3 + dt/6 J2^T r3;
//               r1 = r2 + dt/2 J1^T r2; r0 = 2/3 r3 + r1 + dt/2 J0^T r1
//   SSPRK(3,3): r2 = 2/3 w + 2 dt/3 J2^T w; r1 = r2/4 + dt/4 J1^T r2;
//               r0 = w/3 + 3/4 r2 + r1 + dt J0^T r1
// with J_s the Jacobian of the right-hand side at stage state u_s.
extern "C" dg_status dg_rk_step_vjp(dg_handle* h, const void* Un, const void* W, void* Ub0, const double* dt,
                                    hipStream_t s) {
  dg_status st = ready(h);
  if (st != DG_OK) return st;
  if (h->P.basis != DG_BASIS_LOBATTO || h->sip)
    return fail(DG_EUNSUPPORTED, "adjoints exist for the Lobatto basis without diffusion only");
  if (!Un || !W || !Ub0 || !dt) return fail(DG_EINVAL, "null pointer");
  if (Ub0 == Un || Ub0 == W) return fail(DG_EINVAL, "U_n_bar must not alias U_n or U_np1_bar");
  st = upload_dt(h, dt, s);
  if (st != DG_OK) return st;
  void* u1 = h->stage_x[0];
  void* u2 = h->stage_x[1];
  void* u3 = h->stage_x[2];
  void* B1 = h->stage[0];
  void* B2 = h->stage[1];
  void* B3 = h->stage_x[3];
  double* aT[4] = {h->auxT, h->auxT2, h->auxT3, h->auxT4};
  double* aS[4] = {h->auxS, h->auxS2, h->auxS3, h->auxS4};
  // the step ends with the sponge: its transpose acts first
  const void* Wt = W;
  if (h->sponge) {
    const LaunchCfg lc = launch_cfg(h);
    KTimer kt(h, DG_K_ADJOINT, s);
    if (h->prec == DG_FP64) Launch<double>::sponge_vjp(h->ka, lc, h->order, h->dim, h->rain, W, h->stage_w, s);
    else Launch<float>::sponge_vjp(h->ka, lc, h->order, h->dim, h->rain, W, h->stage_w, s);
    Wt = h->stage_w;
  }
  // recompute the stages
  do_split(h, Un, nullptr, aT[0], aS[0], nullptr, 0, s);
  if (h->rk == DG_SSPRK43) {
    do_rhs(h, 2, Un, aT[0], aS[0], u1, Un, kSSP43[0].c0, kSSP43[0].c1, kSSP43[0].c2, s, aT[1], aS[1], 0);
    do_rhs(h, 2, u1, aT[1], aS[1], u2, Un, kSSP43[1].c0, kSSP43[1].c1, kSSP43[1].c2, s, aT[2], aS[2], 0);
    do_rhs(h, 2, u2, aT[2], aS[2], u3, Un, kSSP43[2].c0, kSSP43[2].c1, kSSP43[2].c2, s, aT[3], aS[3], 0);
    do_vjp(h, u3, aT[3], aS[3], Wt, B3, nullptr, nullptr, h->dt_d, 0, 0, 1.0, 0.5, s);
    do_vjp(h, u2, aT[2], aS[2], B3, B2, nullptr, nullptr, h->dt_d, 0, 0, 1.0 / 3.0, 1.0 / 6.0, s);
    do_vjp(h, u1, aT[1], aS[1], B2, B1, nullptr, nullptr, h->dt_d, 0, 0, 1.0, 0.5, s);
    do_vjp(h, Un, aT[0], aS[0], B1, Ub0, B3, nullptr, h->dt_d, 2.0 / 3.0, 0, 1.0, 0.5, s);
  } else {
    do_rhs(h, 2, Un, aT[0], aS[0], u1, Un, kSSP33[0].c0, kSSP33[0].c1, kSSP33[0].c2, s, aT[1], aS[1], 0);
    do_rhs(h, 2, u1, aT[1], aS[1], u2, Un, kSSP33[1].c0, kSSP33[1].c1, kSSP33[1].c2, s, aT[2], aS[2], 0);
    do_vjp(h, u2, aT[2], aS[2], Wt, B2, nullptr, nullptr, h->dt_d, 0, 0, 2.0 / 3.0, 2.0 / 3.0, s);
    do_vjp(h, u1, aT[1], aS[1], B2, B1, nullptr, nullptr, h->dt_d, 0, 0, 0.25, 0.25, s);
    do_vjp(h, Un, aT[0], aS[0], B1, Ub0, Wt, B2, h->dt_d, 1.0 / 3.0, 0.75, 1.0, 1.0, s);
  }
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

extern "C" dg_status dg_timing_enable(dg_handle* h, int enable) {
  if (!h) return fail(DG_EINVAL, "null handle");
  if (enable) {
    if (h->ev.empty()) {
      h->ev.resize(2 * kEvPairs);
      h->ev_class.resize(kEvPairs);
      for (auto& e : h->ev) HIP_TRY(hipEventCreate(&e));
    }
    timing_flush(h);
    for (int c = 0; c < 4; ++c) { h->t_ms[c] = 0; h->t_n[c] = 0; }
    h->timing = true;
  } else {
    timing_flush(h);
    h->timing = false;
  }
  return DG_OK;
}

extern "C" dg_status dg_timing_read(dg_handle* h, int kclass, double* total_ms, long long* launches) {
  if (!h || kclass < 0 || kclass > 3) return fail(DG_EINVAL, "bad handle or class");
  timing_flush(h);
  if (total_ms) *total_ms = h->t_ms[kclass];
  if (launches) *launches = h->t_n[kclass];
  return DG_OK;
}

static dg_status upload_items(dg_handle* h) {
  HIP_TRY(hipMemcpy(h->items_d, h->items.data(), sizeof(Item) * h->items.size(), hipMemcpyHostToDevice));
  h->ka.nitems = (int)h->items.size();
  HIP_TRY(hipMemcpy(h->ka_d, &h->ka, sizeof(KArgs), hipMemcpyHostToDevice));
  return DG_OK;
}

extern "C" dg_status dg_set_launch(dg_handle* h, int epb, int persist) {
  if (!h) return fail(DG_EINVAL, "null handle");
  const int emax = elems_per_block(h->order, h->dim, h->prec == DG_FP64);
  if (epb < 1 || epb > emax) return fail(DG_EINVAL, "elements per block must be in 1..%d", emax);
  if (persist < 0 || persist > 64) return fail(DG_EINVAL, "persistent blocks per CU must be in 0..64");
  HIP_TRY(hipDeviceSynchronize());
  if (epb != h->epb) {
    build_items(h, epb);
    dg_status st = upload_items(h);
    if (st != DG_OK) return st;
  }
  h->persist = persist;
  return DG_OK;
}

extern "C" dg_status dg_set_item_order(dg_handle* h, int order) {
  if (!h) return fail(DG_EINVAL, "null handle");
  if (order < 0 || order > 3) return fail(DG_EINVAL, "item order must be 0, 1, 2 or 3");
  HIP_TRY(hipDeviceSynchronize());
  if (order != h->item_order) {
    build_items(h, h->epb, order);
    dg_status st = upload_items(h);
    if (st != DG_OK) return st;
  }
  return DG_OK;
}

extern "C" dg_status dg_get_item_order(const dg_handle* h, int* order) {
  if (!h || !order) return fail(DG_EINVAL, "null pointer");
  *order = h->item_order;
  return DG_OK;
}

extern "C" dg_status dg_get_launch(const dg_handle* h, int* epb, int* persist) {
  if (!h) return fail(DG_EINVAL, "null handle");
  if (epb) *epb = h->epb;
  if (persist) *persist = h->persist;
  return DG_OK;
}

// Time `nsteps` RK steps of a copy of U for each launch geometry and keep the
// fastest: elements per block in {max, max/2, max/4} x persistent blocks per
// CU in {0, 1, 2, 4}.
extern "C" dg_status dg_autotune(dg_handle* h, const void* U, const double* dt, int nsteps, int* best_epb,
                                 int* best_persist, double* best_ms) {
  dg_status st = ready(h);
  if (st != DG_OK) return st;
  if (!U || !dt || nsteps < 1) return fail(DG_EINVAL, "bad autotune arguments");
  st = upload_dt(h, dt, 0);
  if (st != DG_OK) return st;
  const int emax = elems_per_block(h->order, h->dim, h->prec == DG_FP64);
  const int cand_e[3] = {emax, emax / 2, emax / 4};
  const int cand_p[4] = {0, 1, 2, 4};
  const int norders = h->dim == 3 ? 4 : 1;   // 2D items are always in element order
  void* W = h->stage_x[0];
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const bool timing = h->timing;
  h->timing = false;
  double best = 1e300;
  int be = h->epb, bp = h->persist, bo = h->item_order;
  for (int io = 0; io < norders; ++io)
  for (int ie = 0; ie < 3; ++ie) {
    if (cand_e[ie] < 1 || (ie > 0 && cand_e[ie] == cand_e[ie - 1])) continue;
    for (int ip = 0; ip < 4; ++ip) {
      st = dg_set_item_order(h, io);
      if (st == DG_OK) st = dg_set_launch(h, cand_e[ie], cand_p[ip]);
      if (st != DG_OK) { h->timing = timing; return st; }
      HIP_TRY(hipMemcpy(W, U, h->state_bytes, hipMemcpyDeviceToDevice));
      int cur = 0;
      rk_one(h, W, true, &cur, 0);                       // warm-up
      HIP_TRY(hipMemcpy(W, U, h->state_bytes, hipMemcpyDeviceToDevice));
      HIP_TRY(hipEventRecord(e0, 0));
      for (int i = 0; i < nsteps; ++i) rk_one(h, W, i == 0, &cur, 0, i);
      HIP_TRY(hipEventRecord(e1, 0));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best) { best = ms; be = cand_e[ie]; bp = cand_p[ip]; bo = io; }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->timing = timing;
  st = dg_set_item_order(h, bo);
  if (st == DG_OK) st = dg_set_launch(h, be, bp);
  if (st != DG_OK) return st;
  if (best_epb) *best_epb = be;
  if (best_persist) *best_persist = bp;
  if (best_ms) *best_ms = best / nsteps;
  return DG_OK;
}

// nsteps RK steps replayed from a captured hipGraph.  The graph holds the
// split and stage kernels of all steps; dt is read from device memory, which
// is updated before each replay.  It is captured again when U, nsteps or the
// launch geometry change.
extern "C" dg_status dg_rk_step_graph(dg_handle* h, void* U, const double* dt, int nsteps, hipStream_t s) {
  dg_status st = ready(h);
  if (st != DG_OK) return st;
  if (!U || !dt) return fail(DG_EINVAL, "null pointer");
  if (nsteps < 1) return fail(DG_EINVAL, "nsteps must be >= 1");
  if (h->timing) return fail(DG_EINVAL, "disable kernel timing before using graphs");
  if (!h->graph_exec || h->graph_U != U || h->graph_nsteps != nsteps || h->graph_epb != h->epb ||
      h->graph_persist != h->persist) {
    if (h->graph_exec) { (void)hipGraphExecDestroy(h->graph_exec); h->graph_exec = nullptr; }
    if (h->graph) { (void)hipGraphDestroy(h->graph); h->graph = nullptr; }
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    int cur = 0;
    dg_status cs = DG_OK;
    for (int i = 0; i < nsteps && cs == DG_OK; ++i) cs = rk_one(h, U, i == 0, &cur, h->cap_stream, i);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(h->cap_stream, &g);
    if (cs != DG_OK) { if (g) (void)hipGraphDestroy(g); return cs; }
    if (ce != hipSuccess) return fail(DG_EHIP, "graph capture failed: %s", hipGetErrorString(ce));
    h->graph = g;
    HIP_TRY(hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0));
    h->graph_U = U;
    h->graph_nsteps = nsteps;
    h->graph_epb = h->epb;
    h->graph_persist = h->persist;
  }
  st = upload_dt(h, dt, s);
  if (st != DG_OK) return st;
  HIP_TRY(hipGraphLaunch(h->graph_exec, s));
  h->splits += (long long)h->nnodes * nsteps * (h->rk == DG_SSPRK43 ? 4 : 3);
  return DG_OK;
}
