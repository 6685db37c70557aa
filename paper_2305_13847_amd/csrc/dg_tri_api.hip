// Host side of the triangle interface (include/dg_tri.h): validation, the
// reference tables of the Dubiner basis and the Duffy-mapped rule, mesh and
// background buffers, and the sequencing of the kernels of dg_tri.h on the
// caller's stream.  Every step of the method runs in those kernels.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <type_traits>

#include "dg_tri.h"
#include "dg_tri_dev.h"
#include "dg_tri_tables.h"

using namespace dgm;

namespace dgm {
dg_status api_fail(dg_status s, const char* msg);
void fill_thermo(KArgs& a, const dg_params* p);
}

static dg_status tfail(dg_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return api_fail(s, buf);
}

#define TRI_HIP(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return tfail(DG_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

template <typename R, int K>
static hipError_t upload_tab() {
  TriTab<R, K> T;
  std::memset(&T, 0, sizeof T);
  fill_tab(T);
#define TRI_UP(S) return hipMemcpyToSymbol(HIP_SYMBOL(S), &T, sizeof T, 0, hipMemcpyHostToDevice)
  if constexpr (sizeof(R) == 4) {
    if constexpr (K == 1) TRI_UP(c_tri_f1);
    else if constexpr (K == 2) TRI_UP(c_tri_f2);
    else if constexpr (K == 3) TRI_UP(c_tri_f3);
    else TRI_UP(c_tri_f4);
  } else {
    if constexpr (K == 1) TRI_UP(c_tri_d1);
    else if constexpr (K == 2) TRI_UP(c_tri_d2);
    else if constexpr (K == 3) TRI_UP(c_tri_d3);
    else TRI_UP(c_tri_d4);
  }
#undef TRI_UP
}

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct dg_tri {
  int order = 0, nvars = 0, rain = 0, prec = 0, rk = 0, np = 0, nq = 0;
  int ne = 0, nz = 0;
  double z0 = 0.0, dz = 1.0;
  dg_params P{};
  std::vector<double> xy_h;
  bool bg_set = false;
  size_t state_bytes = 0;
  double* xy_d = nullptr;
  int* nbr_d = nullptr;
  double* bgl_d = nullptr;
  void* stage[2] = {nullptr, nullptr};
  double* aux[2] = {nullptr, nullptr};   // (T_h, rho_v,h) coefficients, ping-pong
  unsigned* stats = nullptr;
  long long splits = 0;
  KArgs ka{};
  TriArgs ta{};
  // kernel timing
  bool timing = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_class;
  int ev_used = 0;
  double t_ms[4] = {0, 0, 0, 0};
  long long t_n[4] = {0, 0, 0, 0};
};

static const int kTriEvPairs = 1024;

static void tri_flush(dg_tri* h) {
  if (!h->timing) return;
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

struct TriTimer {
  dg_tri* h;
  int slot = -1;
  hipStream_t s;
  TriTimer(dg_tri* hh, int cls, hipStream_t ss) : h(hh), s(ss) {
    if (!h->timing) return;
    if (h->ev_used == kTriEvPairs) tri_flush(h);
    slot = h->ev_used++;
    h->ev_class[slot] = cls;
    (void)hipEventRecord(h->ev[2 * slot], s);
  }
  ~TriTimer() {
    if (slot >= 0) (void)hipEventRecord(h->ev[2 * slot + 1], s);
  }
};

static void tri_free(dg_tri* h) {
  (void)hipFree(h->xy_d);
  (void)hipFree(h->nbr_d);
  (void)hipFree(h->bgl_d);
  for (auto p : h->stage) (void)hipFree(p);
  for (auto p : h->aux) (void)hipFree(p);
  (void)hipFree(h->stats);
  for (auto e : h->ev) (void)hipEventDestroy(e);
  h->ev.clear();
}

// run f(k, rain) with compile-time order and rain flag
template <typename F>
static bool tri_dispatch(int K, int rain, F&& f) {
#define TRI_CASE(k, r)                                                              \
  if (K == k && rain == r) {                                                        \
    f(std::integral_constant<int, k>{}, std::integral_constant<int, r>{});          \
    return true;                                                                    \
  }
  TRI_CASE(1, 0) TRI_CASE(1, 1) TRI_CASE(2, 0) TRI_CASE(2, 1)
  TRI_CASE(3, 0) TRI_CASE(3, 1) TRI_CASE(4, 0) TRI_CASE(4, 1)
#undef TRI_CASE
  return false;
}

static unsigned tri_blocks(long long n) { return (unsigned)((n + 63) / 64); }

// blocks of the point-per-thread kernels: EPB elements each, rounded up to a
// multiple of the 8 XCDs (tri_first_element)
template <int K>
static unsigned tri_grid(long long ne) {
  const long long nb = (ne + TriBlock<K>::EPB - 1) / TriBlock<K>::EPB;
  return (unsigned)(((nb + 7) / 8) * 8);
}

extern "C" dg_status dg_tri_create(const dg_tri_mesh* m, int order, int nvars, const dg_params* p, dg_tri** out) {
  if (!m || !p || !out) return tfail(DG_EINVAL, "null argument");
  *out = nullptr;
  if (order < 1 || order > 4) return tfail(DG_EINVAL, "order must be in 1..4 on triangles (got %d)", order);
  if (p->rain != 0 && p->rain != 1) return tfail(DG_EINVAL, "rain must be 0 or 1");
  if (nvars != (p->rain ? 6 : 5))
    return tfail(DG_EINVAL, "nvars must be %d for rain=%d (got %d)", p->rain ? 6 : 5, p->rain, nvars);
  if (p->precision != DG_FP64 && p->precision != DG_FP32_BULK) return tfail(DG_EINVAL, "bad precision");
  if (p->rk != DG_SSPRK43 && p->rk != DG_SSPRK33) return tfail(DG_EINVAL, "bad rk scheme");
  if (p->vr_mode != DG_VR_CONST && p->vr_mode != DG_VR_COSMO) return tfail(DG_EINVAL, "bad vr_mode");
  if (!(p->newton_rtol > 0) || p->newton_maxit < 1) return tfail(DG_EINVAL, "bad Newton settings");
  if (p->sponge_alpha != 0.0 || p->sip_gamma != 0.0)
    return tfail(DG_EUNSUPPORTED, "the sponge and the artificial diffusion are not available on triangles");
  if (m->ne < 1 || m->ne >= (1 << 29)) return tfail(DG_EINVAL, "ne must be in 1..2^29-1 (got %d)", m->ne);
  if (!m->xy || !m->nb || !m->nbf) return tfail(DG_EINVAL, "null mesh array");
  if (m->nz < 1 || !(m->dz > 0.0) || !std::isfinite(m->dz) || !std::isfinite(m->z0))
    return tfail(DG_EINVAL, "background layers need nz >= 1 and a finite dz > 0");
  const int ne = m->ne;
  std::vector<int> nbr((size_t)ne * 3);
  for (int e = 0; e < ne; ++e) {
    const double* v = m->xy + (size_t)e * 6;
    for (int i = 0; i < 6; ++i)
      if (!std::isfinite(v[i])) return tfail(DG_EINVAL, "non-finite vertex in element %d", e);
    const double det = (v[2] - v[0]) * (v[5] - v[1]) - (v[4] - v[0]) * (v[3] - v[1]);
    if (!(det > 0.0)) return tfail(DG_EINVAL, "element %d is not counter-clockwise (det A = %g)", e, det);
    for (int f = 0; f < 3; ++f) {
      const int e2 = m->nb[(size_t)e * 3 + f], f2 = m->nbf[(size_t)e * 3 + f];
      if (e2 < 0) { nbr[(size_t)e * 3 + f] = -1; continue; }
      if (e2 >= ne || f2 < 0 || f2 > 2 || m->nb[(size_t)e2 * 3 + f2] != e || m->nbf[(size_t)e2 * 3 + f2] != f)
        return tfail(DG_EINVAL, "neighbour table is not symmetric at element %d face %d", e, f);
      nbr[(size_t)e * 3 + f] = e2 * 4 + f2;
    }
  }
  dg_tri* h = new dg_tri();
  h->order = order; h->nvars = nvars; h->rain = p->rain; h->prec = p->precision; h->rk = p->rk;
  h->np = (order + 1) * (order + 2) / 2;
  h->nq = (order + 1) * (order + 2);
  h->ne = ne; h->nz = m->nz; h->z0 = m->z0; h->dz = m->dz;
  h->P = *p;
  h->xy_h.assign(m->xy, m->xy + (size_t)ne * 6);
  const size_t es = p->precision == DG_FP64 ? sizeof(double) : sizeof(float);
  h->state_bytes = (size_t)nvars * ne * h->np * es;
  bool ok = true;
  auto A = [&](void** ptr, size_t bytes) { return hipMalloc(ptr, bytes) == hipSuccess; };
  ok = ok && A((void**)&h->xy_d, sizeof(double) * 6 * ne);
  ok = ok && A((void**)&h->nbr_d, sizeof(int) * 3 * ne);
  ok = ok && A((void**)&h->bgl_d, sizeof(double) * 5 * m->nz * (order + 1));
  ok = ok && A(&h->stage[0], h->state_bytes) && A(&h->stage[1], h->state_bytes);
  ok = ok && A((void**)&h->aux[0], sizeof(double) * 2 * ne * h->np);
  ok = ok && A((void**)&h->aux[1], sizeof(double) * 2 * ne * h->np);
  ok = ok && A((void**)&h->stats, sizeof(unsigned) * 8);
  if (!ok) {
    tri_free(h);
    delete h;
    return tfail(DG_ENOMEM, "device allocation failed");
  }
  hipError_t e1 = hipMemcpy(h->xy_d, m->xy, sizeof(double) * 6 * ne, hipMemcpyHostToDevice);
  hipError_t e2 = hipMemcpy(h->nbr_d, nbr.data(), sizeof(int) * 3 * ne, hipMemcpyHostToDevice);
  hipError_t e3 = hipMemset(h->stats, 0, sizeof(unsigned) * 8);
  hipError_t e4 = p->precision == DG_FP64 ? (order == 1 ? upload_tab<double, 1>() : order == 2 ? upload_tab<double, 2>()
                                             : order == 3 ? upload_tab<double, 3>() : upload_tab<double, 4>())
                                          : (order == 1 ? upload_tab<float, 1>() : order == 2 ? upload_tab<float, 2>()
                                             : order == 3 ? upload_tab<float, 3>() : upload_tab<float, 4>());
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess) {
    tri_free(h);
    delete h;
    return tfail(DG_EHIP, "initial upload failed");
  }
  fill_thermo(h->ka, p);
  h->ka.stats = h->stats;
  h->ta.xy = h->xy_d;
  h->ta.nbr = h->nbr_d;
  h->ta.bgl = h->bgl_d;
  h->ta.z0 = m->z0;
  h->ta.inv_dz = 1.0 / m->dz;
  h->ta.nz = m->nz;
  h->ta.ne = ne;
  *out = h;
  return DG_OK;
}

extern "C" dg_status dg_tri_destroy(dg_tri* h) {
  if (!h) return DG_OK;
  (void)hipDeviceSynchronize();
  tri_free(h);
  delete h;
  return DG_OK;
}

extern "C" long long dg_tri_state_size(const dg_tri* h) { return h ? (long long)h->nvars * h->ne * h->np : 0; }
extern "C" long long dg_tri_npoints(const dg_tri* h) { return h ? (long long)h->ne * h->nq : 0; }

extern "C" dg_status dg_tri_set_background(dg_tri* h, const double* rd, const double* rm, const double* rr,
                                           const double* E) {
  if (!h) return tfail(DG_EINVAL, "null handle");
  if (!rd || !rm || !E) return tfail(DG_EINVAL, "null background array");
  const int n = h->nz * (h->order + 1);
  std::vector<double> b((size_t)n * 5, 0.0);
  for (int i = 0; i < n; ++i) {
    const double r2 = rr ? rr[i] : 0.0;
    if (!std::isfinite(rd[i]) || !std::isfinite(rm[i]) || !std::isfinite(E[i]) || !std::isfinite(r2))
      return tfail(DG_EINVAL, "non-finite background value at index %d", i);
    b[(size_t)i * 5 + 0] = rd[i];
    b[(size_t)i * 5 + 1] = rm[i];
    b[(size_t)i * 5 + 2] = h->rain ? r2 : 0.0;
    b[(size_t)i * 5 + 3] = E[i];
  }
  TRI_HIP(hipMemcpy(h->bgl_d, b.data(), sizeof(double) * 5 * n, hipMemcpyHostToDevice));
  hipLaunchKernelGGL(tri_bg_pressure_kernel, dim3((n + 127) / 128), dim3(128), 0, 0, h->ka, h->bgl_d, n);
  TRI_HIP(hipGetLastError());
  TRI_HIP(hipDeviceSynchronize());
  TRI_HIP(hipMemcpy(b.data(), h->bgl_d, sizeof(double) * 5 * n, hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(b[(size_t)i * 5 + 4]) || !(b[(size_t)i * 5 + 4] > 0))
      return tfail(DG_EINVAL, "background state at index %d has no valid temperature", i);
  h->bg_set = true;
  return DG_OK;
}

extern "C" dg_status dg_tri_points(const dg_tri* h, double* xz) {
  if (!h || !xz) return tfail(DG_EINVAL, "null pointer");
  const int K = h->order;
  std::vector<double> xa(K + 2), wa(K + 2), xb(K + 2), wb(K + 2);
  gl_rule(K + 1, xa.data(), wa.data());
  gl_rule(K + 2, xb.data(), wb.data());
  for (int e = 0; e < h->ne; ++e) {
    const double* v = &h->xy_h[(size_t)e * 6];
    for (int j = 0; j < K + 2; ++j)
      for (int i = 0; i < K + 1; ++i) {
        const int q = j * (K + 1) + i;
        const double s = 0.5 * (1.0 + xb[j]);
        const double r = 0.5 * (1.0 + xa[i]) * (1.0 - s);
        for (int c = 0; c < 2; ++c)
          xz[((size_t)e * h->nq + q) * 2 + c] = v[c] + (v[2 + c] - v[c]) * r + (v[4 + c] - v[c]) * s;
      }
  }
  return DG_OK;
}

static dg_status tri_ready(dg_tri* h) {
  if (!h) return tfail(DG_EINVAL, "null handle");
  if (!h->bg_set) return tfail(DG_EINVAL, "background not set");
  return DG_OK;
}

template <typename R>
static bool launch_split(dg_tri* h, const void* C, double* Tn, double* Rn, hipStream_t s) {
  TriTimer kt(h, DG_K_SPLIT, s);
  h->splits += (long long)h->ne * h->nq;
  return tri_dispatch(h->order, h->rain, [&](auto k, auto r) {
    constexpr int K = decltype(k)::value, RN = decltype(r)::value;
    hipLaunchKernelGGL((tri_split_kernel<R, K, RN>), dim3(tri_grid<K>(h->ne)), dim3(256), 0, s, h->ka, h->ta,
                       (const R*)C, Tn, Rn);
  });
}

template <typename R>
static bool launch_stage(dg_tri* h, int mode, const void* C, const double* aux, void* out, const void* C0,
                         double c0, double c1, double c2dt, double* Tn, double* Rn, hipStream_t s) {
  TriTimer kt(h, DG_K_STAGE, s);
  if (mode == 2) h->splits += (long long)h->ne * h->nq;
  return tri_dispatch(h->order, h->rain, [&](auto k, auto r) {
    constexpr int K = decltype(k)::value, RN = decltype(r)::value;
    const dim3 grid(tri_grid<K>(h->ne)), block(256);
    if (mode == 0)
      hipLaunchKernelGGL((tri_stage_kernel<R, K, RN, 0>), grid, block, 0, s, h->ka, h->ta, (const R*)C, aux,
                         (R*)out, (const R*)C0, c0, c1, c2dt, Tn, Rn);
    else
      hipLaunchKernelGGL((tri_stage_kernel<R, K, RN, 2>), grid, block, 0, s, h->ka, h->ta, (const R*)C, aux,
                         (R*)out, (const R*)C0, c0, c1, c2dt, Tn, Rn);
  });
}

static bool do_split(dg_tri* h, const void* C, double* Tn, double* Rn, hipStream_t s) {
  return h->prec == DG_FP64 ? launch_split<double>(h, C, Tn, Rn, s) : launch_split<float>(h, C, Tn, Rn, s);
}

static bool do_stage(dg_tri* h, int mode, const void* C, const double* aux, void* out, const void* C0, double c0,
                     double c1, double c2dt, double* Tn, double* Rn, hipStream_t s) {
  return h->prec == DG_FP64 ? launch_stage<double>(h, mode, C, aux, out, C0, c0, c1, c2dt, Tn, Rn, s)
                            : launch_stage<float>(h, mode, C, aux, out, C0, c0, c1, c2dt, Tn, Rn, s);
}

extern "C" dg_status dg_tri_project(dg_tri* h, const double* vals, int nfields, void* C, hipStream_t s) {
  if (!h) return tfail(DG_EINVAL, "null handle");
  if (!vals || !C || nfields < 1) return tfail(DG_EINVAL, "bad projection arguments");
  TriTimer kt(h, DG_K_OTHER, s);
  const long long n = (long long)nfields * h->ne;
  const bool ok = tri_dispatch(h->order, 0, [&](auto k, auto) {
    constexpr int K = decltype(k)::value;
    if (h->prec == DG_FP64)
      hipLaunchKernelGGL((tri_project_kernel<double, K>), dim3(tri_blocks(n)), dim3(64), 0, s, h->ta, vals, nfields,
                         (double*)C);
    else
      hipLaunchKernelGGL((tri_project_kernel<float, K>), dim3(tri_blocks(n)), dim3(64), 0, s, h->ta, vals, nfields,
                         (float*)C);
  });
  if (!ok) return tfail(DG_EINVAL, "no kernel for this order");
  TRI_HIP(hipGetLastError());
  return DG_OK;
}

extern "C" dg_status dg_tri_split(dg_tri* h, const void* C, double* Tc, double* Rvc, hipStream_t s) {
  dg_status st = tri_ready(h);
  if (st != DG_OK) return st;
  if (!C || !Tc || !Rvc) return tfail(DG_EINVAL, "null array");
  if (!do_split(h, C, Tc, Rvc, s)) return tfail(DG_EINVAL, "no kernel for this order");
  TRI_HIP(hipGetLastError());
  return DG_OK;
}

extern "C" dg_status dg_tri_rhs(dg_tri* h, const void* C, void* dC, hipStream_t s) {
  dg_status st = tri_ready(h);
  if (st != DG_OK) return st;
  if (!C || !dC) return tfail(DG_EINVAL, "null array");
  if (C == dC) return tfail(DG_EINVAL, "C and dCdt must not alias");
  const size_t N = (size_t)h->ne * h->np;
  if (!do_split(h, C, h->aux[0], h->aux[0] + N, s)) return tfail(DG_EINVAL, "no kernel for this order");
  do_stage(h, 0, C, h->aux[0], dC, nullptr, 0.0, 0.0, 0.0, nullptr, nullptr, s);
  TRI_HIP(hipGetLastError());
  return DG_OK;
}

// Shu-Osher coefficients (c0 U0 + c1 U + c2 dt L(U)) of the Section 3.3 schemes
struct TriStage {
  double c0, c1, c2;
};
static const TriStage kTri43[4] = {{0, 1, 0.5}, {0, 1, 0.5}, {2.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0}, {0, 1, 0.5}};
static const TriStage kTri33[3] = {{0, 1, 1}, {0.75, 0.25, 0.25}, {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0}};

extern "C" dg_status dg_tri_rk_step(dg_tri* h, void* C, double dt, int nsteps, hipStream_t s) {
  dg_status st = tri_ready(h);
  if (st != DG_OK) return st;
  if (!C) return tfail(DG_EINVAL, "null array");
  if (!(dt > 0.0) || !std::isfinite(dt)) return tfail(DG_EINVAL, "dt must be positive and finite");
  if (nsteps < 0) return tfail(DG_EINVAL, "nsteps must be >= 0");
  if (nsteps == 0) return DG_OK;
  const size_t N = (size_t)h->ne * h->np;
  // the reconstruction of the initial state; every stage then splits its own
  // output for the next one
  if (!do_split(h, C, h->aux[0], h->aux[0] + N, s)) return tfail(DG_EINVAL, "no kernel for this order");
  const TriStage* S = h->rk == DG_SSPRK43 ? kTri43 : kTri33;
  const int ns = h->rk == DG_SSPRK43 ? 4 : 3;
  int a = 0;   // aux buffer of the current stage input
  for (int step = 0; step < nsteps; ++step) {
    // SSPRK(4,3): C -> s0 -> s1 -> s0 (with C) -> C; SSPRK(3,3): C -> s0 -> s1 (with C) -> C
    const void* in = C;
    for (int k = 0; k < ns; ++k) {
      void* out = (k == ns - 1) ? C : h->stage[k % 2];
      const int b = 1 - a;
      do_stage(h, 2, in, h->aux[a], out, C, S[k].c0, S[k].c1, S[k].c2 * dt, h->aux[b], h->aux[b] + N, s);
      a = b;
      in = out;
    }
  }
  TRI_HIP(hipGetLastError());
  return DG_OK;
}

extern "C" dg_status dg_tri_get_stats(dg_tri* h, dg_stats* out) {
  if (!h || !out) return tfail(DG_EINVAL, "null pointer");
  unsigned w[8];
  TRI_HIP(hipDeviceSynchronize());
  TRI_HIP(hipMemcpy(w, h->stats, sizeof w, hipMemcpyDeviceToHost));
  out->max_iters = (int)w[0];
  out->nonconverged = w[1];
  out->nonfinite = w[2] ? 1 : 0;
  out->splits = h->splits;
  if (out->nonfinite) return tfail(DG_ENONFINITE, "a state with no valid temperature was seen");
  if (out->nonconverged) return tfail(DG_ENOCONV, "%lld Newton solves hit the iteration cap", out->nonconverged);
  return DG_OK;
}

extern "C" dg_status dg_tri_reset_stats(dg_tri* h) {
  if (!h) return tfail(DG_EINVAL, "null handle");
  TRI_HIP(hipDeviceSynchronize());
  TRI_HIP(hipMemset(h->stats, 0, sizeof(unsigned) * 8));
  h->splits = 0;
  return DG_OK;
}

extern "C" dg_status dg_tri_timing_enable(dg_tri* h, int enable) {
  if (!h) return tfail(DG_EINVAL, "null handle");
  if (enable && !h->timing) {
    if (h->ev.empty()) {
      h->ev.resize(2 * kTriEvPairs);
      h->ev_class.resize(kTriEvPairs);
      for (auto& e : h->ev) TRI_HIP(hipEventCreate(&e));
    }
    for (int c = 0; c < 4; ++c) { h->t_ms[c] = 0.0; h->t_n[c] = 0; }
    h->ev_used = 0;
    h->timing = true;
  } else if (!enable && h->timing) {
    tri_flush(h);
    h->timing = false;
  }
  return DG_OK;
}

extern "C" dg_status dg_tri_timing_read(dg_tri* h, int kclass, double* total_ms, long long* launches) {
  if (!h || kclass < 0 || kclass > 3) return tfail(DG_EINVAL, "bad handle or class");
  tri_flush(h);
  if (total_ms) *total_ms = h->t_ms[kclass];
  if (launches) *launches = h->t_n[kclass];
  return DG_OK;
}
