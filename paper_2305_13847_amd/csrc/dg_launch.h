// Host-side launchers: map runtime (order, dimension, rain) to the kernel
// instantiations.  Each precision is instantiated in its own translation unit.
#pragma once
#include <type_traits>
#include "dg_kernels.h"
#include "dg_q3.h"
#include "dg_gauss.h"
#include "dg_sip.h"
#include "dg_vjp.h"

namespace dgm {

template <typename F>
bool dispatch_shape(int K, int D, int rain, F&& f) {
#define DGM_CASE(k, d, r)                                                         \
  if (K == k && D == d && rain == r) {                                            \
    f(std::integral_constant<int, k>{}, std::integral_constant<int, d>{},         \
      std::integral_constant<int, r>{});                                          \
    return true;                                                                  \
  }
  DGM_CASE(1, 2, 0) DGM_CASE(1, 2, 1) DGM_CASE(1, 3, 0) DGM_CASE(1, 3, 1)
  DGM_CASE(2, 2, 0) DGM_CASE(2, 2, 1) DGM_CASE(2, 3, 0) DGM_CASE(2, 3, 1)
  DGM_CASE(3, 2, 0) DGM_CASE(3, 2, 1) DGM_CASE(3, 3, 0) DGM_CASE(3, 3, 1)
  DGM_CASE(4, 2, 0) DGM_CASE(4, 2, 1) DGM_CASE(4, 3, 0) DGM_CASE(4, 3, 1)
  // 2D only above 4: a 3D element of order >= 5 has more nodes than a block
  DGM_CASE(5, 2, 0) DGM_CASE(5, 2, 1) DGM_CASE(6, 2, 0) DGM_CASE(6, 2, 1)
  DGM_CASE(7, 2, 0) DGM_CASE(7, 2, 1)
#undef DGM_CASE
  return false;
}

inline int threads_per_block(int K, int D) {
  int np = (D == 2) ? (K + 1) * (K + 1) : (K + 1) * (K + 1) * (K + 1);
  int epb = 256 / np > 0 ? 256 / np : 1;
  return epb * np;
}

inline int elems_per_block(int K, int D, bool fp64) {
  const int np = (D == 2) ? (K + 1) * (K + 1) : (K + 1) * (K + 1) * (K + 1);
  const int bt = fp64 ? block_threads<double>() : block_threads<float>();
  return bt / np > 0 ? bt / np : 1;
}

// Launch geometry of a handle: threads per block (EPB elements) and grid size.
struct LaunchCfg {
  int threads;
  int grid;
};

template <typename R>
struct Launch {
  // API != 0: write T, rho_v, rho_c; otherwise T and rho_vs(T)
  static bool split(const KArgs& a, LaunchCfg lc, int K, int D, int rain, int item0, int nitems,
                    const void* U, const double* guess, double* oT, double* o1, double* o2, int api,
                    hipStream_t s) {
    if (nitems <= 0) return true;
    return dispatch_shape(K, D, rain, [&](auto k, auto d, auto r) {
      constexpr int K_ = decltype(k)::value, D_ = decltype(d)::value, R_ = decltype(r)::value;
      // one block per work item whatever the persistence setting (the split
      // kernel has no item loop)
      dim3 grid(grid_for_items(nitems)), block(lc.threads);
      if (api)
        hipLaunchKernelGGL((split_kernel<R, K_, D_, R_, 1>), grid, block, 0, s, a, item0, nitems,
                           (const R*)U, guess, oT, o1, o2);
      else
        hipLaunchKernelGGL((split_kernel<R, K_, D_, R_, 0>), grid, block, 0, s, a, item0, nitems,
                           (const R*)U, guess, oT, o1, o2);
    });
  }

  // mode 0: out = dU/dt; mode 1: out = c0 U0 + c1 U + c2 dt dU/dt; mode 2: mode 1 and the split
  // of out into (oT, oS)
  static bool rhs(const KArgs& a, const KArgs* a_dev, LaunchCfg lc, int K, int D, int rain, int mode, const void* U,
                  const double* auxT, const double* auxS, void* out, const void* U0,
                  const double* dt, double c0, double c1, double c2, double* oT, double* oS,
                  int flags, hipStream_t s) {
    return dispatch_shape(K, D, rain, [&](auto k, auto d, auto r) {
      constexpr int K_ = decltype(k)::value, D_ = decltype(d)::value, R_ = decltype(r)::value;
      dim3 grid(lc.grid), block(lc.threads);
#define DGM_RHS(KER, M)                                                                           \
  hipLaunchKernelGGL((KER<R, K_, D_, R_, M>), grid, block, 0, s, a, (const R*)U, auxT, auxS,       \
                     (R*)out, (const R*)U0, dt, c0, c1, c2, oT, oS, flags)
      // the persistent (looping) variant only when the grid is smaller than the items
      const bool persist = (int)grid.x < grid_for_items(a.nitems);
      if (a.basis == 1) {
        // Gauss nodes: one block per work item whatever the persistence
        // setting (the kernel has no item loop)
        grid = dim3(grid_for_items(a.nitems));
        if (mode == 0) DGM_RHS(rhs_gauss_kernel, 0);
        else if (mode == 1) DGM_RHS(rhs_gauss_kernel, 1);
        else DGM_RHS(rhs_gauss_kernel, 2);
      } else if (K_ == 3 && D_ == 3) {
        // Q3 hexahedra: one wavefront per element, one work item per block
        // whatever the persistence setting (the kernel has no item loop)
        grid = dim3(grid_for_items(a.nitems));
        if (mode == 0) hipLaunchKernelGGL((rhs_q3_kernel<R, R_, 0>), grid, block, 0, s, a, (const R*)U, auxT, auxS,
                                           (R*)out, (const R*)U0, dt, c0, c1, c2, oT, oS, flags);
        else if (mode == 1) hipLaunchKernelGGL((rhs_q3_kernel<R, R_, 1>), grid, block, 0, s, a, (const R*)U, auxT,
                                                auxS, (R*)out, (const R*)U0, dt, c0, c1, c2, oT, oS, flags);
        else hipLaunchKernelGGL((rhs_q3_kernel<R, R_, 2>), grid, block, 0, s, a, (const R*)U, auxT, auxS,
                                (R*)out, (const R*)U0, dt, c0, c1, c2, oT, oS, flags);
      } else if (mode != 2 || !persist) {
        // rhs_kernel takes one work item per block: the full grid
        grid = dim3(grid_for_items(a.nitems));
        if (mode == 0) DGM_RHS(rhs_kernel, 0);
        else if (mode == 1) DGM_RHS(rhs_kernel, 1);
        else DGM_RHS(rhs_kernel, 2);
      } else
        hipLaunchKernelGGL((rhs_kernel_persistent<R, K_, D_, R_, 2>), grid, block, 0, s, a, a_dev, (const R*)U,
                           auxT, auxS, (R*)out, (const R*)U0, dt, c0, c1, c2, oT, oS, flags);
#undef DGM_RHS
    });
  }

  // Gauss basis: face traces of a state and its split
  static bool gauss_trace(const KArgs& a, LaunchCfg lc, int K, int D, int rain, const void* U,
                          const double* auxT, const double* auxS, hipStream_t s) {
    return dispatch_shape(K, D, rain, [&](auto k, auto d, auto r) {
      constexpr int K_ = decltype(k)::value, D_ = decltype(d)::value, R_ = decltype(r)::value;
      hipLaunchKernelGGL((gauss_trace_kernel<R, K_, D_, R_>), dim3(lc.grid), dim3(lc.threads), 0, s, a,
                         (const R*)U, auxT, auxS);
    });
  }

  // artificial diffusion: alpha_K (unless the previous stage wrote it),
  // vertex means (all members), tendency
  static bool sip(const KArgs& a, LaunchCfg lc, int K, int D, int rain, int nmembers, const long long* nvert,
                  const void* U, bool alpha, hipStream_t s) {
    return dispatch_shape(K, D, rain, [&](auto k, auto d, auto r) {
      constexpr int K_ = decltype(k)::value, D_ = decltype(d)::value, R_ = decltype(r)::value;
      // one block per work item whatever the persistence setting (the SIP
      // kernels have no item loop)
      const dim3 grid(grid_for_items(a.nitems));
      if (alpha)
        hipLaunchKernelGGL((sip_alpha_kernel<R, K_, D_, R_>), grid, dim3(lc.threads), 0, s, a,
                           (const R*)U);
      hipLaunchKernelGGL((sip_vertex_kernel<D_>), dim3((unsigned)((a.nvert + 127) / 128)), dim3(128), 0, s, a);
      hipLaunchKernelGGL((sip_kernel<R, K_, D_, R_>), grid, dim3(lc.threads), 0, s, a, (const R*)U);
    });
  }

  static bool sponge_vjp(const KArgs& a, LaunchCfg lc, int K, int D, int rain, const void* W, void* Wp,
                         hipStream_t s) {
    return dispatch_shape(K, D, rain, [&](auto k, auto d, auto r) {
      constexpr int K_ = decltype(k)::value, D_ = decltype(d)::value, R_ = decltype(r)::value;
      hipLaunchKernelGGL((sponge_vjp_kernel<R, K_, D_, R_>), dim3(lc.grid), dim3(lc.threads), 0, s, a,
                         (const R*)W, (R*)Wp);
    });
  }

  static bool mass(const KArgs& a, LaunchCfg lc, int K, int D, int rain, int item0, int nitems,
                   const void* U, double* partial, hipStream_t s) {
    return dispatch_shape(K, D, rain, [&](auto k, auto d, auto r) {
      constexpr int K_ = decltype(k)::value, D_ = decltype(d)::value, R_ = decltype(r)::value;
      hipLaunchKernelGGL((mass_kernel<R, K_, D_, R_>), dim3(nitems), dim3(lc.threads), 0, s, a, item0,
                         (const R*)U, partial);
    });
  }

  // adjoint of the right-hand side (dg_vjp.h):
  // out = cx1 X1 + cx2 X2 + c1 lam + c2 dt (d rhs/dU)^T lam   (dt = 1 if null)
  static bool rhs_vjp(const KArgs& a, LaunchCfg lc, int K, int D, int rain, const void* U,
                      const double* auxT, const double* auxS, const void* lam, void* out,
                      const void* X1, const void* X2, const double* dt, double cx1, double cx2,
                      double c1, double c2, hipStream_t s) {
    return dispatch_shape(K, D, rain, [&](auto k, auto d, auto r) {
      constexpr int K_ = decltype(k)::value, D_ = decltype(d)::value, R_ = decltype(r)::value;
      hipLaunchKernelGGL((rhs_vjp_kernel<R, K_, D_, R_>), dim3(lc.grid), dim3(lc.threads), 0, s, a, (const R*)U, auxT, auxS, (const R*)lam,
                         (R*)out, (const R*)X1, (const R*)X2, dt, cx1, cx2, c1, c2);
    });
  }

  static bool split_vjp(const KArgs& a, LaunchCfg lc, int K, int D, int rain, const void* U,
                        const double* auxT, const double* auxS, const double* Tb, const double* rvb,
                        const double* rcb, void* out, hipStream_t s) {
    return dispatch_shape(K, D, rain, [&](auto k, auto d, auto r) {
      constexpr int K_ = decltype(k)::value, D_ = decltype(d)::value, R_ = decltype(r)::value;
      hipLaunchKernelGGL((split_vjp_kernel<R, K_, D_, R_>), dim3(lc.grid), dim3(lc.threads), 0, s, a, (const R*)U, auxT, auxS, Tb, rvb, rcb,
                         (R*)out);
    });
  }
};

}  // namespace dgm
