// Adjoint kernels of libdgmoist (vector-Jacobian products).
#pragma once
#include "dg_kernels.h"

namespace dgm {

template <typename R, int K, int D, int RAIN>
__global__ void rhs_vjp_kernel(KArgs a, const R* __restrict__ U, const double* __restrict__ auxT,
                               const double* __restrict__ auxS, const R* __restrict__ lam,
                               R* __restrict__ out) {}

template <typename R, int K, int D, int RAIN>
__global__ void split_vjp_kernel(KArgs a, const R* __restrict__ U, const double* __restrict__ auxT,
                                 const double* __restrict__ auxS, const double* __restrict__ Tb,
                                 const double* __restrict__ rvb, const double* __restrict__ rcb,
                                 R* __restrict__ out) {}

}  // namespace dgm
