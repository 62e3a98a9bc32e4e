// Inviscid Euler fluxes of App. A on a Cartesian grid, shared by the stage
// kernels and the fused stage-pair kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels_common.hpp"

namespace atns {

// The fluxes of a point are computed by its own thread or, at a tile edge, by
// an apron thread of the neighbouring tile.  The fused multiply-adds are
// written out and no other contraction is allowed here, so both call sites
// give the same bits and results do not depend on the tile shape.
template <typename T>
__device__ __forceinline__ void euler_prims(const T u[5], T gm1, T& iv_rho, T& p) {
#pragma clang fp contract(off)
  iv_rho = recip(u[0]);   // FP32: reciprocal estimate and one Newton step
  const T m2 = fma(u[1], u[1], fma(u[2], u[2], u[3] * u[3]));
  p = gm1 * fma(T(-0.5) * m2, iv_rho, u[4]);
}

// Inviscid flux along direction d (0, 1, 2) of conserved state u.
template <typename T>
__device__ __forceinline__ void euler_flux(const T u[5], int d, T gm1, T f[5]) {
#pragma clang fp contract(off)
  T ir, p;
  euler_prims(u, gm1, ir, p);
  const T vel = u[1 + d] * ir;
  f[0] = u[1 + d];
  f[1] = d == 0 ? fma(u[1], vel, p) : u[1] * vel;
  f[2] = d == 1 ? fma(u[2], vel, p) : u[2] * vel;
  f[3] = d == 2 ? fma(u[3], vel, p) : u[3] * vel;
  f[4] = (u[4] + p) * vel;
}

}  // namespace atns
