// Kernel launchers (defined in the .hip files).
#pragma once
#include <hip/hip_runtime.h>

#include "layout.hpp"

namespace atns {

template <typename T>
hipError_t launch_euler_stage(const StageParams<T>& p, int ntiles, int kind, hipStream_t s);
template <typename T>
hipError_t launch_ns_stage(const StageParams<T>& p, int ntiles, int kind, hipStream_t s);

hipError_t launch_delays(int8_t* out, const int8_t* inject, long long n, int nblocks, int L,
                         unsigned long long seed, int algo, hipStream_t s);
template <typename T>
hipError_t launch_ring_fill(const StageParams<T>& p, const T* U, int slot, int nblocks, hipStream_t s);
template <typename T>
hipError_t launch_diag(const T* U, const int n[3], int ndim, const double inv12h[3], double dV,
                       double* partials, int nparts, double* out, hipStream_t s);

}  // namespace atns
