// Kernel launchers (defined in the .hip files).
#pragma once
#include <hip/hip_runtime.h>

#include "layout.hpp"

namespace atns {

// Free-running asynchronous steps (one persistent workgroup per block) of a
// 3-D Navier-Stokes or an Euler context; with resident set, only the number
// of workgroups that fit on one CU is returned.
// Two consecutive classical RK4 stages of a 3-D Euler context in one pass
// (pair 0: stages 1-2 with the parameters of stages 0 and 1; pair 1: stages
// 3-4), single precision.
template <typename T>
hipError_t launch_euler_pair(const StageParams<T>& pA, const StageParams<T>& pB, int ntiles, int pair, int tx,
                             int ty, hipStream_t s);
template <typename T>
hipError_t launch_ns_async(const StageParams<T>* ps, const AsyncArgs& a, int stages, int tx, int ty, hipStream_t s,
                           int* resident = nullptr);
template <typename T>
hipError_t launch_euler_async(const StageParams<T>* ps, const AsyncArgs& a, int stages, int tx, int ty,
                              hipStream_t s, int* resident = nullptr);
template <typename T>
hipError_t launch_euler_stage(const StageParams<T>& p, int ntiles, int kind, int tx, int ty, hipStream_t s);
template <typename T>
hipError_t launch_ns_stage(const StageParams<T>& p, int ntiles, int kind, int tx, int ty, hipStream_t s);

template <typename T>
hipError_t launch_euler_batch(const StageParams<T>* ps, const BatchTile* tl, int ntiles, int grid, int kind, int tx,
                              int ty, hipStream_t s, int* resident = nullptr);
template <typename T>
hipError_t launch_ns_batch(const StageParams<T>* ps, const BatchTile* tl, int ntiles, int grid, int kind, int tx,
                           int ty, hipStream_t s, int* resident = nullptr);
hipError_t launch_step_set(long long* nstep, long long value, hipStream_t s);
hipError_t launch_step_inc(long long* const* counters, int n, hipStream_t s);

template <typename T>
hipError_t launch_halo(const T* ring, T* halo, const HaloRegion* regions, const HaloWork* work, int nwork,
                       int8_t* delays, const double* W, long long slot_stride, long long halo_stride,
                       int D, int slot_now, int L, int stages, bool stale, hipStream_t s,
                       const long long* nstep = nullptr, DelayDraw dd = DelayDraw{0, 0, 0, 0ull});
template <typename T>
hipError_t launch_init_case(T* U, const int n[3], const double h[3], const double len[3], int kind, int ndim,
                            double gamma, double mach, double beta, double t, double xc, double yc, hipStream_t s);
hipError_t launch_copy_probe(const void* src, void* dst, long long bytes, hipStream_t s);
hipError_t launch_delays(int8_t* out, const int8_t* inject, long long n, int nblocks, int L, int C,
                         unsigned long long seed, int algo, hipStream_t s, const long long* nstep = nullptr);
// nstep set (graph-captured steps): the slot is *nstep mod D instead.
template <typename T>
hipError_t launch_ring_fill(const StageParams<T>& p, const T* U, int slot, int nblocks, hipStream_t s,
                            const long long* nstep = nullptr);
// One pass of the block-local filter along axis f.dir: max_lines, the most
// lines of one block along the axis; min_len and max_len, the shortest and
// longest block side along it (at most kFilterMaxLen).  Blocks of one common
// side of 8, 16 or 32 take a register-only kernel; otherwise the launch's
// LDS holds max_len x 64 doubles.
constexpr int kFilterMaxLen = 256;
inline bool filter_pass_fixed(int min_len, int max_len) {
  return min_len == max_len && (max_len == 8 || max_len == 16 || max_len == 32);
}
template <typename T>
hipError_t launch_filter_pass(const FilterArgs<T>& f, int nblocks, int max_lines, int min_len, int max_len,
                              hipStream_t s);
// All three passes of a step with delayed halos in one launch, and the ring
// write of the filtered field: 3-D blocks that are all cubes of side 8, 16 or
// 32 (16 at most in double precision).  Synchronous steps, whose y and z
// passes read the neighbours' values of the pass before, take the per-axis
// passes (with f.nstep the kernel checks, and returns on such a step).
inline bool filter_fused_fits(int side, int esz) {
  return (side == 8 || side == 16 || side == 32) && (esz == 4 || side <= 16);
}
template <typename T>
hipError_t launch_filter_fused(const FilterArgs<T>& f, int nblocks, int side, hipStream_t s);
// Workgroups (and FP64 partial sets of 7) of the diagnostics reduction; the
// allocation-free form keeps its partials in a fixed device array of this size.
constexpr int kDiagMaxParts = 1024;
template <typename T>
hipError_t launch_diag_noalloc(const T* U, const int n[3], int ndim, const double inv12h[3], double dV,
                               double* out, hipStream_t s);
template <typename T>
hipError_t launch_diag(const T* U, const int n[3], int ndim, const double inv12h[3], double dV,
                       double* partials, int nparts, double* out, hipStream_t s);

}  // namespace atns
