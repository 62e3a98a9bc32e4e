// Small kernels: the per-step delay draw, the ring fill of a given state, and
// the FP64 diagnostics (conserved totals, kinetic energy, enstrophy).
#include <mutex>

#include "kernels_common.hpp"
#include "launch.hpp"

namespace atns {

// Delays of step n for every (block, slot): the rule above, or the injected
// value (guarded the same way).
__global__ void delays_kernel(int8_t* out, const int8_t* inject, long long n, int nblocks, int L, int C,
                              unsigned long long seed, int algo, const long long* nstep) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nblocks * kNumSlots) return;
  if (nstep) n = *nstep;
  out[i] = (int8_t)(inject ? guard_delay(inject[i], n, L, C) : draw_delay(n, i, nblocks, L, seed, algo, C));
}

hipError_t launch_delays(int8_t* out, const int8_t* inject, long long n, int nblocks, int L, int C,
                         unsigned long long seed, int algo, hipStream_t s, const long long* nstep) {
  const int cnt = nblocks * kNumSlots;
  delays_kernel<<<(cnt + 255) / 256, 256, 0, s>>>(out, inject, n, nblocks, L, C, seed, algo, nstep);
  return hipGetLastError();
}

// Device step counters of graph-captured steps.
__global__ void step_set_kernel(long long* nstep, long long value) { *nstep = value; }
__global__ void step_inc_kernel(long long* const* counters, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) *counters[i] += 1;
}
hipError_t launch_step_set(long long* nstep, long long value, hipStream_t s) {
  step_set_kernel<<<1, 1, 0, s>>>(nstep, value);
  return hipGetLastError();
}
hipError_t launch_step_inc(long long* const* counters, int n, hipStream_t s) {
  step_inc_kernel<<<(n + 63) / 64, 64, 0, s>>>(counters, n);
  return hipGetLastError();
}

// Stage halos of one step.  For every halo point of every block and every
// variable: read the C delayed levels U^{n-k-l} of the neighbour's boundary
// layer from the ring, and write the s stage values
//   Uhat^(e) = sum_l W[e][k][l] U^{n-k-l}          (FP64 arithmetic)
// (AT: buffer extrapolation and RK-consistent updates, Eqs. 7-15; AS: the
// stale level itself).  One thread per point, consecutive threads on
// consecutive points of a region, so reads and writes are contiguous runs.
template <typename T, int S, int CL, bool STALE>
__global__ void __launch_bounds__(kHaloChunk)
    halo_kernel(const T* __restrict__ ring, T* __restrict__ halo, const HaloRegion* __restrict__ regions,
                const HaloWork* __restrict__ work, int8_t* __restrict__ delays,
                const double* __restrict__ W, long long slot_stride, long long halo_stride, int D,
                int slot_now, int L, const long long* nstep, DelayDraw dd) {
  long long n = 0;
  if (nstep) {
    n = *nstep;
    slot_now = (int)(n % D);
  }
  const HaloWork wk = work[blockIdx.x];
  const HaloRegion rg = regions[wk.region];
  int k;
  if (dd.draw) {
    // the step's delay of this region, drawn here (graph-captured steps);
    // the region's first chunk records it for the learned-halo correction
    k = draw_delay(n, rg.kidx, dd.nblocks, L, dd.seed, dd.algo, CL);
    if (wk.start == 0 && threadIdx.x == 0) delays[rg.kidx] = (int8_t)k;
  } else {
    k = delays[rg.kidx];
  }
  const int i = wk.start + threadIdx.x;
  if (i >= rg.npts) return;
  assemble_halo_point<T, S, CL, STALE>(ring, halo, rg, i, k, slot_now, D, W, L, slot_stride, halo_stride);
}

template <typename T>
hipError_t launch_halo(const T* ring, T* halo, const HaloRegion* regions, const HaloWork* work, int nwork,
                       int8_t* delays, const double* W, long long slot_stride, long long halo_stride,
                       int D, int slot_now, int L, int stages, bool stale, hipStream_t s,
                       const long long* nstep, DelayDraw dd) {
  dim3 grid(nwork), block(kHaloChunk);
#define ATNS_HALO(SS, CC, ST)                                                                               \
  halo_kernel<T, SS, CC, ST><<<grid, block, 0, s>>>(ring, halo, regions, work, delays, W, slot_stride, \
                                                     halo_stride, D, slot_now, L, nstep, dd)
  // the stage count identifies the scheme: RK4 and LSERK4 pair with AT4
  // (C = 5), LSERK2 with AT2 (C = 3)
  // (one more slot than stages: the filter's halo at the new level)
  if (stages == 4) {
    if (stale) ATNS_HALO(4, 5, true); else ATNS_HALO(4, 5, false);
  } else if (stages == 5) {
    if (stale) ATNS_HALO(5, 5, true); else ATNS_HALO(5, 5, false);
  } else if (stages == 6) {
    if (stale) ATNS_HALO(6, 5, true); else ATNS_HALO(6, 5, false);
  } else if (stages == 2) {
    if (stale) ATNS_HALO(2, 3, true); else ATNS_HALO(2, 3, false);
  } else if (stages == 3) {
    if (stale) ATNS_HALO(3, 3, true); else ATNS_HALO(3, 3, false);
  } else {
    return hipErrorInvalidValue;
  }
#undef ATNS_HALO
  return hipGetLastError();
}
template hipError_t launch_halo<float>(const float*, float*, const HaloRegion*, const HaloWork*, int, int8_t*,
                                       const double*, long long, long long, int, int, int, int, bool, hipStream_t,
                                       const long long*, DelayDraw);
template hipError_t launch_halo<double>(const double*, double*, const HaloRegion*, const HaloWork*, int, int8_t*,
                                        const double*, long long, long long, int, int, int, int, bool, hipStream_t,
                                        const long long*, DelayDraw);

// Copy the boundary layers of every block of field U into ring slot `slot`.
template <typename T>
__global__ void ring_fill_kernel(const StageParams<T> p, const T* U, int slot, const long long* nstep) {
  if (nstep) slot = (int)(*nstep % p.D);
  const int b = blockIdx.y;
  const BlockDev* B = p.blocks + b;
  const long long cnt = (long long)B->s[0] * B->s[1] * B->s[2];
  T* dst = p.ring + (long long)slot * p.slot_stride;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < cnt;
       i += (long long)gridDim.x * blockDim.x) {
    const int lx = (int)(i % B->s[0]);
    const int ly = (int)((i / B->s[0]) % B->s[1]);
    const int lz = (int)(i / ((long long)B->s[0] * B->s[1]));
    const long long g = ((long long)(B->o[2] + lz) * p.n[1] + (B->o[1] + ly)) * p.n[0] + (B->o[0] + lx);
    T u[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = U[v * p.field + g];
    ring_write_col(B, ring_column(B, p.H, lx, ly), p.H, true, lx, ly, lz, u, dst);
  }
}

template <typename T>
hipError_t launch_ring_fill(const StageParams<T>& p, const T* U, int slot, int nblocks, hipStream_t s,
                            const long long* nstep) {
  dim3 grid(64, nblocks), block(256);
  ring_fill_kernel<T><<<grid, block, 0, s>>>(p, U, slot, nstep);
  return hipGetLastError();
}
template hipError_t launch_ring_fill<float>(const StageParams<float>&, const float*, int, int, hipStream_t,
                                            const long long*);
template hipError_t launch_ring_fill<double>(const StageParams<double>&, const double*, int, int, hipStream_t,
                                             const long long*);

// ------------------------------------------------------------------ HBM probe
// Plain streaming copy, 16 bytes per lane per iteration: the achievable HBM
// bandwidth of the device, and the reference a byte-counter run is scaled by.
__global__ void __launch_bounds__(256) copy_probe_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                         long long n16) {
  // one 16-byte element per thread over an exact grid: the fastest plain
  // copy form measured on this device (grid-stride loops reach less)
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n16) dst[i] = src[i];
}

// Analytic initial fields, evaluated in FP64 and rounded to the state type.
// kind 0: isentropic vortex (uniform freestream of speed mach*sqrt(gamma)
// along the diagonal, Gaussian vortex of strength beta about (xc, yc) carried
// by it for time t, minimum-image distance on the periodic box);
// kind 1: Taylor-Green vortex (Sec. 5.2, Eq. 16, with the divergence-free sign
// of v and uniform initial temperature).
struct InitArgs {
  int n[3];
  double h[3], len[3];
  int kind, ndim;
  double gamma, mach, beta, t, xc, yc;
};

__device__ __forceinline__ double floor_mod(double a, double L) {
  double m = fmod(a, L);
  if (m < 0.0) m += L;
  return m;
}

template <typename T>
__global__ void init_case_kernel(T* __restrict__ U, InitArgs a, long long field) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= field) return;
  const int x = (int)(i % a.n[0]);
  const long long r = i / a.n[0];
  const int y = (int)(r % a.n[1]);
  const int z = (int)(r / a.n[1]);
  const double X = x * a.h[0], Y = y * a.h[1], Z = z * a.h[2];
  const double g = a.gamma;
  double rho, u, v, w, p;
  if (a.kind == 0) {
    const double speed = a.mach * sqrt(g);
    double ui[3];
    if (a.ndim == 2) {
      ui[0] = ui[1] = speed / sqrt(2.0);
      ui[2] = 0.0;
    } else {
      ui[0] = ui[1] = ui[2] = speed / sqrt(3.0);
    }
    const double xc = a.xc + ui[0] * a.t, yc = a.yc + ui[1] * a.t;
    const double dx = floor_mod(X - xc + 0.5 * a.len[0], a.len[0]) - 0.5 * a.len[0];
    const double dy = floor_mod(Y - yc + 0.5 * a.len[1], a.len[1]) - 0.5 * a.len[1];
    const double r2 = dx * dx + dy * dy;
    const double f = exp(0.5 * (1.0 - r2));
    const double pi = 3.14159265358979323846;
    u = ui[0] - a.beta / (2.0 * pi) * dy * f;
    v = ui[1] + a.beta / (2.0 * pi) * dx * f;
    w = ui[2];
    const double temp = 1.0 - (g - 1.0) * a.beta * a.beta * exp(1.0 - r2) / (8.0 * g * pi * pi);
    rho = pow(temp, 1.0 / (g - 1.0));
    p = rho * temp;
  } else {
    u = sin(X) * cos(Y) * cos(Z);
    v = -cos(X) * sin(Y) * cos(Z);
    w = 0.0;
    p = 1.0 / (g * a.mach * a.mach) + (cos(2.0 * X) + cos(2.0 * Y)) * (cos(2.0 * Z) + 2.0) / 16.0;
    rho = g * a.mach * a.mach * p;
  }
  const double et = p / (g - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
  U[i] = (T)rho;
  U[field + i] = (T)(rho * u);
  U[2 * field + i] = (T)(rho * v);
  U[3 * field + i] = (T)(rho * w);
  U[4 * field + i] = (T)et;
}

template <typename T>
hipError_t launch_init_case(T* U, const int n[3], const double h[3], const double len[3], int kind, int ndim,
                            double gamma, double mach, double beta, double t, double xc, double yc, hipStream_t s) {
  InitArgs a;
  for (int d = 0; d < 3; ++d) {
    a.n[d] = n[d];
    a.h[d] = h[d];
    a.len[d] = len[d];
  }
  a.kind = kind;
  a.ndim = ndim;
  a.gamma = gamma;
  a.mach = mach;
  a.beta = beta;
  a.t = t;
  a.xc = xc;
  a.yc = yc;
  const long long field = (long long)n[0] * n[1] * n[2];
  init_case_kernel<T><<<(unsigned)((field + 255) / 256), 256, 0, s>>>(U, a, field);
  return hipGetLastError();
}
template hipError_t launch_init_case<float>(float*, const int*, const double*, const double*, int, int, double, double,
                                            double, double, double, double, hipStream_t);
template hipError_t launch_init_case<double>(double*, const int*, const double*, const double*, int, int, double,
                                             double, double, double, double, double, hipStream_t);

hipError_t launch_copy_probe(const void* src, void* dst, long long bytes, hipStream_t s) {
  const long long n16 = bytes / 16;
  copy_probe_kernel<<<(unsigned)((n16 + 255) / 256), 256, 0, s>>>((const float4*)src, (float4*)dst, n16);
  return hipGetLastError();
}

// ----------------------------------------------------------------- diagnostics
// Per-workgroup FP64 partial sums of: the five conserved variables, rho|u|^2
// and rho|w|^2 with w = curl u by CD4 on the periodic global field.
constexpr int kDiagThreads = 256;

template <typename T>
__device__ __forceinline__ void vel_at(const T* U, int field, int g, double vel[3]) {
  const double ir = 1.0 / (double)U[g];
  vel[0] = (double)U[field + g] * ir;
  vel[1] = (double)U[2 * field + g] * ir;
  vel[2] = (double)U[3 * field + g] * ir;
}

// Per-workgroup partial sums of the five conserved totals, rho |u|^2 and
// rho |omega|^2 (omega from CD4 velocity derivatives on the periodic global
// field), in FP64.  Grid-stride over the points in a fixed order, so the
// result does not depend on timing.  Indices are 32-bit (5 fields of a
// 512^3 grid stay below 2^31), and each thread walks its points with an
// incremental (x, y, z) instead of a division per point.
template <typename T>
__global__ void __launch_bounds__(kDiagThreads)
    diag_partial_kernel(const T* U, int nx, int ny, int nz, int ndim, double ihx, double ihy,
                        double ihz, double* partials) {
  const int plane = nx * ny;
  const int field = plane * nz;
  const int stride = gridDim.x * blockDim.x;
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  // (x, y, z) of g and of the stride (stride < field is not required)
  int x = g % nx, y = (g / nx) % ny, z = g / plane;
  const int dx = stride % nx, dy = (stride / nx) % ny, dz = stride / plane;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  const bool three = ndim == 3;
  for (; g < field; g += stride) {
    double u[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = (double)U[v * field + g];
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[v] += u[v];
    acc[5] += (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) / u[0];
    // CD4 velocity derivatives along each direction: dv[d][c] = d u_c / d x_d
    double dv[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d == 2 && !three) break;
      const int n = d == 0 ? nx : (d == 1 ? ny : nz);
      const int st = d == 0 ? 1 : (d == 1 ? nx : plane);
      const int c = d == 0 ? x : (d == 1 ? y : z);
      const double ih = d == 0 ? ihx : (d == 1 ? ihy : ihz);
      double vm2[3], vm1[3], vp1[3], vp2[3];
      vel_at(U, field, g + (wrap(c - 2, n) - c) * st, vm2);
      vel_at(U, field, g + (wrap(c - 1, n) - c) * st, vm1);
      vel_at(U, field, g + (wrap(c + 1, n) - c) * st, vp1);
      vel_at(U, field, g + (wrap(c + 2, n) - c) * st, vp2);
#pragma unroll
      for (int k = 0; k < 3; ++k) dv[d][k] = (8.0 * (vp1[k] - vm1[k]) - (vp2[k] - vm2[k])) * ih;
    }
    const double wx = dv[1][2] - dv[2][1];
    const double wy = dv[2][0] - dv[0][2];
    const double wz = dv[0][1] - dv[1][0];
    acc[6] += u[0] * (wx * wx + wy * wy + wz * wz);
    // advance (x, y, z) by the stride
    x += dx;
    int cy = 0;
    if (x >= nx) {
      x -= nx;
      cy = 1;
    }
    y += dy + cy;
    int cz = 0;
    while (y >= ny) {
      y -= ny;
      ++cz;
    }
    z += dz + cz;
  }
  // workgroup reduction in a fixed order
  __shared__ double red[7][kDiagThreads];
#pragma unroll
  for (int i = 0; i < 7; ++i) red[i][threadIdx.x] = acc[i];
  __syncthreads();
  for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int i = 0; i < 7; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 7) partials[blockIdx.x * 7 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(kDiagThreads)
    diag_final_kernel(const double* partials, int nparts, double dV, double inv_npts, double* out) {
  __shared__ double red[7][kDiagThreads];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nparts; b += blockDim.x)
#pragma unroll
    for (int i = 0; i < 7; ++i) acc[i] += partials[b * 7 + i];
#pragma unroll
  for (int i = 0; i < 7; ++i) red[i][threadIdx.x] = acc[i];
  __syncthreads();
  for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int i = 0; i < 7; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 5) out[threadIdx.x] = red[threadIdx.x][0] * dV;
  if (threadIdx.x == 5) out[5] = 0.5 * red[5][0] * inv_npts;
  if (threadIdx.x == 6) out[6] = 0.5 * red[6][0] * inv_npts;
}

template <typename T>
hipError_t launch_diag(const T* U, const int n[3], int ndim, const double inv12h[3], double dV,
                       double* partials, int nparts, double* out, hipStream_t s) {
  diag_partial_kernel<T><<<nparts, kDiagThreads, 0, s>>>(U, n[0], n[1], n[2], ndim, inv12h[0],
                                                         inv12h[1], inv12h[2], partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double npts = (double)n[0] * n[1] * n[2];
  diag_final_kernel<<<1, kDiagThreads, 0, s>>>(partials, nparts, dV, 1.0 / npts, out);
  return hipGetLastError();
}
template hipError_t launch_diag<float>(const float*, const int*, int, const double*, double, double*, int,
                                       double*, hipStream_t);
template hipError_t launch_diag<double>(const double*, const int*, int, const double*, double, double*, int,
                                        double*, hipStream_t);

// Diagnostics without allocation (atns_reduce_noalloc): the workgroup
// partials go to `scratch`, a fixed device array that each GPU holds for the
// life of the process.  Host code never uses the array's name as an address:
// the first call on a device, with that device current, resolves the array's
// device address there (hipGetSymbolAddress) and keeps it per device.  Every
// call fully rewrites the partials it reads, so nothing is cleared; calls that
// overlap on one GPU share the array and race.
static __device__ __align__(256) double scratch[kDiagMaxParts * 7];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t diag_scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

template <typename T>
hipError_t launch_diag_noalloc(const T* U, const int n[3], int ndim, const double inv12h[3], double dV,
                               double* out, hipStream_t s) {
  double* part = nullptr;
  const hipError_t e = diag_scratch_address(&part);
  if (e != hipSuccess) return e;
  return launch_diag<T>(U, n, ndim, inv12h, dV, part, kDiagMaxParts, out, s);
}
template hipError_t launch_diag_noalloc<float>(const float*, const int*, int, const double*, double, double*,
                                               hipStream_t);
template hipError_t launch_diag_noalloc<double>(const double*, const int*, int, const double*, double, double*,
                                                hipStream_t);

}  // namespace atns
