// Fused Euler right-hand side + RK stage kernel.
//
// R = -(D_x F + D_y G + D_z H) with the explicit CD4 derivative
// (Eq. 2 with a = 4/3, b = -1/3: D phi_i = [8(phi_{i+1} - phi_{i-1})
// - (phi_{i+2} - phi_{i-2})] / (12 h)) of the inviscid fluxes of App. A on a
// Cartesian grid, followed in the same kernel by the RK update of the stage
// (Eq. 3 / classical RK4) and, in the last stage, by the write of the new
// boundary layers into the delayed-level ring.
//
// Work decomposition (2.5D): a workgroup owns a TX x TY column tile of one
// block and walks it along z.  Each thread keeps the state of planes
// z..z+2 of its column and the z-fluxes of planes z-2..z+2 (each computed
// once, when its plane arrives) in registers; the x- and y-fluxes of the current
// plane (tile plus a 2-point apron) are staged in LDS, double-buffered so one
// barrier per plane suffices.  Points outside the block -- the apron at a
// block face and the z-levels beyond it -- come from fetch(), which applies
// the halo rule of the stage (synchronous, stale, or AT-weighted levels).
#include "euler_flux.hpp"
#include "kernels_common.hpp"

namespace atns {


// LDS of a tile: the block descriptor and the x/y flux planes.  One object
// per (T, TX, TY), shared by every stage kind a kernel instantiates.
template <typename T, int TX, int TY>
struct EulerLds {
  BlockDev B;
  T F[2][5][TY][TX + 4];
  T G[2][5][TY + 4][TX];
};
template <typename T, int TX, int TY>
__device__ __forceinline__ EulerLds<T, TX, TY>& euler_lds() {
  __shared__ EulerLds<T, TX, TY> s;
  return s;
}

// FUSE: the kernel may assemble the step's halos in its first stage (the
// per-launch stage kernels); the batch and free-running kernels never do.
template <typename T, int TX, int TY, int KIND, bool FUSE = false, bool COMP = false>
__device__ __forceinline__ void euler_tile(const StageParams<T>& p, const TileDev t) {
  // every apron point (4 per tile row and column) has a thread of its own
  static_assert(4 * (TX + TY) <= TX * TY, "tile shape too narrow for its apron");
  if (t.nx == 0) return;
  // The block descriptor lives in LDS for the whole kernel: re-reading it from
  // global memory inside the plane loop would make every such load wait for
  // all outstanding (prefetch) loads.
  EulerLds<T, TX, TY>& lds = euler_lds<T, TX, TY>();
  stage_block(p.blocks + t.blk, &lds.B);
  const BlockDev* __restrict__ B = &lds.B;
  if constexpr (FUSE && (KIND == kRK4First || KIND == kLSFirst)) {
    // graph-captured steps with fused halo assembly: this tile's halo values
    // of every stage, before they are read (the condition is uniform)
    if (p.fuse_halo && p.nstep && p.halo != kHaloSync) fused_first_stage_halos(p, B, t);
  }
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const bool act = (tx < t.nx) && (ty < t.ny);
  const int lx = t.x0 + tx, ly = t.y0 + ty;
  const bool three = (p.ndim == 3);
  const T gm1 = (T)(p.gamma - 1.0);
  const T ihx = (T)p.dscale[0], ihy = (T)p.dscale[1], ihz = (T)p.dscale[2];
  // central-difference weights of the inner and outer neighbour pairs
  const T w1 = p.cd2 ? T(1) : T(8), w2 = p.cd2 ? T(0) : T(1);

  auto& sF = lds.F;
  auto& sG = lds.G;

  // Apron role: x-apron columns {-2,-1,nx,nx+1} x ny rows, then the y-apron.
  const int nxa = 4 * t.ny, nya = 4 * t.nx;
  int arole = 0, ax = 0, ay = 0;
  if (tid < nxa) {
    const int code = tid / t.ny;
    ay = tid % t.ny;
    ax = (code < 2) ? code - 2 : t.nx + code - 2;
    arole = 1;
  } else if (tid < nxa + nya) {
    const int b = tid - nxa;
    const int code = b / t.nx;
    ax = b % t.nx;
    ay = (code < 2) ? code - 2 : t.ny + code - 2;
    arole = 2;
  }

  // each thread's column(s) resolved once: its own, and its apron column
  ColumnSource<T> colq{}, cola{};
  if (act) colq = column_source(p, B, lx, ly);
  if (arole) cola = column_source(p, B, t.x0 + ax, t.y0 + ay);

  // z-queues of the own column: the state of planes lz..lz+2 (the centre
  // and the two planes behind it) and the z-fluxes of planes lz-2..lz+2, each
  // computed once, when its plane arrives
  T uq[3][5], hq[5][5];
  T nq[5], nq2[5], na[5];   // prefetched: own column at z+2, z+3 and the apron point at z
  if (act && three) {
    T u[5];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      fetch_col(p, B, colq, t.blk, lx, ly, t.z0 - 2 + j, u);
      euler_flux(u, 2, gm1, hq[j + 1]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      fetch_col(p, B, colq, t.blk, lx, ly, t.z0 + j, uq[j + 1]);
      euler_flux(uq[j + 1], 2, gm1, hq[j + 3]);
    }
    fetch_col(p, B, colq, t.blk, lx, ly, t.z0 + 2, nq);
    if (t.nz > 1) fetch_col(p, B, colq, t.blk, lx, ly, t.z0 + 3, nq2);
  }
  if (arole) fetch_col(p, B, cola, t.blk, t.x0 + ax, t.y0 + ay, t.z0, na);

  T* ring_slot = nullptr;
  RingColumn rcol{};
  if (p.ring_write) {
    ring_slot = p.ring + (long long)((p.slot_now + 1) % p.D) * p.slot_stride;
    if (act) rcol = ring_column(B, p.H, lx, ly);
  }

  // global index of the thread's column at plane z0, and the stride per plane
  const long long g0 = ((long long)(B->o[2] + t.z0) * p.n[1] + (B->o[1] + ly)) * p.n[0] + (B->o[0] + lx);
  const long long gplane = (long long)p.n[0] * p.n[1];
  T accv[5], u0v[5];
  if (act) epilogue_load<T, KIND, COMP>(p, g0, accv, u0v);

  for (int iz = 0; iz < t.nz; ++iz) {
    const int lz = t.z0 + iz;
    const int buf = iz & 1;
    if (act) {
      if (three) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 5; ++v) hq[j][v] = hq[j + 1][v];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int v = 0; v < 5; ++v) uq[j][v] = uq[j + 1][v];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          uq[2][v] = nq[v];
          nq[v] = nq2[v];
        }
        euler_flux(uq[2], 2, gm1, hq[4]);
        // next plane's column value: in flight while this plane is computed
        if (iz + 2 < t.nz) fetch_col(p, B, colq, t.blk, lx, ly, lz + 4, nq2);
      } else {
        fetch_col(p, B, colq, t.blk, lx, ly, lz, uq[0]);
      }
      T f[5];
      euler_flux(uq[0], 0, gm1, f);
#pragma unroll
      for (int v = 0; v < 5; ++v) sF[buf][v][ty][tx + 2] = f[v];
      euler_flux(uq[0], 1, gm1, f);
#pragma unroll
      for (int v = 0; v < 5; ++v) sG[buf][v][ty + 2][tx] = f[v];
    }
    if (arole) {
      T u[5], f[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) u[v] = na[v];
      if (iz + 1 < t.nz) fetch_col(p, B, cola, t.blk, t.x0 + ax, t.y0 + ay, lz + 1, na);
      if (arole == 1) {
        euler_flux(u, 0, gm1, f);
#pragma unroll
        for (int v = 0; v < 5; ++v) sF[buf][v][ay][ax + 2] = f[v];
      } else {
        euler_flux(u, 1, gm1, f);
#pragma unroll
        for (int v = 0; v < 5; ++v) sG[buf][v][ay + 2][ax] = f[v];
      }
    }
    lds_barrier();
    if (act) {
      T R[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const T dx = (w1 * (sF[buf][v][ty][tx + 3] - sF[buf][v][ty][tx + 1]) -
                      w2 * (sF[buf][v][ty][tx + 4] - sF[buf][v][ty][tx])) * ihx;
        const T dy = (w1 * (sG[buf][v][ty + 3][tx] - sG[buf][v][ty + 1][tx]) -
                      w2 * (sG[buf][v][ty + 4][tx] - sG[buf][v][ty][tx])) * ihy;
        R[v] = -(dx + dy);
      }
      if (three) {
#pragma unroll
        for (int v = 0; v < 5; ++v)
          R[v] -= (w1 * (hq[3][v] - hq[1][v]) - w2 * (hq[4][v] - hq[0][v])) * ihz;
      }
      const long long g = g0 + iz * gplane;
      T out[5];
      epilogue_pre<T, KIND, COMP>(p, g, uq[0], R, accv, u0v, out);
      if (iz + 1 < t.nz) epilogue_load<T, KIND, COMP>(p, g + gplane, accv, u0v);
      if (ring_slot) ring_write_col(B, rcol, p.H, true, lx, ly, lz, out, ring_slot);
    }
  }
}

template <typename T, int TX, int TY, int KIND, bool COMP = false>
__global__ void __launch_bounds__(TX* TY) euler_stage_kernel(const StageParams<T> p) {
  const StageParams<T> q = resolve_step(p);
  euler_tile<T, TX, TY, KIND, true, COMP>(q, p.tiles[blockIdx.x]);
  if (p.step_end) finish_step(p.step_end, p.done);
}

// Persistent form for a batch: every workgroup walks the combined tile list
// of all members (grid stride); the member's parameters are staged in LDS.
template <typename T, int TX, int TY, int KIND>
__global__ void __launch_bounds__(TX* TY)
    euler_batch_kernel(const StageParams<T>* __restrict__ ps, const BatchTile* __restrict__ tl, int ntiles) {
  __shared__ StageParams<T> sp;
  for (int i = blockIdx.x; i < ntiles; i += gridDim.x) {
    const BatchTile bt = tl[i];
    __syncthreads();
    stage_struct(ps + bt.inst, &sp);
    if (threadIdx.x == 0 && sp.nstep) sp = resolve_step(sp);
    __syncthreads();
    euler_tile<T, TX, TY, KIND>(sp, bt.t);
  }
}

// Free-running asynchronous steps of an Euler context (see async_run).
template <typename T, int TX, int TY, int S, int CL>
__global__ void __launch_bounds__(TX* TY)
    euler_async_kernel(const StageParams<T>* __restrict__ ps, const AsyncArgs a) {
  __shared__ StageParams<T> sp;
  async_run<T, S, CL>(ps, a, sp, [](const StageParams<T>& q, const TileDev& td, int e) {
    if constexpr (S == 2) {
      if (e == 0)
        euler_tile<T, TX, TY, kLSFirst>(q, td);
      else
        euler_tile<T, TX, TY, kLSMid>(q, td);
    } else {
      if (e == 0)
        euler_tile<T, TX, TY, kRK4First>(q, td);
      else if (e == S - 1)
        euler_tile<T, TX, TY, kRK4Last>(q, td);
      else
        euler_tile<T, TX, TY, kRK4Mid>(q, td);
    }
  });
}

template <typename T, int TX, int TY>
hipError_t launch_euler_async_shape(const StageParams<T>* ps, const AsyncArgs& a, int stages, hipStream_t s,
                                    int* resident) {
  const void* fn = stages == 2 ? (const void*)euler_async_kernel<T, TX, TY, 2, 3>
                               : (const void*)euler_async_kernel<T, TX, TY, 4, 5>;
  if (resident) return hipOccupancyMaxActiveBlocksPerMultiprocessor(resident, fn, TX * TY, 0);
  dim3 g(a.nb), b(TX * TY);
  if (stages == 2)
    euler_async_kernel<T, TX, TY, 2, 3><<<g, b, 0, s>>>(ps, a);
  else
    euler_async_kernel<T, TX, TY, 4, 5><<<g, b, 0, s>>>(ps, a);
  return hipGetLastError();
}

// With resident != nullptr: only report how many workgroups of the kernel
// fit on one CU (nothing is launched).
template <typename T>
hipError_t launch_euler_async(const StageParams<T>* ps, const AsyncArgs& a, int stages, int tx, int ty,
                              hipStream_t s, int* resident) {
  if (stages != 2 && stages != 4) return hipErrorInvalidValue;
  if (tx == 16 && ty == 16) return launch_euler_async_shape<T, 16, 16>(ps, a, stages, s, resident);
  if (tx == 32 && ty == 8) return launch_euler_async_shape<T, 32, 8>(ps, a, stages, s, resident);
  if (tx == 16 && ty == 8) return launch_euler_async_shape<T, 16, 8>(ps, a, stages, s, resident);
  if (tx == 64 && ty == 8) return launch_euler_async_shape<T, 64, 8>(ps, a, stages, s, resident);
  if (tx == 32 && ty == 16) return launch_euler_async_shape<T, 32, 16>(ps, a, stages, s, resident);
  return hipErrorInvalidValue;
}
template hipError_t launch_euler_async<float>(const StageParams<float>*, const AsyncArgs&, int, int, int, hipStream_t,
                                              int*);
template hipError_t launch_euler_async<double>(const StageParams<double>*, const AsyncArgs&, int, int, int,
                                               hipStream_t, int*);

template <typename T, int TX, int TY>
hipError_t launch_euler_batch_shape(const StageParams<T>* ps, const BatchTile* tl, int ntiles, int grid, int kind,
                                    hipStream_t s, int* resident) {
  if (resident) {   // the least over the three stage kinds
    const void* fns[3] = {(const void*)euler_batch_kernel<T, TX, TY, kRK4First>, (const void*)euler_batch_kernel<T, TX, TY, kRK4Mid>,
                          (const void*)euler_batch_kernel<T, TX, TY, kRK4Last>};
    int least = 1 << 30;
    for (const void* f : fns) {
      int r = 0;
      const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, f, TX * TY, 0);
      if (e != hipSuccess) return e;
      least = r < least ? r : least;
    }
    *resident = least;
    return hipSuccess;
  }
  dim3 g(grid), b(TX * TY);
  switch (kind) {
    case kRK4First: euler_batch_kernel<T, TX, TY, kRK4First><<<g, b, 0, s>>>(ps, tl, ntiles); break;
    case kRK4Mid: euler_batch_kernel<T, TX, TY, kRK4Mid><<<g, b, 0, s>>>(ps, tl, ntiles); break;
    case kRK4Last: euler_batch_kernel<T, TX, TY, kRK4Last><<<g, b, 0, s>>>(ps, tl, ntiles); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// With resident != nullptr: only report how many workgroups of the kernel
// fit on one CU (the least over its stage kinds).
template <typename T>
hipError_t launch_euler_batch(const StageParams<T>* ps, const BatchTile* tl, int ntiles, int grid, int kind, int tx,
                              int ty, hipStream_t s, int* resident) {
  if (tx == 16 && ty == 16) return launch_euler_batch_shape<T, 16, 16>(ps, tl, ntiles, grid, kind, s, resident);
  if (tx == 32 && ty == 8) return launch_euler_batch_shape<T, 32, 8>(ps, tl, ntiles, grid, kind, s, resident);
  if (tx == 16 && ty == 8) return launch_euler_batch_shape<T, 16, 8>(ps, tl, ntiles, grid, kind, s, resident);
  if (tx == 64 && ty == 8) return launch_euler_batch_shape<T, 64, 8>(ps, tl, ntiles, grid, kind, s, resident);
  if (tx == 32 && ty == 16) return launch_euler_batch_shape<T, 32, 16>(ps, tl, ntiles, grid, kind, s, resident);
  return hipErrorInvalidValue;
}
template hipError_t launch_euler_batch<float>(const StageParams<float>*, const BatchTile*, int, int, int, int, int,
                                              hipStream_t, int*);
template hipError_t launch_euler_batch<double>(const StageParams<double>*, const BatchTile*, int, int, int, int, int,
                                               hipStream_t, int*);

template <typename T, int TX, int TY>
hipError_t launch_euler_shape(const StageParams<T>& p, int ntiles, int kind, hipStream_t s) {
  dim3 grid(ntiles), block(TX * TY);
  switch (kind) {
    case kRhsOnly: euler_stage_kernel<T, TX, TY, kRhsOnly><<<grid, block, 0, s>>>(p); break;
    case kRK4First: euler_stage_kernel<T, TX, TY, kRK4First><<<grid, block, 0, s>>>(p); break;
    case kRK4Mid: euler_stage_kernel<T, TX, TY, kRK4Mid><<<grid, block, 0, s>>>(p); break;
    case kRK4Last:
      if (p.comp)
        euler_stage_kernel<T, TX, TY, kRK4Last, true><<<grid, block, 0, s>>>(p);
      else
        euler_stage_kernel<T, TX, TY, kRK4Last><<<grid, block, 0, s>>>(p);
      break;
    case kLSFirst: euler_stage_kernel<T, TX, TY, kLSFirst><<<grid, block, 0, s>>>(p); break;
    default: euler_stage_kernel<T, TX, TY, kLSMid><<<grid, block, 0, s>>>(p); break;
  }
  return hipGetLastError();
}

// Tile shapes (TX x TY) the Euler kernel is built for.
template <typename T>
hipError_t launch_euler_stage(const StageParams<T>& p, int ntiles, int kind, int tx, int ty, hipStream_t s) {
  if (tx == 16 && ty == 16) return launch_euler_shape<T, 16, 16>(p, ntiles, kind, s);
  if (tx == 32 && ty == 8) return launch_euler_shape<T, 32, 8>(p, ntiles, kind, s);
  if (tx == 16 && ty == 8) return launch_euler_shape<T, 16, 8>(p, ntiles, kind, s);
  if (tx == 64 && ty == 8) return launch_euler_shape<T, 64, 8>(p, ntiles, kind, s);
  if (tx == 32 && ty == 16) return launch_euler_shape<T, 32, 16>(p, ntiles, kind, s);
  return hipErrorInvalidValue;
}

template hipError_t launch_euler_stage<float>(const StageParams<float>&, int, int, int, int, hipStream_t);
template hipError_t launch_euler_stage<double>(const StageParams<double>&, int, int, int, int, hipStream_t);

}  // namespace atns
