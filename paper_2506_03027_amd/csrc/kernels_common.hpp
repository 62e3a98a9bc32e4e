// Device helpers shared by the stage kernels: halo-aware point fetch, the
// ring write and the RK epilogues.
#pragma once
#include <hip/hip_runtime.h>

#include "layout.hpp"

namespace atns {

constexpr int kLevels = 5;  // AT4: C = 5 (the learned halo works on AT4)

// Workgroup barrier that orders LDS only: finish this wave's LDS operations,
// then meet at s_barrier.  Unlike __syncthreads() it does not wait for
// outstanding global loads, so loads issued for the next plane stay in
// flight across the barrier (the compiler still waits before their use).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ int wrap(int g, int n) {
  g += (g < 0) ? n : 0;
  g -= (g >= n) ? n : 0;
  return g;
}

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output i of the stream
// seeded with `seed` is mix(seed + (i + 1) * golden).
__device__ __forceinline__ unsigned long long sm64(unsigned long long seed, unsigned long long i) {
  unsigned long long z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Alg. 3 guard: delays beyond L-1 or beyond the available history are 0.
__device__ __forceinline__ int guard_delay(long long k, long long n, int L, int C) {
  return (k < 0 || k > L - 1 || k > n - C + 1) ? 0 : (int)k;
}

// Delay of step n (n >= C) for (block, slot) index i = b * 18 + slot:
// CAA (n - C) mod L, SAA SplitMix64 draw mod L; then the guard.
// x mod L for a small L (1 <= L <= 16) from 32-bit pieces: with
// x = hi 2^32 + lo, x mod L = ((hi mod L)(2^32 mod L) + lo mod L) mod L,
// the same value as the 64-bit remainder, at 32-bit cost.
__device__ __forceinline__ unsigned mod_small(unsigned long long x, unsigned L) {
  const unsigned hi = (unsigned)(x >> 32), lo = (unsigned)x;
  const unsigned p32 = (unsigned)((1ull << 32) % L);
  return ((hi % L) * p32 + lo % L) % L;
}

__device__ __forceinline__ int draw_delay(long long n, int i, int nblocks, int L, unsigned long long seed, int algo,
                                          int C) {
  if (n < C) return 0;   // synchronous steps (not drawn)
  long long k;
  if (algo == 0) {
    k = mod_small((unsigned long long)(n - C), (unsigned)L);
  } else {
    const unsigned long long draw = (unsigned long long)n * (unsigned long long)nblocks * kNumSlots + i;
    k = mod_small(sm64(seed, draw), (unsigned)L);
  }
  return guard_delay(k, n, L, C);
}

// Stage halos of one halo point i of region rg for delay k (Eq. 7 with
// Eqs. 8-15): read the C delayed levels U^{n-k-l} of the neighbour's layer
// from the ring (slots slot_now - k - l mod D) and write the S stage values
//   Uhat^(e) = sum_l W[e][k][l] U^{n-k-l}   (FP64 arithmetic; AT)
// or the stale level itself (AS, STALE).
template <typename T, int S, int CL, bool STALE>
__device__ __forceinline__ void assemble_halo_point(const T* __restrict__ ring, T* __restrict__ halo,
                                                    const HaloRegion& rg, int i, int k, int slot_now, int D,
                                                    const double* __restrict__ W, int L, long long slot_stride,
                                                    long long halo_stride) {
  int sl[CL];
#pragma unroll
  for (int l = 0; l < CL; ++l) {
    int q = slot_now - k - l;
    sl[l] = q + ((q < 0) ? D : 0);
  }
  for (int v = 0; v < 5; ++v) {
    const long long so = rg.src + (long long)v * rg.npts + i;
    const long long dof = rg.dst + (long long)v * rg.npts + i;
    if (STALE) {
      const T x = ring[(long long)sl[0] * slot_stride + so];
#pragma unroll
      for (int e = 0; e < S; ++e) halo[e * halo_stride + dof] = x;
      continue;
    }
    double lev[CL];
#pragma unroll
    for (int l = 0; l < CL; ++l) lev[l] = (double)ring[(long long)sl[l] * slot_stride + so];
#pragma unroll
    for (int e = 0; e < S; ++e) {
      const double* w = W + ((long long)e * L + k) * CL;
      double a = 0.0;
#pragma unroll
      for (int l = 0; l < CL; ++l) a = fma(w[l], lev[l], a);
      halo[e * halo_stride + dof] = (T)a;
    }
  }
}

// Halo values of the first stage of a step with fused halo assembly: every
// halo point a tile's plane loop reads gets its S stage values, by the
// arithmetic of halo_kernel (assemble_halo_point), written to the stage-halo
// buffers (stage e at hbuf + e * slot_stride).  The Euler tile reads a
// 2-point apron: along x the columns x0-2 .. x0+nx+1 at its rows and planes,
// along y likewise, and along z its own columns at planes z0-2 .. z0+nz+1
// (3-D); the parts of these ranges beyond a block face are that face's halo
// points.  A point read by two tiles (next to a tile thinner than the apron)
// is written by both with the same bits.  Ends with a workgroup barrier,
// after which the tile reads the values.
template <typename T, int S, int CL, bool STALE>
__device__ void assemble_tile_halos(const StageParams<T>& p, const BlockDev* __restrict__ B, const TileDev& t,
                                    long long n) {
  constexpr int A = 2;   // apron width of the Euler tile
  T* hb = const_cast<T*>(p.hbuf);
  const int H = p.H;
  const int lo[3] = {t.x0, t.y0, t.z0};
  const int len[3] = {t.nx, t.ny, t.nz};
  for (int f = 0; f < 6; ++f) {
    if (B->hoff[f] < 0) continue;
    const int ax = f >> 1;
    const int r0 = lo[ax] - A, r1 = lo[ax] + len[ax] + A;   // read range along the face normal
    int a0, a1;                                              // its part beyond the face, layer-local
    if (f & 1) {
      a0 = (r0 > B->s[ax] ? r0 : B->s[ax]) - B->s[ax];
      a1 = r1 - B->s[ax];
    } else {
      a0 = r0 + H;
      a1 = (r1 < 0 ? r1 : 0) + H;
    }
    a0 = a0 > 0 ? a0 : 0;
    a1 = a1 < H ? a1 : H;
    if (a1 <= a0) continue;
    int e0[3], c0[3], b0[3];   // region extents; this tile's box in it and the box origin
    for (int d = 0; d < 3; ++d) {
      e0[d] = d == ax ? H : B->s[d];
      c0[d] = d == ax ? a1 - a0 : len[d];
      b0[d] = d == ax ? a0 : lo[d];
    }
    HaloRegion rg;
    rg.dst = B->hoff[f];
    rg.src = B->roff[f];
    rg.npts = e0[0] * e0[1] * e0[2];
    const int k = draw_delay(n, t.blk * kNumSlots + f, p.dd.nblocks, p.L, p.dd.seed, p.dd.algo, CL);
    const int cnt = c0[0] * c0[1] * c0[2];
    for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
      const int ix = b0[0] + j % c0[0];
      const int iy = b0[1] + (j / c0[0]) % c0[1];
      const int iz = b0[2] + j / (c0[0] * c0[1]);
      const int li = (iz * e0[1] + iy) * e0[0] + ix;
      assemble_halo_point<T, S, CL, STALE>(p.ring, hb, rg, li, k, p.slot_now, p.D, p.W, p.L, p.slot_stride,
                                           p.slot_stride);
    }
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ void fused_first_stage_halos(const StageParams<T>& p, const BlockDev* __restrict__ B,
                                                        const TileDev& t) {
  const long long n = *p.nstep;
  const bool stale = p.halo == kHaloStale;
  if (p.S == 4) {
    if (stale) assemble_tile_halos<T, 4, 5, true>(p, B, t, n); else assemble_tile_halos<T, 4, 5, false>(p, B, t, n);
  } else if (p.S == 5) {
    if (stale) assemble_tile_halos<T, 5, 5, true>(p, B, t, n); else assemble_tile_halos<T, 5, 5, false>(p, B, t, n);
  } else {
    if (stale) assemble_tile_halos<T, 2, 3, true>(p, B, t, n); else assemble_tile_halos<T, 2, 3, false>(p, B, t, n);
  }
}

// Stage parameters with the step-dependent fields resolved from the device
// step counter when present.
template <typename T>
__device__ __forceinline__ StageParams<T> resolve_step(const StageParams<T>& p) {
  StageParams<T> q = p;
  if (p.nstep) {
    const long long n = *p.nstep;
    q.slot_now = p.D ? (int)(n % p.D) : 0;
    q.halo = (n >= p.C) ? p.async_halo : kHaloSync;
  }
  return q;
}

// End of a captured step: every workgroup of the last stage kernel counts
// itself done; the last one (all others have finished, so nobody reads the
// step counter any more in this launch) advances the counter and resets the
// done count for the next step.  No fence is needed: each workgroup read the
// counter before counting itself done, and the next kernel sees the new
// value at the kernel boundary.
__device__ __forceinline__ void finish_step(long long* step, unsigned int* done) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int prev = atomicAdd(done, 1u);
    if (prev == gridDim.x - 1) {
      *step += 1;
      *done = 0u;
    }
  }
}

// Copy a block descriptor into LDS (cooperatively, 32-bit words) and wait.
__device__ __forceinline__ void stage_block(const BlockDev* __restrict__ src, BlockDev* dst) {
  constexpr int nw = (int)(sizeof(BlockDev) / 4);
  const int* s = reinterpret_cast<const int*>(src);
  int* d = reinterpret_cast<int*>(dst);
  for (int i = threadIdx.x; i < nw; i += blockDim.x) d[i] = s[i];
  __syncthreads();
}

// Copy any 4-byte-multiple struct into LDS (cooperatively) and wait.
template <typename S>
__device__ __forceinline__ void stage_struct(const S* __restrict__ src, S* dst) {
  static_assert(sizeof(S) % 4 == 0, "struct size");
  constexpr int nw = (int)(sizeof(S) / 4);
  const int* s = reinterpret_cast<const int*>(src);
  int* d = reinterpret_cast<int*>(dst);
  for (int i = threadIdx.x; i < nw; i += blockDim.x) d[i] = s[i];
  __syncthreads();
}

// Conserved variables at block-local point (lx, ly, lz) of block B as seen by
// that block in the current stage:
//  * owned points, and every point under synchronous halos: the stage field
//    Y at the periodic global position;
//  * halo points (outside the block): the stage's halo value, assembled once
//    per step by halo_kernel (AT weights or the stale level) into a buffer
//    laid out like the neighbour's ring layer.
template <typename T>
__device__ __forceinline__ void fetch(const StageParams<T>& p, const BlockDev* __restrict__ B,
                                      int blk, int lx, int ly, int lz, T u[5]) {
  const int sx = (lx < 0) ? -1 : (lx >= B->s[0] ? 1 : 0);
  const int sy = (ly < 0) ? -1 : (ly >= B->s[1] ? 1 : 0);
  const int sz = (lz < 0) ? -1 : (lz >= B->s[2] ? 1 : 0);
  if (((sx | sy | sz) == 0) || p.halo == kHaloSync) {
    const int gx = wrap(B->o[0] + lx, p.n[0]);
    const int gy = wrap(B->o[1] + ly, p.n[1]);
    const int gz = wrap(B->o[2] + lz, p.n[2]);
    const long long g = ((long long)gz * p.n[1] + gy) * p.n[0] + gx;
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = p.Y[v * p.field + g];
    return;
  }
  const int s = slot_index(sx, sy, sz);
  const int dep = ((sx != 0) + (sy != 0) + (sz != 0) == 1) ? p.H : 2;
  const int ix = sx < 0 ? lx + dep : (sx > 0 ? lx - B->s[0] : lx);
  const int iy = sy < 0 ? ly + dep : (sy > 0 ? ly - B->s[1] : ly);
  const int iz = sz < 0 ? lz + dep : (sz > 0 ? lz - B->s[2] : lz);
  const int ex = sx ? dep : B->s[0];
  const int ey = sy ? dep : B->s[1];
  const int ez = sz ? dep : B->s[2];
  const long long li = ((long long)iz * ey + iy) * ex + ix;
  const long long vs = (long long)ex * ey * ez;
  const T* r = p.hbuf + B->hoff[s] + li;
#pragma unroll
  for (int v = 0; v < 5; ++v) u[v] = r[v * vs];
}

// Where the values of a column (fixed block-local lx, ly) come from for the
// planes 0 <= lz < s_z of its block: an affine address, plane lz at
// base + lz * zs and variable v at + v * vs.  Columns inside the block in x
// and y, and every column under synchronous halos, read the stage field; the
// others read the stage's halo region of their (x, y) slot.  Planes outside
// the block in z go through fetch()'s general rule.  Equal to fetch() value
// for value; it only hoists the column's address arithmetic out of the
// plane loop.
template <typename T>
struct ColumnSource {
  const T* base;
  long long vs;
  long long zs;
};

template <typename T>
__device__ __forceinline__ ColumnSource<T> column_source(const StageParams<T>& p, const BlockDev* __restrict__ B,
                                                        int lx, int ly) {
  ColumnSource<T> c;
  const int sx = (lx < 0) ? -1 : (lx >= B->s[0] ? 1 : 0);
  const int sy = (ly < 0) ? -1 : (ly >= B->s[1] ? 1 : 0);
  if (((sx | sy) == 0) || p.halo == kHaloSync) {
    const int gx = wrap(B->o[0] + lx, p.n[0]);
    const int gy = wrap(B->o[1] + ly, p.n[1]);
    const long long gplane = (long long)p.n[0] * p.n[1];
    c.base = p.Y + (long long)B->o[2] * gplane + (long long)gy * p.n[0] + gx;
    c.vs = p.field;
    c.zs = gplane;
  } else {
    const int s = slot_index(sx, sy, 0);
    const int dep = (sx != 0 && sy != 0) ? 2 : p.H;
    const int ix = sx < 0 ? lx + dep : (sx > 0 ? lx - B->s[0] : lx);
    const int iy = sy < 0 ? ly + dep : (sy > 0 ? ly - B->s[1] : ly);
    const int ex = sx ? dep : B->s[0];
    const int ey = sy ? dep : B->s[1];
    c.base = p.hbuf + B->hoff[s] + (long long)iy * ex + ix;
    c.zs = (long long)ex * ey;
    c.vs = c.zs * B->s[2];
  }
  return c;
}

template <typename T>
__device__ __forceinline__ void fetch_col(const StageParams<T>& p, const BlockDev* __restrict__ B,
                                          const ColumnSource<T>& c, int blk, int lx, int ly, int lz, T u[5]) {
  if (lz >= 0 && lz < B->s[2]) {
    const T* r = c.base + lz * c.zs;
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = r[v * c.vs];
  } else {
    fetch(p, B, blk, lx, ly, lz, u);
  }
}

// The boundary layers an owned column (lx, ly) of block B belongs to in its
// x and y conditions, resolved once per column: for the -x, +x, -y and +y
// faces and the xy edge, the column's offset in that layer at plane 0 (-1
// when the column is not in it).  A layer [ez][ey][ex] is stored
// contiguously per variable (layout.hpp); x-faces are [s_z][s_y][H], y-faces
// [s_z][H][s_x], xy edges [s_z][2][2].  Blocks narrower than 2H can put a
// column in both faces of one axis; edges are 2 deep and blocks at least H = 4
// wide, so a column is in at most one xy edge.
struct RingColumn {
  int off[5];   // -x face, +x face, -y face, +y face, xy edge
  int slot[5];  // their ring slots
};

__device__ __forceinline__ RingColumn ring_column(const BlockDev* __restrict__ B, int H, int lx, int ly) {
  RingColumn r;
  const int sx = B->s[0], sy = B->s[1];
  r.slot[0] = 0;
  r.slot[1] = 1;
  r.slot[2] = 2;
  r.slot[3] = 3;
  r.off[0] = (B->lay[0] >= 0 && lx < H) ? ly * H + lx : -1;
  r.off[1] = (B->lay[1] >= 0 && lx >= sx - H) ? ly * H + (lx - (sx - H)) : -1;
  r.off[2] = (B->lay[2] >= 0 && ly < H) ? ly * sx + lx : -1;
  r.off[3] = (B->lay[3] >= 0 && ly >= sy - H) ? (ly - (sy - H)) * sx + lx : -1;
  const int ex = lx < 2 ? 0 : (lx >= sx - 2 ? 1 : -1);
  const int ey = ly < 2 ? 0 : (ly >= sy - 2 ? 1 : -1);
  r.slot[4] = 6 + ex + 2 * ey;   // (+-x, +-y) edge slot
  const int ix = ex == 0 ? lx : lx - (sx - 2), iy = ey == 0 ? ly : ly - (sy - 2);
  r.off[4] = (ex >= 0 && ey >= 0 && B->lay[r.slot[4]] >= 0) ? iy * 2 + ix : -1;
  return r;
}

// Every boundary layer of block B in ring slot `slot` that contains owned
// point (lx, ly, lz): the column's x/y layers (rc) at plane lz, and, at the
// planes within H (faces) or 2 (edges) of a z face, the z-face layer and the
// xz and yz edge layers.  put(w, vs) receives the address of variable 0 of
// the point in one layer and the variable stride there.  lz is the plane of
// the whole workgroup (or a compile-time plane), so the z tests are
// uniform.  Readers find these values through the region offsets of
// layout.hpp (roff), so the layer layout here is the one build_layout()
// assigns.
template <typename T, typename F>
__device__ __forceinline__ void ring_visit(const BlockDev* __restrict__ B, const RingColumn& rc, int H, int lx,
                                           int ly, int lz, T* __restrict__ slot, F&& put) {
  const int sx = B->s[0], sy = B->s[1], sz = B->s[2];
  // x and y faces and the xy edge: the layer holds every plane of the block
  const int zs[5] = {sy * H, sy * H, H * sx, H * sx, 4};
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    if (rc.off[j] < 0) continue;
    put(slot + B->lay[rc.slot[j]] + lz * zs[j] + rc.off[j], zs[j] * sz);
  }
  // z faces and the xz / yz edges
  const int izf = lz < H ? lz : (lz >= sz - H ? lz - (sz - H) : -1);
  if (izf < 0) return;
  for (int side = 0; side < 2; ++side) {   // a block lower than 2H has planes in both
    const bool lo = side == 0;
    if (lo ? lz >= H : lz < sz - H) continue;
    const int s = lo ? 4 : 5;
    if (B->lay[s] >= 0) {
      const int iz = lo ? lz : lz - (sz - H);
      put(slot + B->lay[s] + (iz * sy + ly) * sx + lx, H * sy * sx);
    }
    if (lo ? lz >= 2 : lz < sz - 2) continue;
    const int iz2 = lo ? lz : lz - (sz - 2);
    const int ex = lx < 2 ? 0 : (lx >= sx - 2 ? 1 : -1);
    if (ex >= 0) {   // (+-x, +-z) edge, [2][s_y][2]
      const int se = 10 + ex + 2 * (lo ? 0 : 1);
      if (B->lay[se] >= 0) {
        const int ix = ex == 0 ? lx : lx - (sx - 2);
        put(slot + B->lay[se] + (iz2 * sy + ly) * 2 + ix, 4 * sy);
      }
    }
    const int ey = ly < 2 ? 0 : (ly >= sy - 2 ? 1 : -1);
    if (ey >= 0) {   // (+-y, +-z) edge, [2][2][s_x]
      const int se = 14 + ey + 2 * (lo ? 0 : 1);
      if (B->lay[se] >= 0) {
        const int iy = ey == 0 ? ly : ly - (sy - 2);
        put(slot + B->lay[se] + (iz2 * 2 + iy) * sx + lx, 4 * sx);
      }
    }
  }
}

// Write u[5], the new value of owned point (lx, ly, lz), into every ring
// layer that contains it.  act: the thread holds an owned point.
template <typename T>
__device__ __forceinline__ void ring_write_col(const BlockDev* __restrict__ B, const RingColumn& rc, int H,
                                               bool act, int lx, int ly, int lz, const T u[5],
                                               T* __restrict__ slot) {
  if (!act) return;
  ring_visit(B, rc, H, lx, ly, lz, slot, [&](T* w, int vs) {
#pragma unroll
    for (int v = 0; v < 5; ++v) w[v * vs] = u[v];
  });
}

// The same for one variable v of the point.
template <typename T>
__device__ __forceinline__ void ring_write_var(const BlockDev* __restrict__ B, const RingColumn& rc, int H, int lx,
                                               int ly, int lz, int v, T val, T* __restrict__ slot) {
  ring_visit(B, rc, H, lx, ly, lz, slot, [&](T* w, int vs) { w[v * vs] = val; });
}

// 1 / a: IEEE division in FP64; in FP32 the hardware reciprocal estimate
// refined by one Newton-Raphson step, r' = r + r (1 - a r).
template <typename T>
__device__ __forceinline__ T recip(T a) {
  return T(1) / a;
}
template <>
__device__ __forceinline__ float recip<float>(float a) {
  const float r = __builtin_amdgcn_rcpf(a);
  return fmaf(r, fmaf(-a, r, 1.0f), r);
}

// u0 + d with the rounding error of the sum carried in c across steps
// (Knuth's TwoSum on d + c): returns the new value and leaves in c the part
// of u0 + d + c that the returned value misses.
template <typename T>
__device__ __forceinline__ T comp_add(T u0, T d, T& c) {
#pragma clang fp contract(off)
  const T y = d + c;
  const T s = u0 + y;
  const T bb = s - u0;
  c = (u0 - (s - bb)) + (y - bb);
  return s;
}

// Operands the RK epilogue reads at a point besides the stage input: the
// accumulator / Q register and, for the middle RK4 stages and the compensated
// last one, U^n.  Loaded one plane ahead so their latency hides behind the
// stencil work.  COMP (compensated last RK4 stage, p.comp != null) is a
// template flag so that the plain last stage holds no registers for it.
template <typename T, int KIND, bool COMP = false>
__device__ __forceinline__ void epilogue_load(const StageParams<T>& p, long long g, T accv[5], T u0v[5]) {
  static_assert(!COMP || KIND == kRK4Last, "compensation is a last-RK4-stage variant");
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const long long i = v * p.field + g;
    if (KIND == kRK4Mid || KIND == kRK4Last || KIND == kLSMid) accv[v] = p.acc[i];
    if (KIND == kRK4Mid || COMP) u0v[v] = p.U0[i];
  }
}

// RK epilogue with preloaded operands (see epilogue_load).
template <typename T, int KIND, bool COMP = false>
__device__ __forceinline__ void epilogue_pre(const StageParams<T>& p, long long g, const T Y[5], const T R[5],
                                             const T accv[5], const T u0v[5], T out[5]) {
  const T dt = (T)p.dt, cA = (T)p.cA, cB = (T)p.cB;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const long long i = v * p.field + g;
    const T r = R[v];
    if (KIND == kRhsOnly) {
      out[v] = r;
    } else if (KIND == kRK4First) {
      const T dr = dt * r;
      p.acc[i] = cA * dr;
      out[v] = Y[v] + cB * dr;
    } else if (KIND == kRK4Mid) {
      const T dr = dt * r;
      const T a = accv[v] + cA * dr;
      p.acc[i] = p.fold ? u0v[v] + a : a;
      out[v] = u0v[v] + cB * dr;
    } else if (KIND == kRK4Last) {
      if constexpr (COMP) {
        T c = p.comp[i];
        out[v] = comp_add<T>(u0v[v], accv[v] + cA * (dt * r), c);
        p.comp[i] = c;
      } else {
        out[v] = accv[v] + cA * (dt * r);
      }
    } else if (KIND == kLSFirst) {
      const T q = dt * r;
      p.acc[i] = q;
      out[v] = Y[v] + cB * q;
    } else {  // kLSMid
      const T q = cA * accv[v] + dt * r;
      p.acc[i] = q;
      out[v] = Y[v] + cB * q;
    }
    p.Yout[i] = out[v];
  }
}


// Free-running asynchronous steps (the body shared by the Euler and
// Navier-Stokes kernels): workgroup b owns block b for the whole
// run and advances it without any grid-wide barrier.  Per step n:
//  1. the delay from each neighbour is what that neighbour has published:
//     k = max(0, n - prog[q]); while k > L - 1 the workgroup waits (bounded
//     by spin_limit polls; past it, *abort is set and every workgroup
//     leaves).  This is the synchronization-avoiding rule of Alg. 3 with
//     delays that come from the run itself instead of a schedule;
//  2. the block's stage halos are assembled from the ring with those delays;
//  3. the s stages run over the block's tiles, the last one writing ring
//     level n+1 of the block's boundary layers;
//  4. the block publishes prog[b] = n + 1.
// Ordering across workgroups: every thread fences at agent scope (release)
// before the publishing store; a reader polls with relaxed loads and fences
// (acquire) once the level it needs is published, before the workgroup
// barrier behind which all its threads read the ring, so ring data written
// on another XCD is seen.  A neighbour can run at most L - 1 steps ahead of
// a reader, so a ring of C + 2L - 1 levels keeps every level a reader may
// still need.
template <typename T, int S, int CL, typename TileFn>
__device__ __forceinline__ void async_run(const StageParams<T>* __restrict__ ps, const AsyncArgs& a,
                                          StageParams<T>& sp, TileFn&& tile) {
  __shared__ int sk[kNumSlots];
  __shared__ int sabort;
  const int b = blockIdx.x;
  const BlockDev* __restrict__ Bg = ps[0].blocks + b;
  for (int it = 0; it < a.nsteps; ++it) {
    const long long n = a.n0 + it;
    // 1. delays from the neighbours' published levels
    if (threadIdx.x == 0) sabort = 0;
    __syncthreads();
    if (threadIdx.x < kNumSlots) {
      const int s = threadIdx.x;
      int k = -1;
      if (Bg->hoff[s] >= 0) {
        const int q = Bg->nbr[s];
        for (long long poll = 0;; ++poll) {
          const int m = __hip_atomic_load(a.prog + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const long long kk = n - m;
          if (kk <= a.L - 1) {
            k = kk < 0 ? 0 : (int)kk;
            // pairs with the neighbour's release: its ring level m is visible
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            break;
          }
          if (poll >= a.spin_limit || __hip_atomic_load(a.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            __hip_atomic_store(a.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            atomicOr(&sabort, 1);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      sk[s] = k;
      a.log[((long long)it * a.nb + b) * kNumSlots + s] = (int8_t)k;
    }
    __syncthreads();
    if (sabort) return;
    // 2. the block's stage halos of step n
    const int slot_now = (int)(n % a.D);
    for (int r = a.reg_begin[b]; r < a.reg_begin[b + 1]; ++r) {
      const HaloRegion rg = a.regions[r];
      const int k = sk[rg.kidx - b * kNumSlots];
      for (int i = threadIdx.x; i < rg.npts; i += blockDim.x) {
        if (a.stale)
          assemble_halo_point<T, S, CL, true>(ps[0].ring, (T*)ps[0].hbuf, rg, i, k, slot_now, a.D, a.W, a.L,
                                             a.slot_stride, a.slot_stride);
        else
          assemble_halo_point<T, S, CL, false>(ps[0].ring, (T*)ps[0].hbuf, rg, i, k, slot_now, a.D, a.W, a.L,
                                              a.slot_stride, a.slot_stride);
      }
    }
    __syncthreads();
    // 3. the stages over the block's tiles
    for (int e = 0; e < S; ++e) {
      stage_struct(ps + e, &sp);
      if (threadIdx.x == 0) sp.slot_now = slot_now;
      __syncthreads();
      for (int t = a.tile_begin[b]; t < a.tile_begin[b + 1]; ++t) {
        tile(sp, a.tiles[t], e);
        __syncthreads();
      }
    }
    // 4. publish ring level n + 1
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(a.prog + b, (int)(n + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace atns
