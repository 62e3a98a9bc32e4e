// Two consecutive classical RK4 stages of the Euler equations in one pass.
//
// Under asynchronous halos (AT or AS) the halo values of every stage of a
// step come from the delayed-level ring, never from the neighbours' current
// stages, so a tile can compute stage A on its own points plus a 2-point
// apron and go straight on to stage B without any exchange.  The
// intermediate stage field never leaves the chip: per point and pair, the
// stage-A output (20 B written, 20 B read back) and the first RK register
// update (40 B) disappear from the HBM traffic.  Under synchronous halos
// the apron points outside the block are computed from the global field in
// the same way.  Results equal the two separate stage kernels bit for bit:
// the fluxes, the derivative expressions and the RK updates are the same.
//
// Work decomposition: a workgroup owns a TX x TY column tile of one block,
// one thread per point of the tile plus a 2-point apron (the E2 columns),
// and walks it along z.  Iteration i loads plane i of the stage-A input;
// stage A is evaluated at plane m = i - 2 on the tile and its x/y cross
// apron, stage B at plane p = i - 4 on the tile.  Registers hold, per
// column, the five stage-A input planes m-2..m+2, the five stage-B input
// planes p-2..p+2 and the stage-A RK register of planes p..m.  The x and y
// fluxes of both stages are staged in LDS (double-buffered, one barrier per
// plane); the x/y fluxes two and three points out (the outer ring) come from
// the first 4(TX + TY) threads.  Pairs: PAIR 0 = stages 1, 2 (first, middle),
// PAIR 1 = stages 3, 4 (middle, last; the last writes the ring).  PAIR 1
// reads U^n at apron points that other tiles own, so its new state goes to a
// buffer no tile reads in that pass (the context swaps state buffers after
// each step) instead of overwriting U^n in place.
#include "euler_flux.hpp"
#include "kernels_common.hpp"

namespace atns {

template <typename T, int TX, int TY>
struct PairLds {
  BlockDev B;
  T FA[2][5][TY + 4][TX + 8];   // stage-A x-flux, x in [-4, nx+4), y in [-2, ny+2)
  T GA[2][5][TY + 8][TX + 4];   // stage-A y-flux, x in [-2, nx+2), y in [-4, ny+4)
  T FB[2][5][TY][TX + 4];       // stage-B x-flux, x in [-2, nx+2), y in [0, ny)
  T GB[2][5][TY + 4][TX];       // stage-B y-flux, x in [0, nx), y in [-2, ny+2)
};

// The RK point update of a stage kind, as in the stage kernels' epilogue.
template <typename T, int KIND>
__device__ __forceinline__ void pair_update(T dt, T cA, T cB, int fold, T Y, T r, T accv, T u0v, T& out, T& acc) {
  if (KIND == kRK4First) {
    const T dr = dt * r;
    acc = cA * dr;
    out = Y + cB * dr;
  } else if (KIND == kRK4Mid) {
    const T dr = dt * r;
    const T a = accv + cA * dr;
    acc = fold ? u0v + a : a;
    out = u0v + cB * dr;
  } else {  // kRK4Last
    out = accv + cA * (dt * r);
  }
}

// Whether the value at block-local (lx, ly, lz) exists for stage parameters
// p: anywhere under synchronous halos; otherwise inside the block or in a
// face halo (outside along one axis, by at most the halo depth).
template <typename T>
__device__ __forceinline__ bool pair_valid(const StageParams<T>& p, const BlockDev* __restrict__ B, int lx, int ly,
                                           int lz) {
  if (p.halo == kHaloSync) return true;
  const int ox = lx < 0 ? -lx : (lx >= B->s[0] ? lx - B->s[0] + 1 : 0);
  const int oy = ly < 0 ? -ly : (ly >= B->s[1] ? ly - B->s[1] + 1 : 0);
  const int oz = lz < 0 ? -lz : (lz >= B->s[2] ? lz - B->s[2] + 1 : 0);
  const int out = (ox > 0) + (oy > 0) + (oz > 0);
  return out == 0 || (out == 1 && ox + oy + oz <= p.H);
}

template <typename T>
__device__ __forceinline__ void pair_dummy(T u[5]) {
  u[0] = T(1);
  u[1] = T(0);
  u[2] = T(0);
  u[3] = T(0);
  u[4] = T(1);
}

template <typename T, int TX, int TY, int PAIR>
__global__ void __launch_bounds__((TX + 4) * (TY + 4))
    euler_pair_kernel(const StageParams<T> pA0, const StageParams<T> pB0) {
  constexpr int KA = PAIR == 0 ? kRK4First : kRK4Mid;
  constexpr int KB = PAIR == 0 ? kRK4Mid : kRK4Last;
  static_assert(4 * (TX + TY) <= (TX + 4) * (TY + 4), "tile too narrow for its outer ring");
  const StageParams<T> pA = resolve_step(pA0);
  const StageParams<T> pB = resolve_step(pB0);
  const TileDev t = pA.tiles[blockIdx.x];
  __shared__ PairLds<T, TX, TY> L;
  if (t.nx != 0) {
    stage_block(pA.blocks + t.blk, &L.B);
    const BlockDev* __restrict__ B = &L.B;
    const int tid = threadIdx.x;
    const int nx = t.nx, ny = t.ny;
    // E2 column of this thread (tile-relative), and its role
    const int x = tid % (TX + 4) - 2, y = tid / (TX + 4) - 2;
    const bool e2 = x < nx + 2 && y < ny + 2;
    const bool inx = x >= 0 && x < nx, iny = y >= 0 && y < ny;
    const bool tile = inx && iny;
    const bool xcross = e2 && iny && !inx;    // x in [-2, 0) or [nx, nx+2)
    const bool ycross = e2 && inx && !iny;
    const bool cross = tile || xcross || ycross;
    const int lx = t.x0 + x, ly = t.y0 + y;
    // outer ring: x-flux columns x in {-4, -3, nx+2, nx+3} for y in [0, ny),
    // y-flux rows y in {-4, -3, ny+2, ny+3} for x in [0, nx)
    int rrole = 0, rx = 0, ry = 0;
    if (tid < 4 * ny) {
      const int c = tid / ny;
      ry = tid % ny;
      rx = c < 2 ? c - 4 : nx + c;
      rrole = 1;
    } else if (tid < 4 * ny + 4 * nx) {
      const int q = tid - 4 * ny;
      const int c = q / nx;
      rx = q % nx;
      ry = c < 2 ? c - 4 : ny + c;
      rrole = 2;
    }
    const T gm1 = (T)(pA.gamma - 1.0);
    const T ihx = (T)pA.dscale[0], ihy = (T)pA.dscale[1], ihz = (T)pA.dscale[2];
    const T w1 = pA.cd2 ? T(1) : T(8), w2 = pA.cd2 ? T(0) : T(1);
    const T dtA = (T)pA.dt, cAA = (T)pA.cA, cBA = (T)pA.cB;
    const T dtB = (T)pB.dt, cAB = (T)pB.cA, cBB = (T)pB.cB;
    ColumnSource<T> col{}, rcol{};
    if (e2) col = column_source(pA, B, lx, ly);
    if (rrole) rcol = column_source(pA, B, t.x0 + rx, t.y0 + ry);
    T* ring_slot = nullptr;
    RingColumn rlay{};
    if (pB.ring_write) {
      ring_slot = pB.ring + (long long)((pB.slot_now + 1) % pB.D) * pB.slot_stride;
      if (tile) rlay = ring_column(B, pB.H, lx, ly);
    }
    const int z0 = t.z0, nz = t.nz;
    T Uq[5][5], Yq[5][5], aq[3][5];
    T nxt[5], rnx[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      pair_dummy(Uq[j]);
      pair_dummy(Yq[j]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) pair_dummy(aq[j]);
    pair_dummy(nxt);
    pair_dummy(rnx);
    const int i_begin = z0 - 4, i_end = z0 + nz + 4;   // exclusive
    if (e2 && pair_valid(pA, B, lx, ly, i_begin)) fetch_col(pA, B, col, t.blk, lx, ly, i_begin, nxt);
    for (int i = i_begin; i < i_end; ++i) {
      const int buf = i & 1;
      const int m = i - 2, p = i - 4;
      const bool actA = m >= z0 - 2 && m < z0 + nz + 2;
      const bool actB = p >= z0 && p < z0 + nz;
      // ------------------------------------------------ plane i in, prefetch
      if (e2) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 5; ++v) Uq[j][v] = Uq[j + 1][v];
#pragma unroll
        for (int v = 0; v < 5; ++v) Uq[4][v] = nxt[v];
        pair_dummy(nxt);
        if (i + 1 < i_end && pair_valid(pA, B, lx, ly, i + 1)) fetch_col(pA, B, col, t.blk, lx, ly, i + 1, nxt);
      }
      T ur[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) ur[v] = rnx[v];
      if (rrole) {
        // the ring's plane m + 1, used in the next iteration
        pair_dummy(rnx);
        if (m + 1 >= z0 - 2 && m + 1 < z0 + nz + 2 && pair_valid(pA, B, t.x0 + rx, t.y0 + ry, m + 1))
          fetch_col(pA, B, rcol, t.blk, t.x0 + rx, t.y0 + ry, m + 1, rnx);
      }
      // stage-A operands of plane m that are loaded (middle stage)
      T u0v[5], accv[5];
      pair_dummy(u0v);
      pair_dummy(accv);
      const bool inside = lx >= 0 && lx < B->s[0] && ly >= 0 && ly < B->s[1] && m >= 0 && m < B->s[2];
      const bool needA = actA && cross && (inside || pA.halo == kHaloSync);
      long long gm = 0;
      if (needA) {
        const int gx = wrap(B->o[0] + lx, pA.n[0]);
        const int gy = wrap(B->o[1] + ly, pA.n[1]);
        const int gz = wrap(B->o[2] + m, pA.n[2]);
        gm = ((long long)gz * pA.n[1] + gy) * pA.n[0] + gx;
        if (KA == kRK4Mid) {
#pragma unroll
          for (int v = 0; v < 5; ++v) u0v[v] = pA.U0[v * pA.field + gm];
          if (tile) {
#pragma unroll
            for (int v = 0; v < 5; ++v) accv[v] = pA.acc[v * pA.field + gm];
          }
        }
      }
      // ------------------------------------- A. x/y fluxes of both stages
      if (actA && e2) {
        T f[5];
        euler_flux(Uq[2], 0, gm1, f);
#pragma unroll
        for (int v = 0; v < 5; ++v) L.FA[buf][v][y + 2][x + 4] = f[v];
        euler_flux(Uq[2], 1, gm1, f);
#pragma unroll
        for (int v = 0; v < 5; ++v) L.GA[buf][v][y + 4][x + 2] = f[v];
      }
      if (actA && rrole) {
        T f[5];
        if (rrole == 1) {
          euler_flux(ur, 0, gm1, f);
#pragma unroll
          for (int v = 0; v < 5; ++v) L.FA[buf][v][ry + 2][rx + 4] = f[v];
        } else {
          euler_flux(ur, 1, gm1, f);
#pragma unroll
          for (int v = 0; v < 5; ++v) L.GA[buf][v][ry + 4][rx + 2] = f[v];
        }
      }
      if (actB && cross) {
        // stage-B input of plane p sits in Yq[3] until this plane's stage A
        T f[5];
        if (iny) {
          euler_flux(Yq[3], 0, gm1, f);
#pragma unroll
          for (int v = 0; v < 5; ++v) L.FB[buf][v][y][x + 2] = f[v];
        }
        if (inx) {
          euler_flux(Yq[3], 1, gm1, f);
#pragma unroll
          for (int v = 0; v < 5; ++v) L.GB[buf][v][y + 2][x] = f[v];
        }
      }
      lds_barrier();
      // ------------------------------------------------ B. stage A at plane m
      if (actA && e2) {
        T ya[5];
        pair_dummy(ya);
        if (needA) {
          T R[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const T dx = (w1 * (L.FA[buf][v][y + 2][x + 5] - L.FA[buf][v][y + 2][x + 3]) -
                          w2 * (L.FA[buf][v][y + 2][x + 6] - L.FA[buf][v][y + 2][x + 2])) * ihx;
            const T dy = (w1 * (L.GA[buf][v][y + 5][x + 2] - L.GA[buf][v][y + 3][x + 2]) -
                          w2 * (L.GA[buf][v][y + 6][x + 2] - L.GA[buf][v][y + 2][x + 2])) * ihy;
            R[v] = -(dx + dy);
          }
          T h0[5], h1[5], h3[5], h4[5];
          euler_flux(Uq[0], 2, gm1, h0);
          euler_flux(Uq[1], 2, gm1, h1);
          euler_flux(Uq[3], 2, gm1, h3);
          euler_flux(Uq[4], 2, gm1, h4);
#pragma unroll
          for (int v = 0; v < 5; ++v) R[v] -= (w1 * (h3[v] - h1[v]) - w2 * (h4[v] - h0[v])) * ihz;
          T acc[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) pair_update<T, KA>(dtA, cAA, cBA, pA.fold, Uq[2][v], R[v], accv[v], u0v[v], ya[v], acc[v]);
#pragma unroll
          for (int v = 0; v < 5; ++v) accv[v] = acc[v];
        } else if (cross && pair_valid(pB, B, lx, ly, m)) {
          fetch(pB, B, t.blk, lx, ly, m, ya);   // stage-B halo value (AT/AS)
        }
        if (tile) {
          // stage A's RK register of plane m (planes outside the block: unused)
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            aq[0][v] = aq[1][v];
            aq[1][v] = aq[2][v];
            aq[2][v] = needA ? accv[v] : T(0);
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 5; ++v) Yq[j][v] = Yq[j + 1][v];
#pragma unroll
        for (int v = 0; v < 5; ++v) Yq[4][v] = ya[v];
      }
      // ------------------------------------------------ C. stage B at plane p
      if (actB && tile) {
        T R[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const T dx = (w1 * (L.FB[buf][v][y][x + 3] - L.FB[buf][v][y][x + 1]) -
                        w2 * (L.FB[buf][v][y][x + 4] - L.FB[buf][v][y][x])) * ihx;
          const T dy = (w1 * (L.GB[buf][v][y + 3][x] - L.GB[buf][v][y + 1][x]) -
                        w2 * (L.GB[buf][v][y + 4][x] - L.GB[buf][v][y][x])) * ihy;
          R[v] = -(dx + dy);
        }
        T h0[5], h1[5], h3[5], h4[5];
        euler_flux(Yq[0], 2, gm1, h0);
        euler_flux(Yq[1], 2, gm1, h1);
        euler_flux(Yq[3], 2, gm1, h3);
        euler_flux(Yq[4], 2, gm1, h4);
#pragma unroll
        for (int v = 0; v < 5; ++v) R[v] -= (w1 * (h3[v] - h1[v]) - w2 * (h4[v] - h0[v])) * ihz;
        const long long g = ((long long)(B->o[2] + p) * pA.n[1] + (B->o[1] + ly)) * pA.n[0] + (B->o[0] + lx);
        T out[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          T acc;
          // the stage-B RK register input is stage A's, two planes back; the
          // middle stage's U^n is the stage-A input of plane p (pair 0)
          pair_update<T, KB>(dtB, cAB, cBB, pB.fold, Yq[2][v], R[v], aq[0][v], Uq[0][v], out[v], acc);
          if (KB == kRK4Mid) pB.acc[v * pB.field + g] = acc;
          pB.Yout[v * pB.field + g] = out[v];
        }
        if (ring_slot) ring_write_col(B, rlay, pB.H, true, lx, ly, p, out, ring_slot);
      }
    }
  }
  if (pB.step_end) finish_step(pB.step_end, pB.done);
}

template <typename T, int TX, int TY>
hipError_t launch_pair_shape(const StageParams<T>& pA, const StageParams<T>& pB, int ntiles, int pair,
                             hipStream_t s) {
  dim3 grid(ntiles), block((TX + 4) * (TY + 4));
  if (pair == 0)
    euler_pair_kernel<T, TX, TY, 0><<<grid, block, 0, s>>>(pA, pB);
  else
    euler_pair_kernel<T, TX, TY, 1><<<grid, block, 0, s>>>(pA, pB);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_euler_pair(const StageParams<T>& pA, const StageParams<T>& pB, int ntiles, int pair, int tx,
                             int ty, hipStream_t s) {
  if (tx == 16 && ty == 16) return launch_pair_shape<T, 16, 16>(pA, pB, ntiles, pair, s);
  if (tx == 32 && ty == 8) return launch_pair_shape<T, 32, 8>(pA, pB, ntiles, pair, s);
  if (tx == 16 && ty == 8) return launch_pair_shape<T, 16, 8>(pA, pB, ntiles, pair, s);
  if (tx == 32 && ty == 16) return launch_pair_shape<T, 32, 16>(pA, pB, ntiles, pair, s);
  return hipErrorInvalidValue;
}
template hipError_t launch_euler_pair<float>(const StageParams<float>&, const StageParams<float>&, int, int, int,
                                             int, hipStream_t);

}  // namespace atns
