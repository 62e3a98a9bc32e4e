// Fused Navier-Stokes right-hand side + RK stage kernel.
//
// R = -sum_d D_d (F_d - Fv_d / Re), Fv_d = (0, tau_d1, tau_d2, tau_d3,
// u_j tau_dj + kappa dT/dx_d) with tau_ij = du_i/dx_j + du_j/dx_i
// - (2/3) delta_ij div u (mu = 1), every derivative the explicit CD4 of
// Eq. (2).  The viscous terms are repeated first derivatives (gradients of
// u, v, w, T first, then the divergence of the viscous flux), so a point's
// right-hand side reads the state up to 4 points away along each axis and
// 2 x 2 points diagonally in each coordinate plane.
//
// Work decomposition (2.5D, one thread per point of the tile footprint):
// a workgroup covers a TX x TY column tile of one block plus its footprint
// (a 4-point apron in x and y and the 2 x 2 xy corners), EX x EY threads in
// all.  The tile is walked along z.  Every thread keeps the last five planes
// of (u, v, w, T) at its own (x, y) in registers, so z-derivatives need no
// shared memory.  Per plane m:
//   1. the front plane m + 2 is fetched (halo rule of the stage applied by
//      fetch()), turned into primitives and pushed on the queues;
//   2. plane m's (u, v, w, T) goes to one LDS plane;
//   3. threads at the tile and its 2-point cross apron compute the full
//      gradient at plane m and their fluxes: the x-flux F - Fv_x/Re on the
//      x-cross, the y-flux on the y-cross (both into LDS), the z-flux at the
//      tile, which is scattered straight into a register accumulator of the
//      five planes m-2..m+2;
//   4. tile threads add the x and y divergences of plane m;
//   5. plane m-2 is complete: its RK epilogue and ring write run.
#include "kernels_common.hpp"

namespace atns {

template <typename T, int TX, int TY, int KIND, int NDIM>
__global__ void __launch_bounds__((TX + 8) * (TY + 8)) ns_stage_kernel(const StageParams<T> p) {
  constexpr int EX = TX + 8, EY = TY + 8;
  const TileDev t = p.tiles[blockIdx.x];
  if (t.nx == 0) return;
  const BlockDev* __restrict__ B = p.blocks + t.blk;
  const int tid = threadIdx.x;
  const int x = tid % EX - 4, y = tid / EX - 4;   // tile-local, -4 .. T+3
  const int nx = t.nx, ny = t.ny;
  const int dx = x < 0 ? -x : (x >= nx ? x - nx + 1 : 0);   // distance outside, 1-based
  const int dy = y < 0 ? -y : (y >= ny ? y - ny + 1 : 0);
  const bool inx = dx == 0, iny = dy == 0;
  const bool core = inx && iny;
  const bool crossx = iny && dx >= 1 && dx <= 2;
  const bool crossy = inx && dy >= 1 && dy <= 2;
  const bool outer = (iny && dx >= 3 && dx <= 4) || (inx && dy >= 3 && dy <= 4) ||
                     (dx >= 1 && dx <= 2 && dy >= 1 && dy <= 2);
  const bool grad_pt = core || crossx || crossy;
  const int lx = t.x0 + x, ly = t.y0 + y;
  constexpr bool three = (NDIM == 3);

  const T gm1 = (T)(p.gamma - 1.0);
  const T gM2 = (T)p.mach2_gamma;
  const T kap = (T)p.kappa;
  const T ire = (T)p.inv_re;
  const T ihx = (T)p.inv12h[0], ihy = (T)p.inv12h[1], ihz = (T)p.inv12h[2];
  const T two3 = (T)(2.0 / 3.0);

  __shared__ T sP[4][EY][EX];          // u, v, w, T of plane m
  __shared__ T sFX[5][TY][TX + 4];     // F - Fv_x/Re on the x-cross of plane m
  __shared__ T sFY[5][TY + 4][TX];     // G - Fv_y/Re on the y-cross of plane m

  // queues: q*[j] holds plane f-4+j; r*[j] holds plane f-2+j
  T qu[5], qv[5], qw[5], qT[5];
  T rr[3], rp[3], re[3];
  T acc[5][5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    qu[j] = qv[j] = qw[j] = qT[j] = T(0);
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[j][v] = T(0);
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) rr[j] = rp[j] = re[j] = T(0);

  T* ring_slot = nullptr;
  if (p.ring_write) ring_slot = p.ring + (long long)((p.slot_now + 1) % p.D) * p.slot_stride;

  const int z0 = t.z0, nz = t.nz;
  const int f_begin = three ? z0 - 4 : 0;
  const int f_end = three ? z0 + nz + 4 : 1;   // exclusive
  for (int f = f_begin; f < f_end; ++f) {
    const int m = three ? f - 2 : f;   // plane whose gradients are formed now
    // ---------------------------------------------------- 1. fetch plane f
    const int rel = f - z0;
    const bool tileplane = rel >= 0 && rel < nz;
    const bool near = (rel >= -2 && rel < 0) || (rel >= nz && rel < nz + 2);
    const bool far = (rel >= -4 && rel < -2) || (rel >= nz + 2 && rel < nz + 4);
    const bool need = core ? (tileplane || near || far)
                           : ((crossx || crossy) ? (tileplane || near) : (outer && tileplane));
    if (three) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        qu[j] = qu[j + 1];
        qv[j] = qv[j + 1];
        qw[j] = qw[j + 1];
        qT[j] = qT[j + 1];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        rr[j] = rr[j + 1];
        rp[j] = rp[j + 1];
        re[j] = re[j + 1];
      }
    }
    constexpr int qi = three ? 4 : 2;   // queue slot of the fetched plane
    constexpr int ri = three ? 2 : 0;
    if (need) {
      T u[5];
      fetch(p, B, t.blk, lx, ly, f, u);
      const T ir = T(1) / u[0];
      const T vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
      const T pr = gm1 * (u[4] - T(0.5) * (u[1] * vx + u[2] * vy + u[3] * vz));
      qu[qi] = vx;
      qv[qi] = vy;
      qw[qi] = vz;
      qT[qi] = gM2 * pr * ir;
      rr[ri] = u[0];
      rp[ri] = pr;
      re[ri] = u[4];
    }
    // ------------------------------------------ 2. plane m into shared memory
    const int mrel = m - z0;
    const bool m_tile = mrel >= 0 && mrel < nz;
    const bool m_grad = three ? (mrel >= -2 && mrel < nz + 2) : true;
    {
      const bool has_m = core ? (mrel >= -4 && mrel < nz + 4)
                              : ((crossx || crossy) ? (mrel >= -2 && mrel < nz + 2) : (outer && m_tile));
      if (has_m && m_grad) {
        sP[0][y + 4][x + 4] = qu[2];
        sP[1][y + 4][x + 4] = qv[2];
        sP[2][y + 4][x + 4] = qw[2];
        sP[3][y + 4][x + 4] = qT[2];
      }
    }
    __syncthreads();
    // ------------------------------------------- 3. gradients and fluxes
    T zf[5];
    if (m_grad && (core || (m_tile && grad_pt))) {
      const int sx = x + 4, sy = y + 4;
      T g[3][3], gT[3];   // g[i][j] = d u_i / d x_j
      T dz[4] = {T(0), T(0), T(0), T(0)};
      if constexpr (three) {
        dz[0] = (T(8) * (qu[3] - qu[1]) - (qu[4] - qu[0])) * ihz;
        dz[1] = (T(8) * (qv[3] - qv[1]) - (qv[4] - qv[0])) * ihz;
        dz[2] = (T(8) * (qw[3] - qw[1]) - (qw[4] - qw[0])) * ihz;
        dz[3] = (T(8) * (qT[3] - qT[1]) - (qT[4] - qT[0])) * ihz;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const T ddx = (T(8) * (sP[c][sy][sx + 1] - sP[c][sy][sx - 1]) - (sP[c][sy][sx + 2] - sP[c][sy][sx - 2])) * ihx;
        const T ddy = (T(8) * (sP[c][sy + 1][sx] - sP[c][sy - 1][sx]) - (sP[c][sy + 2][sx] - sP[c][sy - 2][sx])) * ihy;
        if (c < 3) {
          g[c][0] = ddx;
          g[c][1] = ddy;
          g[c][2] = dz[c];
        } else {
          gT[0] = ddx;
          gT[1] = ddy;
          gT[2] = dz[3];
        }
      }
      const T div = g[0][0] + g[1][1] + g[2][2];
      const T vel[3] = {qu[2], qv[2], qw[2]};
      const T rho = rr[0], pres = rp[0], et = re[0];
      // flux along direction d: inviscid minus viscous / Re
      auto flux = [&](int d, T out[5]) {
        T tau[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) tau[j] = (g[d][j] + g[j][d]) - (d == j ? two3 * div : T(0));
        const T ud = vel[d];
        out[0] = rho * ud;
        out[1] = rho * vel[0] * ud - ire * tau[0];
        out[2] = rho * vel[1] * ud - ire * tau[1];
        out[3] = rho * vel[2] * ud - ire * tau[2];
        out[1 + d] += pres;
        out[4] = (et + pres) * ud - ire * (vel[0] * tau[0] + vel[1] * tau[1] + vel[2] * tau[2] + kap * gT[d]);
      };
      if (m_tile) {
        T fl[5];
        if (core || crossx) {
          flux(0, fl);
#pragma unroll
          for (int v = 0; v < 5; ++v) sFX[v][y][x + 2] = fl[v];
        }
        if (core || crossy) {
          flux(1, fl);
#pragma unroll
          for (int v = 0; v < 5; ++v) sFY[v][y + 2][x] = fl[v];
        }
      }
      if (core && three) flux(2, zf);
    }
    if (core && three && m_grad) {
      // z-divergence contributions of plane m to planes m-2 .. m+2
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const T z = zf[v] * ihz;
        acc[0][v] += z;
        acc[1][v] -= T(8) * z;
        acc[3][v] += T(8) * z;
        acc[4][v] -= z;
      }
    }
    __syncthreads();
    // -------------------------------------------- 4. x and y divergence
    if (core && m_tile) {
      constexpr int ai = three ? 2 : 0;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const T ddx = (T(8) * (sFX[v][y][x + 3] - sFX[v][y][x + 1]) - (sFX[v][y][x + 4] - sFX[v][y][x])) * ihx;
        const T ddy = (T(8) * (sFY[v][y + 3][x] - sFY[v][y + 1][x]) - (sFY[v][y + 4][x] - sFY[v][y][x])) * ihy;
        acc[ai][v] -= ddx + ddy;
      }
    }
    // --------------------------------------------- 5. finish plane m - 2
    const int pz = three ? m - 2 : m;
    if (core && pz >= z0 && pz < z0 + nz) {
      const int gx = B->o[0] + lx, gy = B->o[1] + ly, gz = B->o[2] + pz;
      const long long gi = ((long long)gz * p.n[1] + gy) * p.n[0] + gx;
      T Y[5], out[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) Y[v] = p.Y[v * p.field + gi];
      epilogue<T, KIND>(p, gi, Y, acc[0], out);
      if (ring_slot) ring_store(p, B, lx, ly, pz, out, ring_slot);
    }
    if (three) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[j][v] = acc[j + 1][v];
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[4][v] = T(0);
    }
  }
}

template <typename T, int KIND>
hipError_t launch_ns_kind(const StageParams<T>& p, int ntiles, hipStream_t s) {
  constexpr int TX = 16, TY = 16;
  dim3 grid(ntiles), block((TX + 8) * (TY + 8));
  if (p.ndim == 3)
    ns_stage_kernel<T, TX, TY, KIND, 3><<<grid, block, 0, s>>>(p);
  else
    ns_stage_kernel<T, TX, TY, KIND, 2><<<grid, block, 0, s>>>(p);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ns_stage(const StageParams<T>& p, int ntiles, int kind, hipStream_t s) {
  switch (kind) {
    case kRhsOnly: return launch_ns_kind<T, kRhsOnly>(p, ntiles, s);
    case kRK4First: return launch_ns_kind<T, kRK4First>(p, ntiles, s);
    case kRK4Mid: return launch_ns_kind<T, kRK4Mid>(p, ntiles, s);
    case kRK4Last: return launch_ns_kind<T, kRK4Last>(p, ntiles, s);
    case kLSFirst: return launch_ns_kind<T, kLSFirst>(p, ntiles, s);
    default: return launch_ns_kind<T, kLSMid>(p, ntiles, s);
  }
}

template hipError_t launch_ns_stage<float>(const StageParams<float>&, int, int, hipStream_t);
template hipError_t launch_ns_stage<double>(const StageParams<double>&, int, int, hipStream_t);

}  // namespace atns
