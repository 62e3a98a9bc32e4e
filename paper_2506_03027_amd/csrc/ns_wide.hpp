// Navier-Stokes stage tile for double precision: one thread per point of the
// tile footprint ((TX + 8) x (TY + 8) threads), so that each thread holds the
// z-queue of one column only.  Used for the FP64 synchronous baseline, where
// the single-precision tile's per-thread queues (a tile and a cross column,
// twice the registers per value) would leave one wave per SIMD.  The
// arithmetic of a point is that of ns_tile (kernels_ns.hip).
//
// Per plane m: the front plane m + 2 is fetched (halo rule of the stage
// applied by fetch()), turned into primitives and pushed on the queues;
// plane m's (u, v, w, T) goes to one LDS plane; threads at the tile and its
// 2-point cross apron compute the full gradient at plane m and their fluxes
// (the x-flux on the x-cross, the y-flux on the y-cross, both into LDS; the
// z-flux at the tile, which with the z-fluxes of the last four planes kept in
// LDS completes the z-divergence of plane m-2); the threads outside the tile
// form the x/y divergence of plane m-1 for the tile threads; plane m-2 gets
// its RK epilogue and ring write.  One barrier per plane.
#pragma once
#include "kernels_common.hpp"

namespace atns {

template <typename T, int TX, int TY>
struct NsWideLds {
  BlockDev B;
  T P[2][4][TY + 8][TX + 8];   // u, v, w, T of plane m (double-buffered)
  T FX[2][5][TY][TX + 4];      // F - Fv_x/Re on the x-cross of plane m
  T FY[2][5][TY + 4][TX];      // G - Fv_y/Re on the y-cross of plane m
  T H[4][5][TY][TX];           // z-fluxes of the last four gradient planes
  T XY[2][5][TY][TX];          // x/y divergence of the tile's points
};
template <typename T, int TX, int TY>
__device__ __forceinline__ NsWideLds<T, TX, TY>& ns_wide_lds() {
  __shared__ NsWideLds<T, TX, TY> s;
  return s;
}

template <typename T, int TX, int TY, int KIND, int NDIM, bool COMP = false>
__device__ __forceinline__ void ns_tile_wide(const StageParams<T>& p, const TileDev t) {
  constexpr int EX = TX + 8, EY = TY + 8;
  constexpr bool three = (NDIM == 3);
  if (t.nx == 0) return;
  // The block descriptor lives in LDS for the whole kernel: re-reading it from
  // global memory inside the plane loop would make every such load wait for
  // all outstanding (prefetch) loads.
  NsWideLds<T, TX, TY>& lds = ns_wide_lds<T, TX, TY>();
  stage_block(p.blocks + t.blk, &lds.B);
  const BlockDev* __restrict__ B = &lds.B;
  const int tid = threadIdx.x;
  // Thread -> footprint point, grouped so that whole waves share a role: the
  // TX x TY tile first, then the 2-point cross apron, then the outer apron
  // (3-4 points out along x or y, and the 2 x 2 xy corners).  Phases that
  // only tile points (or tile and cross points) take part in then run on
  // full waves.  Threads beyond the footprint sit at a point no role needs.
  int x, y;
  {
    int r = tid;
    if (r < TX * TY) {
      x = r % TX;
      y = r / TX;
    } else if ((r -= TX * TY) < 4 * TY) {   // x-cross: 2 columns each side
      const int side = r / (2 * TY), q = r % (2 * TY);
      y = q >> 1;
      x = side ? TX + (q & 1) : -1 - (q & 1);
    } else if ((r -= 4 * TY) < 4 * TX) {    // y-cross: 2 rows each side
      const int side = r / (2 * TX), q = r % (2 * TX);
      x = q % TX;
      y = side ? TY + q / TX : -1 - q / TX;
    } else if ((r -= 4 * TX) < 4 * TY) {    // x-outer: columns 3-4 out
      const int side = r / (2 * TY), q = r % (2 * TY);
      y = q >> 1;
      x = side ? TX + 2 + (q & 1) : -3 - (q & 1);
    } else if ((r -= 4 * TY) < 4 * TX) {    // y-outer: rows 3-4 out
      const int side = r / (2 * TX), q = r % (2 * TX);
      x = q % TX;
      y = side ? TY + 2 + q / TX : -3 - q / TX;
    } else if ((r -= 4 * TX) < 16) {        // 2 x 2 corners
      const int c = r >> 2, q = r & 3;
      x = (c & 1) ? TX + (q & 1) : -1 - (q & 1);
      y = (c & 2) ? TY + (q >> 1) : -1 - (q >> 1);
    } else {
      x = -4;
      y = -4;
    }
  }
  const int nx = t.nx, ny = t.ny;
  // A ragged tile (nx < TX or ny < TY): the far-side apron moves in to the
  // tile's real edge, and tile or apron threads beyond that edge go idle at
  // (-4, -4), a point no role needs.
  {
    const bool idle = (x >= nx && x < TX) || (y >= ny && y < TY);
    if (x >= TX) x -= TX - nx;
    if (y >= TY) y -= TY - ny;
    if (idle) x = y = -4;
  }
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
  const ColumnSource<T> col = column_source(p, B, lx, ly);

  const T gm1 = (T)(p.gamma - 1.0);
  const T gM2 = (T)p.mach2_gamma;
  const T kap = (T)p.kappa;
  const T ire = (T)p.inv_re;
  const T ihx = (T)p.dscale[0], ihy = (T)p.dscale[1], ihz = (T)p.dscale[2];
  // central-difference weights of the inner and outer neighbour pairs
  const T w1 = p.cd2 ? T(1) : T(8), w2 = p.cd2 ? T(0) : T(1);
  const T two3 = (T)(2.0 / 3.0);

  auto& sP = lds.P;     // u, v, w, T of plane m (double-buffered)
  auto& sFX = lds.FX;   // F - Fv_x/Re on the x-cross of plane m
  auto& sFY = lds.FY;   // G - Fv_y/Re on the y-cross of plane m
  // z-fluxes of the last four gradient planes at the tile, plane q in slot
  // q mod 4; each thread reads only its own cells (no barrier needed)
  auto& sH = lds.H;
  // x/y divergence of the tile's points, by plane parity (3D)
  auto& sXY = lds.XY;

  // queues: q*[j] holds plane f-4+j; rr[j] holds the density of plane f-2+j
  // (pressure and energy at the gradient plane are rebuilt from rho, T and u)
  T qu[5], qv[5], qw[5], qT[5];
  T rr[3];
#pragma unroll
  for (int j = 0; j < 5; ++j) qu[j] = qv[j] = qw[j] = qT[j] = T(0);
#pragma unroll
  for (int j = 0; j < 3; ++j) rr[j] = T(1);
  const T igM2 = (T)(1.0 / p.mach2_gamma), igm1 = (T)(1.0 / (p.gamma - 1.0));

  T* ring_slot = nullptr;
  RingColumn rcol{};
  if (p.ring_write) {
    ring_slot = p.ring + (long long)((p.slot_now + 1) % p.D) * p.slot_stride;
    if (core) rcol = ring_column(B, p.H, lx, ly);
  }

  const int z0 = t.z0, nz = t.nz;
  const int f_begin = three ? z0 - 4 : 0;
  // 3D: planes z0-4 .. z0+nz+3 enter; the last tile plane is finished when
  // plane z0+nz+3 has entered.  2D: one plane, and a second pass for the
  // x/y divergence, which runs one pass behind the gradients.
  const int f_end = three ? z0 + nz + 4 : 2;   // exclusive
  // which planes this thread's point is needed at: the tile and the cross
  // apron to 2 planes beyond the tile, the tile column to 4 planes beyond,
  // the outer apron only at tile planes
  auto need_plane = [&](int f) {
    const int rel = f - z0;
    const bool tileplane = rel >= 0 && rel < nz;
    const bool near = (rel >= -2 && rel < 0) || (rel >= nz && rel < nz + 2);
    const bool far = (rel >= -4 && rel < -2) || (rel >= nz + 2 && rel < nz + 4);
    return core ? (tileplane || near || far) : ((crossx || crossy) ? (tileplane || near) : (outer && tileplane));
  };
  T nxt[5] = {T(1), T(0), T(0), T(0), T(1)};
  if (need_plane(f_begin)) fetch_col(p, B, col, t.blk, lx, ly, f_begin, nxt);
  // epilogue operands of the next plane to finish (the tile's first plane)
  const long long gplane = (long long)p.n[0] * p.n[1];
  long long gi = core ? ((long long)(B->o[2] + z0) * p.n[1] + (B->o[1] + ly)) * p.n[0] + (B->o[0] + lx) : 0;
  // the stage input at the point enters only the first RK4 stage and the
  // low-storage updates
  constexpr bool needY = KIND == kRK4First || KIND == kLSFirst || KIND == kLSMid || KIND == kRhsOnly;
  T Yv[5] = {T(0), T(0), T(0), T(0), T(0)}, accv[5], u0v[5];
  if (core) {
    if (needY) {
#pragma unroll
      for (int v = 0; v < 5; ++v) Yv[v] = p.Y[v * p.field + gi];
    }
    epilogue_load<T, KIND, COMP>(p, gi, accv, u0v);
  }

  for (int f = f_begin; f < f_end; ++f) {
    const int it = f - f_begin;
    const int buf = it & 1;
    const int m = three ? f - 2 : f;   // plane whose gradients are formed now
    const int mrel = m - z0;
    const bool m_tile = mrel >= 0 && mrel < nz;
    const bool m_grad = three ? (mrel >= -2 && mrel < nz + 2) : (mrel == 0);
    // ---------------------------------------------------- A. plane f in
    const bool need = (three || f == 0) && need_plane(f);
    if constexpr (three) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        qu[j] = qu[j + 1];
        qv[j] = qv[j + 1];
        qw[j] = qw[j + 1];
        qT[j] = qT[j + 1];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) rr[j] = rr[j + 1];
    }
    constexpr int qi = three ? 4 : 2;   // queue slot of the fetched plane
    constexpr int ri = three ? 2 : 0;
    if (need) {
      // plane f was prefetched during the previous iteration
      const T ir = recip(nxt[0]);
      const T vx = nxt[1] * ir, vy = nxt[2] * ir, vz = nxt[3] * ir;
      const T pr = gm1 * (nxt[4] - T(0.5) * (nxt[1] * vx + nxt[2] * vy + nxt[3] * vz));
      qu[qi] = vx;
      qv[qi] = vy;
      qw[qi] = vz;
      qT[qi] = gM2 * pr * ir;
      rr[ri] = nxt[0];
    }
    // issue the loads of plane f + 1; they complete behind this plane's work
    if (three && f + 1 < f_end && need_plane(f + 1)) fetch_col(p, B, col, t.blk, lx, ly, f + 1, nxt);
    if (m_grad) {
      const bool has_m = core || ((crossx || crossy) && (mrel >= -2 && mrel < nz + 2)) || (outer && m_tile);
      if (has_m) {
        sP[buf][0][y + 4][x + 4] = qu[2];
        sP[buf][1][y + 4][x + 4] = qv[2];
        sP[buf][2][y + 4][x + 4] = qw[2];
        sP[buf][3][y + 4][x + 4] = qT[2];
      }
    }
    lds_barrier();
    // ------------------------------------- B. gradients and fluxes of plane m
    T zd[5] = {T(0), T(0), T(0), T(0), T(0)};   // z-divergence of plane m - 2
    if (m_grad && (core || (m_tile && grad_pt))) {
      const int sx = x + 4, sy = y + 4;
      T g[3][3], gT[3];   // g[i][j] = d u_i / d x_j
      T dz[4] = {T(0), T(0), T(0), T(0)};
      if constexpr (three) {
        dz[0] = (w1 * (qu[3] - qu[1]) - w2 * (qu[4] - qu[0])) * ihz;
        dz[1] = (w1 * (qv[3] - qv[1]) - w2 * (qv[4] - qv[0])) * ihz;
        dz[2] = (w1 * (qw[3] - qw[1]) - w2 * (qw[4] - qw[0])) * ihz;
        dz[3] = (w1 * (qT[3] - qT[1]) - w2 * (qT[4] - qT[0])) * ihz;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const T ddx = (w1 * (sP[buf][c][sy][sx + 1] - sP[buf][c][sy][sx - 1]) -
                       w2 * (sP[buf][c][sy][sx + 2] - sP[buf][c][sy][sx - 2])) * ihx;
        const T ddy = (w1 * (sP[buf][c][sy + 1][sx] - sP[buf][c][sy - 1][sx]) -
                       w2 * (sP[buf][c][sy + 2][sx] - sP[buf][c][sy - 2][sx])) * ihy;
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
      const T rho = rr[0];
      const T pres = rho * qT[2] * igM2;
      const T et = pres * igm1 + T(0.5) * rho * (vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2]);
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
          for (int v = 0; v < 5; ++v) sFX[buf][v][y][x + 2] = fl[v];
        }
        if (core || crossy) {
          flux(1, fl);
#pragma unroll
          for (int v = 0; v < 5; ++v) sFY[buf][v][y + 2][x] = fl[v];
        }
      }
      if constexpr (three) {
        if (core) {
          // the z-flux of plane m completes the CD4 z-divergence of plane
          // m-2 with those of planes m-4, m-3, m-1, then takes plane m-4's slot
          T hz[5];
          flux(2, hz);
          const int s0 = m & 3, s1 = (m - 3) & 3, s3 = (m - 1) & 3;
          const bool zt = mrel - 2 >= 0 && mrel - 2 < nz;
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            if (zt) zd[v] = (w1 * (sH[s3][v][y][x] - sH[s1][v][y][x]) - w2 * (hz[v] - sH[s0][v][y][x])) * ihz;
            sH[s0][v][y][x] = hz[v];
          }
        }
      }
    }
    // ------------------------- C. x and y divergence of plane m - 1 (3D) / m (2D)
    // 3D: the threads outside the tile form it for every tile point, into
    // an LDS plane that the tile threads read one iteration later (after
    // the next barrier); the tile threads meanwhile go on to finish their
    // plane.  2D: the tile threads form it and use it at once.
    const int dm = m - 1;
    const int dbuf = buf ^ 1;
    T xyn[5] = {T(0), T(0), T(0), T(0), T(0)};
    auto xy_div = [&](int v, int px, int py) {
      const T ddx = (w1 * (sFX[dbuf][v][py][px + 3] - sFX[dbuf][v][py][px + 1]) -
                     w2 * (sFX[dbuf][v][py][px + 4] - sFX[dbuf][v][py][px])) * ihx;
      const T ddy = (w1 * (sFY[dbuf][v][py + 3][px] - sFY[dbuf][v][py + 1][px]) -
                     w2 * (sFY[dbuf][v][py + 4][px] - sFY[dbuf][v][py][px])) * ihy;
      return ddx + ddy;
    };
    if constexpr (three) {
      if (tid >= TX * TY && (dm - z0) >= 0 && (dm - z0) < nz) {
        constexpr int nthr = EX * EY - TX * TY;
        for (int i = tid - TX * TY; i < 5 * TX * TY; i += nthr) {
          const int v = i / (TX * TY), q = i % (TX * TY);
          const int px = q % TX, py = q / TX;
          if (px < nx && py < ny) sXY[dbuf][v][py][px] = xy_div(v, px, py);
        }
      }
    } else {
      if (core && (dm - z0) >= 0 && (dm - z0) < nz) {
#pragma unroll
        for (int v = 0; v < 5; ++v) xyn[v] = xy_div(v, x, y);
      }
    }
    // ------------------------------------------------- D. finish plane pz
    const int pz = three ? m - 2 : m - 1;
    if (core && pz >= z0 && pz < z0 + nz) {
      T R[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) R[v] = three ? -(sXY[buf][v][y][x] + zd[v]) : -xyn[v];
      T out[5];
      epilogue_pre<T, KIND, COMP>(p, gi, Yv, R, accv, u0v, out);
      if (pz + 1 < z0 + nz) {
        gi += gplane;
        if (needY) {
#pragma unroll
          for (int v = 0; v < 5; ++v) Yv[v] = p.Y[v * p.field + gi];
        }
        epilogue_load<T, KIND, COMP>(p, gi, accv, u0v);
      }
      if (ring_slot) ring_write_col(B, rcol, p.H, true, lx, ly, pz, out, ring_slot);
    }
  }
}

}  // namespace atns
