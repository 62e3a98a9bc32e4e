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
// Work decomposition (2.5D).  A workgroup of TX * TY threads owns a TX x TY
// column tile of one block and walks it along z.  Thread t owns tile column
// (t % TX, t / TX).  The footprint outside the tile is shared out as extra
// columns, so that every phase runs on the tile's own threads:
//   cross columns: 1-2 points outside the tile along x or y, 4 (TX + TY) of
//                  them, owned by threads 0, 1, ...; their gradients and one
//                  flux (x on the x-cross, y on the y-cross) are needed;
//   outer columns: 3-4 points out along x or y and the 2 x 2 xy corners,
//                  4 (TX + TY) + 16 of them, owned by the last threads; only
//                  their primitives (for the cross gradients) are needed.
// Tile and cross columns keep the primitives (u, v, w, T) of the planes
// m-2 .. m+2 around the gradient plane m in registers, so z-derivatives need
// no shared memory.  Per gradient plane m:
//   X. the tile and cross columns take in plane m+2 and write plane m to an
//      LDS plane of the footprint; the outer columns write plane m; the x/y
//      divergence of plane m-2 is formed from the flux planes of that plane;
//   --- barrier ---
//   Y. gradients at plane m: the tile point's z-flux completes the CD4
//      z-divergence of plane m-2; at the tile planes the x- and y-fluxes of
//      the tile and the cross go to LDS flux planes;
//   then plane m-2 is complete: RK epilogue and, in the last stage, the ring
//   write of the new boundary layers.
// The LDS planes are double-buffered by plane parity, so one barrier per plane
// orders everything: a buffer is rewritten two planes after it was read.
// This tile is the single-precision one; double precision, where the
// per-thread queues would need twice the registers, runs ns_wide.hpp.
// Each column's source (stage field or halo region) and its place in the
// ring's boundary layers are resolved once (column_source, ring_column).
#include "kernels_common.hpp"
#include "ns_wide.hpp"

namespace atns {

template <typename T, int TX, int TY>
struct NsShape {
  static constexpr int NT = TX * TY;               // threads: one per tile column
  static constexpr int EX = TX + 8, EY = TY + 8;   // footprint box
  static constexpr int NC = 4 * (TX + TY);         // cross columns
  static constexpr int NO = 4 * (TX + TY) + 16;    // outer columns and xy corners
  static constexpr int NB = 2;                     // LDS planes by plane parity
  // Row strides of the flux planes.  LDS serves a wave in two halves of 32
  // lanes over 32 banks.  A 32-wide tile puts one row in each half.  A
  // 16-wide tile gives each half the rows r and r + 2 (see ns_tile_lean), so
  // strides with 2 x stride = 16 (mod 32) keep the two rows on disjoint banks:
  // 24 for the footprint plane (TX + 8) and, padded, for both flux planes.
  static constexpr int FXS = TX == 16 ? 24 : TX + 4;
  static constexpr int FYS = TX == 16 ? 24 : TX;
};

// LDS of a tile: the block descriptor, the primitive plane of the footprint
// and the x/y flux planes.  One object per (T, TX, TY), shared by every stage
// kind a kernel instantiates.
template <typename T, int TX, int TY>
struct NsLds {
  using S = NsShape<T, TX, TY>;
  BlockDev B;
  T P[S::NB][4][S::EY][S::EX];   // u, v, w, T of the gradient plane
  T FX[S::NB][5][TY][S::FXS];      // F - Fv_x/Re on the x-cross of the plane
  T FY[S::NB][5][TY + 4][S::FYS];  // G - Fv_y/Re on the y-cross of the plane
};
template <typename T, int TX, int TY>
__device__ __forceinline__ NsLds<T, TX, TY>& ns_lds() {
  __shared__ NsLds<T, TX, TY> s;
  return s;
}

// A footprint column of a tile: tile-local position, flux direction (cross
// columns: 0 for x, 1 for y) and whether it is in use.
struct NsCol {
  int x, y, dir;
  bool on;
};

// A ragged tile (nx < TX or ny < TY): apron columns beyond the nominal tile
// move in to the real edge; columns between the real and the nominal edge
// have no work.
template <int TX, int TY>
__device__ __forceinline__ NsCol place_column(int x, int y, int dir, int nx, int ny) {
  const bool idle = (x >= nx && x < TX) || (y >= ny && y < TY);
  return NsCol{x >= TX ? x - (TX - nx) : x, y >= TY ? y - (TY - ny) : y, dir, !idle};
}

// Cross column c: x-cross first (2 columns on each side of the TY rows),
// then the y-cross.
template <int TX, int TY>
__device__ __forceinline__ NsCol cross_column(int c, int nx, int ny) {
  if (c < 4 * TY) {
    const int side = c / (2 * TY), q = c % (2 * TY);
    return place_column<TX, TY>(side ? TX + (q & 1) : -1 - (q & 1), q >> 1, 0, nx, ny);
  }
  const int r = c - 4 * TY;
  const int side = r / (2 * TX), q = r % (2 * TX);
  return place_column<TX, TY>(q % TX, side ? TY + q / TX : -1 - q / TX, 1, nx, ny);
}

// Outer column o: 3-4 points out along x, then along y, then the 2 x 2
// corners next to the tile's corners.
template <int TX, int TY>
__device__ __forceinline__ NsCol outer_column(int o, int nx, int ny) {
  if (o < 4 * TY) {
    const int side = o / (2 * TY), q = o % (2 * TY);
    return place_column<TX, TY>(side ? TX + 2 + (q & 1) : -3 - (q & 1), q >> 1, 0, nx, ny);
  }
  if (o < 4 * (TX + TY)) {
    const int r = o - 4 * TY;
    const int side = r / (2 * TX), q = r % (2 * TX);
    return place_column<TX, TY>(q % TX, side ? TY + 2 + q / TX : -3 - q / TX, 0, nx, ny);
  }
  const int r = o - 4 * (TX + TY);
  const int c = r >> 2, q = r & 3;
  return place_column<TX, TY>((c & 1) ? TX + (q & 1) : -1 - (q & 1), (c & 2) ? TY + (q >> 1) : -1 - (q >> 1), 0,
                              nx, ny);
}

// Element idx of an array whose base is the same for the whole workgroup:
// a 32-bit byte offset from the base, so the address needs no 64-bit
// arithmetic per thread (idx * sizeof(T) < 2^32).
template <typename T>
__device__ __forceinline__ const T& at_off(const T* base, unsigned idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T& at_off(T* base, unsigned idx) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (unsigned)sizeof(T));
}

// Where a footprint column reads its planes 0 <= lz < s_z from
// (column_source) with 32-bit strides: plane lz, variable v at
// base + lz * zs + v * vs.  Planes outside the block go through fetch().
template <typename T>
struct NsSrc {
  const T* base;
  int zs, vs;
};
template <typename T>
__device__ __forceinline__ NsSrc<T> ns_source(const StageParams<T>& p, const BlockDev* __restrict__ B, int lx,
                                              int ly) {
  const ColumnSource<T> c = column_source(p, B, lx, ly);
  return NsSrc<T>{c.base, (int)c.zs, (int)c.vs};
}
template <typename T>
__device__ __forceinline__ void ns_load(const StageParams<T>& p, const BlockDev* __restrict__ B, const NsSrc<T>& c,
                                        int blk, int lx, int ly, int lz, T u[5]) {
  if (lz >= 0 && lz < B->s[2]) {
    const T* r = c.base + lz * c.zs;
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = r[v * c.vs];
  } else {
    fetch(p, B, blk, lx, ly, lz, u);
  }
}

// The same point's primitives, gradients and fluxes are computed by
// different threads and code paths depending on the tile shape (as a tile,
// cross or outer column).  The fused multiply-adds below are written out and
// no other contraction is allowed, so every path gives the same bits and
// results do not depend on the tile shape.

// Primitives (u, v, w, T) and density of a conserved point.
template <typename T>
__device__ __forceinline__ void ns_prims(const T c[5], T gm1, T gM2, T q[4], T& rho) {
#pragma clang fp contract(off)
  const T ir = recip(c[0]);
  const T vx = c[1] * ir, vy = c[2] * ir, vz = c[3] * ir;
  const T ke = fma(c[3], vz, fma(c[2], vy, c[1] * vx));
  const T pr = gm1 * fma(T(-0.5), ke, c[4]);
  q[0] = vx;
  q[1] = vy;
  q[2] = vz;
  q[3] = (gM2 * pr) * ir;
  rho = c[0];
}

// Central difference of Eq. 2 from the neighbours at +1, -1, +2, -2:
// (w1 (f1 - f_1) - w2 (f2 - f_2)) * s.
template <typename T>
__device__ __forceinline__ T ns_cd(T p1, T m1, T p2, T m2, T w1, T w2, T s) {
#pragma clang fp contract(off)
  return fma(w1, p1 - m1, -(w2 * (p2 - m2))) * s;
}

// Gradient state at one point and its viscous-inviscid fluxes.
template <typename T>
struct NsGrad {
  T g[3][3];   // g[i][j] = d u_i / d x_j
  T gT[3];
  T vel[3];
  T rho, pres, et, div;
};

// Inviscid minus viscous flux along direction d: rho u_d, rho u_i u_d + p
// delta_id - tau_id / Re, (rho E + p) u_d - (u_j tau_dj + kappa dT/dx_d) / Re.
template <typename T>
__device__ __forceinline__ void ns_flux(const NsGrad<T>& s, int d, T ire, T kap, T two3, T out[5]) {
#pragma clang fp contract(off)
  T tau[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) tau[j] = d == j ? fma(-two3, s.div, s.g[d][j] + s.g[j][d]) : s.g[d][j] + s.g[j][d];
  const T ud = s.vel[d];
  const T mu = s.rho * ud;
  out[0] = mu;
#pragma unroll
  for (int i = 0; i < 3; ++i) out[1 + i] = fma(mu, s.vel[i], (i == d ? s.pres : T(0)) - ire * tau[i]);
  const T work = fma(s.vel[0], tau[0], fma(s.vel[1], tau[1], fma(s.vel[2], tau[2], kap * s.gT[d])));
  out[4] = fma(s.et + s.pres, ud, -(ire * work));
}

template <typename T, int TX, int TY, int KIND, int NDIM, bool CD2, bool COMP>
__device__ __forceinline__ void ns_tile_lean(const StageParams<T>& p, const TileDev t) {
#pragma clang fp contract(off)
  using S = NsShape<T, TX, TY>;
  static_assert(sizeof(T) == 4, "the lean tile is the single-precision one");
  constexpr bool three = (NDIM == 3);
  if (t.nx == 0) return;
  // The block descriptor lives in LDS for the whole kernel: re-reading it from
  // global memory inside the plane loop would make every such load wait for
  // all outstanding (prefetch) loads.
  NsLds<T, TX, TY>& lds = ns_lds<T, TX, TY>();
  stage_block(p.blocks + t.blk, &lds.B);
  const BlockDev* __restrict__ B = &lds.B;
  auto& sP = lds.P;
  auto& sFX = lds.FX;
  auto& sFY = lds.FY;
  const int tid = threadIdx.x;
  const int nx = t.nx, ny = t.ny, z0 = t.z0, nz = t.nz;

  // ---- columns of this thread: tile, cross (optional), outer (optional)
  // 16-wide tiles: a wave's four rows go to its half-waves as {0, 2} and
  // {1, 3}, which with the row strides of NsShape avoids LDS bank conflicts
  int tx, ty;
  if constexpr (TX == 16) {
    const int lane = tid & 63, q = lane & 31;
    tx = q & 15;
    ty = (tid >> 6) * 4 + (q >> 4) * 2 + (lane >> 5);
  } else {
    tx = tid % TX;
    ty = tid / TX;
  }
  const bool tact = tx < nx && ty < ny;
  const NsCol cc = tid < S::NC ? cross_column<TX, TY>(tid, nx, ny) : NsCol{0, 0, 0, false};
  const NsCol oc = S::NT - 1 - tid < S::NO ? outer_column<TX, TY>(S::NT - 1 - tid, nx, ny) : NsCol{0, 0, 0, false};
  const bool cact = cc.on, oact = oc.on;
  const int cx = cc.x, cy = cc.y, cdir = cc.dir, ox = oc.x, oy = oc.y;
  const int lx = t.x0 + tx, ly = t.y0 + ty;
  NsSrc<T> ccross{}, couter{};
  if (cact) ccross = ns_source(p, B, t.x0 + cx, t.y0 + cy);
  if (oact) couter = ns_source(p, B, t.x0 + ox, t.y0 + oy);

  const T gm1 = (T)(p.gamma - 1.0);
  const T gM2 = (T)p.mach2_gamma;
  const T kap = (T)p.kappa;
  const T ire = (T)p.inv_re;
  const T ihx = (T)p.dscale[0], ihy = (T)p.dscale[1], ihz = (T)p.dscale[2];
  // central-difference weights of the inner and outer neighbour pairs, known
  // at compile time (w2 = 1 multiplies away for CD4)
  constexpr T w1 = CD2 ? T(1) : T(8), w2 = CD2 ? T(0) : T(1);
  const T two3 = (T)(2.0 / 3.0);
  const T igM2 = (T)(1.0 / p.mach2_gamma), igm1 = (T)(1.0 / (p.gamma - 1.0));

  // Gradient at footprint point (x, y) of plane m from the LDS plane (x, y
  // derivatives) and the column's z-queue (planes m-2 .. m+2 in slots 0..4).
  auto gradient = [&](int b, int x, int y, const T* qu, const T* qv, const T* qw, const T* qT, T rho, NsGrad<T>& s) {
    const int sx = x + 4, sy = y + 4;
    const T* qs[4] = {qu, qv, qw, qT};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const T ddx = ns_cd(sP[b][c][sy][sx + 1], sP[b][c][sy][sx - 1], sP[b][c][sy][sx + 2], sP[b][c][sy][sx - 2],
                          w1, w2, ihx);
      const T ddy = ns_cd(sP[b][c][sy + 1][sx], sP[b][c][sy - 1][sx], sP[b][c][sy + 2][sx], sP[b][c][sy - 2][sx],
                          w1, w2, ihy);
      T ddz = T(0);
      if constexpr (three) {
        const T* q = qs[c];
        ddz = ns_cd(q[3], q[1], q[4], q[0], w1, w2, ihz);
      }
      if (c < 3) {
        s.g[c][0] = ddx;
        s.g[c][1] = ddy;
        s.g[c][2] = ddz;
      } else {
        s.gT[0] = ddx;
        s.gT[1] = ddy;
        s.gT[2] = ddz;
      }
    }
    s.div = (s.g[0][0] + s.g[1][1]) + s.g[2][2];
    s.vel[0] = qu[2];
    s.vel[1] = qv[2];
    s.vel[2] = qw[2];
    s.rho = rho;
    s.pres = (rho * qT[2]) * igM2;
    const T v2 = fma(s.vel[2], s.vel[2], fma(s.vel[1], s.vel[1], s.vel[0] * s.vel[0]));
    s.et = fma(s.pres, igm1, (T(0.5) * rho) * v2);
  };
  auto put_fx = [&](int b, int x, int y, const T f[5]) {
#pragma unroll
    for (int v = 0; v < 5; ++v) sFX[b][v][y][x + 2] = f[v];
  };
  auto put_fy = [&](int b, int x, int y, const T f[5]) {
#pragma unroll
    for (int v = 0; v < 5; ++v) sFY[b][v][y + 2][x] = f[v];
  };
  // x/y divergence of the tile point's fluxes from flux planes b
  auto xy_div = [&](int b, T out[5]) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const T ddx = ns_cd(sFX[b][v][ty][tx + 3], sFX[b][v][ty][tx + 1], sFX[b][v][ty][tx + 4], sFX[b][v][ty][tx],
                          w1, w2, ihx);
      const T ddy = ns_cd(sFY[b][v][ty + 3][tx], sFY[b][v][ty + 1][tx], sFY[b][v][ty + 4][tx], sFY[b][v][ty][tx],
                          w1, w2, ihy);
      out[v] = ddx + ddy;
    }
  };

  // ---- tile column loads, epilogue operands, ring write
  // A tile column lies inside the block in x and y.  Its planes in the block
  // come from the stage field; planes beyond the block's z faces from the
  // z-face halo regions (delayed halos) or the periodic stage field
  // (synchronous).  The plane's base is the same for the whole workgroup;
  // each thread adds its in-plane offset.
  const long long gplane = (long long)p.n[0] * p.n[1];
  const unsigned toff = (unsigned)((B->o[1] + ly) * p.n[0] + (B->o[0] + lx));   // in the field plane
  const unsigned tfoff = (unsigned)(ly * B->s[0] + lx);                          // in a z-face layer
  auto tile_load = [&](int lz, T u[5]) {
    const T* base;
    long long vs;
    unsigned off;
    if (lz >= 0 && lz < B->s[2]) {
      base = p.Y + (long long)(B->o[2] + lz) * gplane;
      vs = p.field;
      off = toff;
    } else if (p.halo == kHaloSync) {
      base = p.Y + (long long)wrap(B->o[2] + lz, p.n[2]) * gplane;
      vs = p.field;
      off = toff;
    } else {
      const long long lay = (long long)B->s[0] * B->s[1];
      const int iz = lz < 0 ? lz + p.H : lz - B->s[2];
      base = p.hbuf + B->hoff[lz < 0 ? 4 : 5] + iz * lay;
      vs = lay * p.H;
      off = tfoff;
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = at_off(base + v * vs, off);
  };
  // the stage input at the point enters only the first RK4 stage and the
  // low-storage updates; the RK registers by stage kind as in epilogue_pre
  constexpr bool needY = KIND == kRK4First || KIND == kLSFirst || KIND == kLSMid || KIND == kRhsOnly;
  constexpr bool needA = KIND == kRK4Mid || KIND == kRK4Last || KIND == kLSMid;
  // the compensated last RK4 stage (COMP) also reads U^n and the carried
  // error, at the update itself rather than a plane ahead: their registers
  // would not fit beside the z-queues
  static_assert(!COMP || KIND == kRK4Last, "compensation is a last-RK4-stage variant");
  constexpr bool needU0 = KIND == kRK4Mid;
  T Yv[5] = {T(0), T(0), T(0), T(0), T(0)}, accv[5] = {T(0), T(0), T(0), T(0), T(0)};
  T u0v[5] = {T(0), T(0), T(0), T(0), T(0)};
  auto epi_load = [&](int pz) {
    const long long zo = (long long)(B->o[2] + pz) * gplane;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const long long o = v * p.field + zo;
      if (needY) Yv[v] = at_off(p.Y + o, toff);
      if (needA) accv[v] = at_off(p.acc + o, toff);
      if (needU0) u0v[v] = at_off(p.U0 + o, toff);
    }
  };
  if (tact) epi_load(z0);
  // only the last stage of a step writes the ring: the last classical RK4
  // stage, or a low-storage middle stage (the last of LSERK2 and LSERK4)
  constexpr bool may_ring = KIND == kRK4Last || KIND == kLSMid;
  T* ring_slot = nullptr;
  if (may_ring && p.ring_write) ring_slot = p.ring + (long long)((p.slot_now + 1) % p.D) * p.slot_stride;
  // finish tile plane pz (block-local) with the x/y divergence xyd and the
  // z-divergence zd of its fluxes: the RK update of epilogue_pre
  auto finish = [&](int pz, const T xyd[5], const T zd[5]) {
    T out[5];
    if (tact) {
      const T dt = (T)p.dt, cA = (T)p.cA, cB = (T)p.cB;
      const long long zo = (long long)(B->o[2] + pz) * gplane;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const long long o = v * p.field + zo;
        const T r = -(xyd[v] + zd[v]);   // R = -(D_x F + D_y G + D_z H)
        if (KIND == kRhsOnly) {
          out[v] = r;
        } else if (KIND == kRK4First) {
          const T dr = dt * r;
          at_off(p.acc + o, toff) = cA * dr;
          out[v] = fma(cB, dr, Yv[v]);
        } else if (KIND == kRK4Mid) {
          const T dr = dt * r;
          const T a = fma(cA, dr, accv[v]);
          at_off(p.acc + o, toff) = p.fold ? u0v[v] + a : a;
          out[v] = fma(cB, dr, u0v[v]);
        } else if (KIND == kRK4Last) {
          if constexpr (COMP) {
            T c = at_off(p.comp + o, toff);
            out[v] = comp_add<T>(at_off(p.U0 + o, toff), fma(cA, dt * r, accv[v]), c);
            at_off(p.comp + o, toff) = c;
          } else {
            out[v] = fma(cA, dt * r, accv[v]);
          }
        } else if (KIND == kLSFirst) {
          const T q = dt * r;
          at_off(p.acc + o, toff) = q;
          out[v] = fma(cB, q, Yv[v]);
        } else {   // kLSMid
          const T q = fma(cA, accv[v], dt * r);
          at_off(p.acc + o, toff) = q;
          out[v] = fma(cB, q, Yv[v]);
        }
        at_off(p.Yout + o, toff) = out[v];
      }
      if (pz + 1 < z0 + nz) epi_load(pz + 1);
    }
    // the column's layers are resolved here, per plane, rather than held in
    // registers across the plane loop
    if constexpr (may_ring)
      if (ring_slot && tact) ring_write_col(B, ring_column(B, p.H, lx, ly), p.H, true, lx, ly, pz, out, ring_slot);
  };

  if constexpr (!three) {
    // ------------------------------------------------------------ 2-D: one plane
    T ct[5] = {T(1), T(0), T(0), T(0), T(1)}, cc[5] = {T(1), T(0), T(0), T(0), T(1)};
    T co[5] = {T(1), T(0), T(0), T(0), T(1)};
    if (tact) tile_load(0, ct);
    if (cact) ns_load(p, B, ccross, t.blk, t.x0 + cx, t.y0 + cy, 0, cc);
    if (oact) ns_load(p, B, couter, t.blk, t.x0 + ox, t.y0 + oy, 0, co);
    T qt[4], qc[4], qo[4], rt, rc, ro;
    ns_prims(ct, gm1, gM2, qt, rt);
    ns_prims(cc, gm1, gM2, qc, rc);
    ns_prims(co, gm1, gM2, qo, ro);
    if (tact) {
#pragma unroll
      for (int c = 0; c < 4; ++c) sP[0][c][ty + 4][tx + 4] = qt[c];
    }
    if (cact) {
#pragma unroll
      for (int c = 0; c < 4; ++c) sP[0][c][cy + 4][cx + 4] = qc[c];
    }
    if (oact) {
#pragma unroll
      for (int c = 0; c < 4; ++c) sP[0][c][oy + 4][ox + 4] = qo[c];
    }
    lds_barrier();
    T zq[5] = {T(0), T(0), T(0), T(0), T(0)};
    if (tact) {
      T u5[5] = {T(0), T(0), qt[0], T(0), T(0)}, v5[5] = {T(0), T(0), qt[1], T(0), T(0)};
      T w5[5] = {T(0), T(0), qt[2], T(0), T(0)}, T5[5] = {T(0), T(0), qt[3], T(0), T(0)};
      NsGrad<T> s;
      gradient(0, tx, ty, u5, v5, w5, T5, rt, s);
      T f[5];
      ns_flux(s, 0, ire, kap, two3, f);
      put_fx(0, tx, ty, f);
      ns_flux(s, 1, ire, kap, two3, f);
      put_fy(0, tx, ty, f);
    }
    if (cact) {
      T u5[5] = {T(0), T(0), qc[0], T(0), T(0)}, v5[5] = {T(0), T(0), qc[1], T(0), T(0)};
      T w5[5] = {T(0), T(0), qc[2], T(0), T(0)}, T5[5] = {T(0), T(0), qc[3], T(0), T(0)};
      NsGrad<T> s;
      gradient(0, cx, cy, u5, v5, w5, T5, rc, s);
      T f[5];
      if (cdir == 0) {
        ns_flux(s, 0, ire, kap, two3, f);
        put_fx(0, cx, cy, f);
      } else {
        ns_flux(s, 1, ire, kap, two3, f);
        put_fy(0, cx, cy, f);
      }
    }
    lds_barrier();
    T xyd[5] = {T(0), T(0), T(0), T(0), T(0)};
    if (tact) xy_div(0, xyd);
    finish(0, xyd, zq);
    return;
  } else {
    // ------------------------------------------------------------ 3-D: walk z
    // z-queues: q*[j] holds plane m-2+j of the column at gradient plane m;
    // r*[j] the density of plane m+j
    T tu[5], tv[5], tw[5], tT[5], tr[3];
    T cu[5], cv[5], cw[5], cT[5], cr[3];
#pragma unroll
    for (int j = 0; j < 5; ++j) tu[j] = tv[j] = tw[j] = tT[j] = cu[j] = cv[j] = cw[j] = cT[j] = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) tr[j] = cr[j] = T(1);
    // z-fluxes of the tile point at planes m-4 .. m-1
    T hq[4][5];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 5; ++v) hq[j][v] = T(0);

    auto push = [&](T* qu, T* qv, T* qw, T* qT, T* qr, const T c[5], bool live) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        qu[j] = qu[j + 1];
        qv[j] = qv[j + 1];
        qw[j] = qw[j + 1];
        qT[j] = qT[j + 1];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) qr[j] = qr[j + 1];
      if (live) {
        T q[4], r;
        ns_prims(c, gm1, gM2, q, r);
        qu[4] = q[0];
        qv[4] = q[1];
        qw[4] = q[2];
        qT[4] = q[3];
        qr[2] = r;
      }
    };
    // planes the columns need: tile z0-4 .. z0+nz+3, cross z0-2 .. z0+nz+1,
    // outer z0 .. z0+nz-1
    auto tile_need = [&](int f) { return tact && f >= z0 - 4 && f < z0 + nz + 4; };
    auto cross_need = [&](int f) { return cact && f >= z0 - 2 && f < z0 + nz + 2; };
    auto outer_need = [&](int f) { return oact && f >= z0 && f < z0 + nz; };

    T nt[5] = {T(1), T(0), T(0), T(0), T(1)}, nc[5] = {T(1), T(0), T(0), T(0), T(1)};
    T no[5] = {T(1), T(0), T(0), T(0), T(1)};
    // prologue: planes z0-4 .. z0-1 into the queues, z0 in flight
    for (int j = 0; j < 4; ++j) {
      const int f = z0 - 4 + j;
      T c[5] = {T(1), T(0), T(0), T(0), T(1)};
      if (tile_need(f)) tile_load(f, c);
      push(tu, tv, tw, tT, tr, c, tile_need(f));
      T d[5] = {T(1), T(0), T(0), T(0), T(1)};
      if (cross_need(f)) ns_load(p, B, ccross, t.blk, t.x0 + cx, t.y0 + cy, f, d);
      push(cu, cv, cw, cT, cr, d, cross_need(f));
    }
    if (tile_need(z0)) tile_load(z0, nt);
    if (cross_need(z0)) ns_load(p, B, ccross, t.blk, t.x0 + cx, t.y0 + cy, z0, nc);
    if (outer_need(z0)) ns_load(p, B, couter, t.blk, t.x0 + ox, t.y0 + oy, z0, no);

    T xyd[5] = {T(0), T(0), T(0), T(0), T(0)};   // x/y divergence of plane m-2
    for (int m = z0 - 2; m < z0 + nz + 2; ++m) {
      const int b = m & 1;
      const bool mtile = m >= z0 && m < z0 + nz;
      // ------------------------------------------------------- phase X
      const int e = m + 2;   // plane entering the tile and cross queues
      push(tu, tv, tw, tT, tr, nt, tile_need(e));
      push(cu, cv, cw, cT, cr, nc, cross_need(e));
      if (tile_need(e + 1)) tile_load(e + 1, nt);
      if (cross_need(e + 1)) ns_load(p, B, ccross, t.blk, t.x0 + cx, t.y0 + cy, e + 1, nc);
      if (tact) {
        sP[b][0][ty + 4][tx + 4] = tu[2];
        sP[b][1][ty + 4][tx + 4] = tv[2];
        sP[b][2][ty + 4][tx + 4] = tw[2];
        sP[b][3][ty + 4][tx + 4] = tT[2];
      }
      if (cross_need(m)) {
        sP[b][0][cy + 4][cx + 4] = cu[2];
        sP[b][1][cy + 4][cx + 4] = cv[2];
        sP[b][2][cy + 4][cx + 4] = cw[2];
        sP[b][3][cy + 4][cx + 4] = cT[2];
      }
      if (outer_need(m)) {
        T q[4], r;
        ns_prims(no, gm1, gM2, q, r);
#pragma unroll
        for (int c = 0; c < 4; ++c) sP[b][c][oy + 4][ox + 4] = q[c];
        if (outer_need(m + 1)) ns_load(p, B, couter, t.blk, t.x0 + ox, t.y0 + oy, m + 1, no);
      }
      // fluxes of plane m-2 were written two planes ago
      if (tact && m - 2 >= z0) xy_div(b, xyd);
      lds_barrier();
      // ------------------------------------------------------- phase Y
      T zd[5] = {T(0), T(0), T(0), T(0), T(0)};   // z-divergence of plane m-2
      if (tact) {
        NsGrad<T> s;
        gradient(b, tx, ty, tu, tv, tw, tT, tr[0], s);
        T hz[5];
        ns_flux(s, 2, ire, kap, two3, hz);
        // the z-flux of plane m completes the CD4 z-divergence of plane m-2
        // with those of planes m-4, m-3 and m-1
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          zd[v] = ns_cd(hq[3][v], hq[1][v], hz[v], hq[0][v], w1, w2, ihz);
          hq[0][v] = hq[1][v];
          hq[1][v] = hq[2][v];
          hq[2][v] = hq[3][v];
          hq[3][v] = hz[v];
        }
        if (mtile) {
          T f[5];
          ns_flux(s, 0, ire, kap, two3, f);
          put_fx(b, tx, ty, f);
          ns_flux(s, 1, ire, kap, two3, f);
          put_fy(b, tx, ty, f);
        }
      }
      if (cact && mtile) {
        NsGrad<T> s;
        gradient(b, cx, cy, cu, cv, cw, cT, cr[0], s);
        T f[5];
        if (cdir == 0) {
          ns_flux(s, 0, ire, kap, two3, f);
          put_fx(b, cx, cy, f);
        } else {
          ns_flux(s, 1, ire, kap, two3, f);
          put_fy(b, cx, cy, f);
        }
      }
      // ------------------------------------------ plane m-2 is complete
      if (m - 2 >= z0) finish(m - 2, xyd, zd);
    }
  }
}

// Threads of a Navier-Stokes workgroup, and the tile function: one thread
// per tile column in single precision; one per footprint point in double
// precision (ns_wide.hpp).
template <typename T, int TX, int TY>
constexpr int ns_threads() {
  return sizeof(T) == 4 ? TX * TY : (TX + 8) * (TY + 8);
}
template <typename T, int TX, int TY, int KIND, int NDIM, bool COMP = false>
__device__ __forceinline__ void ns_tile(const StageParams<T>& p, const TileDev t) {
  if constexpr (sizeof(T) == 4) {
    if (p.cd2)
      ns_tile_lean<T, TX, TY, KIND, NDIM, true, COMP>(p, t);
    else
      ns_tile_lean<T, TX, TY, KIND, NDIM, false, COMP>(p, t);
  } else
    ns_tile_wide<T, TX, TY, KIND, NDIM, COMP>(p, t);
}

// Single precision: at least three waves per SIMD (at most 168 registers),
// which with three workgroups per CU (their LDS) keeps 12 waves per CU.
template <typename T>
constexpr int ns_min_waves() {
  return sizeof(T) == 4 ? 3 : 1;
}

template <typename T, int TX, int TY, int KIND, int NDIM, bool COMP = false>
__global__ void __launch_bounds__((ns_threads<T, TX, TY>())) __attribute__((amdgpu_waves_per_eu(ns_min_waves<T>())))
ns_stage_kernel(const StageParams<T> p) {
  const StageParams<T> q = resolve_step(p);
  ns_tile<T, TX, TY, KIND, NDIM, COMP>(q, p.tiles[blockIdx.x]);
  if (p.step_end) finish_step(p.step_end, p.done);
}

// Persistent form for a batch (see the Euler kernel).
template <typename T, int TX, int TY, int KIND>
__global__ void __launch_bounds__((ns_threads<T, TX, TY>()))
    ns_batch_kernel(const StageParams<T>* __restrict__ ps, const BatchTile* __restrict__ tl, int ntiles) {
  __shared__ StageParams<T> sp;
  for (int i = blockIdx.x; i < ntiles; i += gridDim.x) {
    const BatchTile bt = tl[i];
    __syncthreads();
    stage_struct(ps + bt.inst, &sp);
    if (threadIdx.x == 0 && sp.nstep) sp = resolve_step(sp);
    __syncthreads();
    ns_tile<T, TX, TY, KIND, 3>(sp, bt.t);
  }
}

// Free-running asynchronous steps of a 3-D Navier-Stokes context (see
// async_run).
template <typename T, int TX, int TY, int S, int CL>
__global__ void __launch_bounds__((ns_threads<T, TX, TY>()))
    ns_async_kernel(const StageParams<T>* __restrict__ ps, const AsyncArgs a) {
  __shared__ StageParams<T> sp;
  async_run<T, S, CL>(ps, a, sp, [](const StageParams<T>& q, const TileDev& td, int e) {
    if constexpr (S == 2) {
      if (e == 0)
        ns_tile<T, TX, TY, kLSFirst, 3>(q, td);
      else
        ns_tile<T, TX, TY, kLSMid, 3>(q, td);
    } else {
      if (e == 0)
        ns_tile<T, TX, TY, kRK4First, 3>(q, td);
      else if (e == S - 1)
        ns_tile<T, TX, TY, kRK4Last, 3>(q, td);
      else
        ns_tile<T, TX, TY, kRK4Mid, 3>(q, td);
    }
  });
}

template <typename T, int TX, int TY>
hipError_t launch_ns_async_shape(const StageParams<T>* ps, const AsyncArgs& a, int stages, hipStream_t s,
                                 int* resident) {
  const void* fn = stages == 2 ? (const void*)ns_async_kernel<T, TX, TY, 2, 3>
                               : (const void*)ns_async_kernel<T, TX, TY, 4, 5>;
  if (resident) return hipOccupancyMaxActiveBlocksPerMultiprocessor(resident, fn, ns_threads<T, TX, TY>(), 0);
  dim3 g(a.nb), b(ns_threads<T, TX, TY>());
  if (stages == 2)
    ns_async_kernel<T, TX, TY, 2, 3><<<g, b, 0, s>>>(ps, a);
  else
    ns_async_kernel<T, TX, TY, 4, 5><<<g, b, 0, s>>>(ps, a);
  return hipGetLastError();
}

// With resident != nullptr: only report how many workgroups of the kernel
// fit on one CU (nothing is launched).
template <typename T>
hipError_t launch_ns_async(const StageParams<T>* ps, const AsyncArgs& a, int stages, int tx, int ty, hipStream_t s,
                           int* resident) {
  if (stages != 2 && stages != 4) return hipErrorInvalidValue;
  if (tx == 16 && ty == 16) return launch_ns_async_shape<T, 16, 16>(ps, a, stages, s, resident);
  if (tx == 32 && ty == 8) return launch_ns_async_shape<T, 32, 8>(ps, a, stages, s, resident);
  if (tx == 16 && ty == 8) return launch_ns_async_shape<T, 16, 8>(ps, a, stages, s, resident);
  if constexpr (sizeof(T) == 4)   // 32 x 16 in single precision only (LDS)
    if (tx == 32 && ty == 16) return launch_ns_async_shape<T, 32, 16>(ps, a, stages, s, resident);
  return hipErrorInvalidValue;
}
template hipError_t launch_ns_async<float>(const StageParams<float>*, const AsyncArgs&, int, int, int, hipStream_t,
                                           int*);
template hipError_t launch_ns_async<double>(const StageParams<double>*, const AsyncArgs&, int, int, int, hipStream_t,
                                            int*);

template <typename T, int TX, int TY>
hipError_t launch_ns_batch_shape(const StageParams<T>* ps, const BatchTile* tl, int ntiles, int grid, int kind,
                                 hipStream_t s, int* resident) {
  if (resident) {   // the least over the three stage kinds
    const void* fns[3] = {(const void*)ns_batch_kernel<T, TX, TY, kRK4First>, (const void*)ns_batch_kernel<T, TX, TY, kRK4Mid>,
                          (const void*)ns_batch_kernel<T, TX, TY, kRK4Last>};
    int least = 1 << 30;
    for (const void* f : fns) {
      int r = 0;
      const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, f, ns_threads<T, TX, TY>(), 0);
      if (e != hipSuccess) return e;
      least = r < least ? r : least;
    }
    *resident = least;
    return hipSuccess;
  }
  dim3 g(grid), b(ns_threads<T, TX, TY>());
  switch (kind) {
    case kRK4First: ns_batch_kernel<T, TX, TY, kRK4First><<<g, b, 0, s>>>(ps, tl, ntiles); break;
    case kRK4Mid: ns_batch_kernel<T, TX, TY, kRK4Mid><<<g, b, 0, s>>>(ps, tl, ntiles); break;
    case kRK4Last: ns_batch_kernel<T, TX, TY, kRK4Last><<<g, b, 0, s>>>(ps, tl, ntiles); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// With resident != nullptr: only report how many workgroups of the kernel
// fit on one CU (the least over its stage kinds).
template <typename T>
hipError_t launch_ns_batch(const StageParams<T>* ps, const BatchTile* tl, int ntiles, int grid, int kind, int tx,
                           int ty, hipStream_t s, int* resident) {
  if (tx == 16 && ty == 16) return launch_ns_batch_shape<T, 16, 16>(ps, tl, ntiles, grid, kind, s, resident);
  if (tx == 32 && ty == 8) return launch_ns_batch_shape<T, 32, 8>(ps, tl, ntiles, grid, kind, s, resident);
  if (tx == 16 && ty == 8) return launch_ns_batch_shape<T, 16, 8>(ps, tl, ntiles, grid, kind, s, resident);
  if constexpr (sizeof(T) == 4)   // 32 x 16 in single precision only (LDS)
    if (tx == 32 && ty == 16) return launch_ns_batch_shape<T, 32, 16>(ps, tl, ntiles, grid, kind, s, resident);
  return hipErrorInvalidValue;
}
template hipError_t launch_ns_batch<float>(const StageParams<float>*, const BatchTile*, int, int, int, int, int,
                                           hipStream_t, int*);
template hipError_t launch_ns_batch<double>(const StageParams<double>*, const BatchTile*, int, int, int, int, int,
                                            hipStream_t, int*);

template <typename T, int KIND, int TX, int TY, bool COMP = false>
hipError_t launch_ns_kind(const StageParams<T>& p, int ntiles, hipStream_t s) {
  dim3 grid(ntiles), block(ns_threads<T, TX, TY>());
  if (p.ndim == 3)
    ns_stage_kernel<T, TX, TY, KIND, 3, COMP><<<grid, block, 0, s>>>(p);
  else
    ns_stage_kernel<T, TX, TY, KIND, 2, COMP><<<grid, block, 0, s>>>(p);
  return hipGetLastError();
}

template <typename T, int TX, int TY>
hipError_t launch_ns_shape(const StageParams<T>& p, int ntiles, int kind, hipStream_t s) {
  switch (kind) {
    case kRhsOnly: return launch_ns_kind<T, kRhsOnly, TX, TY>(p, ntiles, s);
    case kRK4First: return launch_ns_kind<T, kRK4First, TX, TY>(p, ntiles, s);
    case kRK4Mid: return launch_ns_kind<T, kRK4Mid, TX, TY>(p, ntiles, s);
    case kRK4Last:
      return p.comp ? launch_ns_kind<T, kRK4Last, TX, TY, true>(p, ntiles, s)
                    : launch_ns_kind<T, kRK4Last, TX, TY>(p, ntiles, s);
    case kLSFirst: return launch_ns_kind<T, kLSFirst, TX, TY>(p, ntiles, s);
    default: return launch_ns_kind<T, kLSMid, TX, TY>(p, ntiles, s);
  }
}

// Tile shapes (TX x TY) the Navier-Stokes kernel is built for.
template <typename T>
hipError_t launch_ns_stage(const StageParams<T>& p, int ntiles, int kind, int tx, int ty, hipStream_t s) {
  if (tx == 16 && ty == 16) return launch_ns_shape<T, 16, 16>(p, ntiles, kind, s);
  if (tx == 32 && ty == 8) return launch_ns_shape<T, 32, 8>(p, ntiles, kind, s);
  if (tx == 16 && ty == 8) return launch_ns_shape<T, 16, 8>(p, ntiles, kind, s);
  if constexpr (sizeof(T) == 4)   // 32 x 16 in single precision only (LDS)
    if (tx == 32 && ty == 16) return launch_ns_shape<T, 32, 16>(p, ntiles, kind, s);
  return hipErrorInvalidValue;
}

template hipError_t launch_ns_stage<float>(const StageParams<float>&, int, int, int, int, hipStream_t);
template hipError_t launch_ns_stage<double>(const StageParams<double>&, int, int, int, int, hipStream_t);

}  // namespace atns
