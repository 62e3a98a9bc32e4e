// Data layout shared by the library's host code and its kernels.
//
// State: structure of arrays, [5][nz][ny][nx], x fastest.
// Blocks: tensor-product index ranges of the global grid (the PEs).
// Ring: D slots; slot m % D holds the boundary layers of U^m of every block.
//   Within a slot, block b's layer for slot direction s (the points of b that
//   the neighbour in direction s reads as its halo) starts at lay[b][s] and
//   is stored [5][ez][ey][ex] with extent ed = depth where s has a nonzero
//   component in d, else the block size.  Faces have depth H (2 Euler,
//   4 Navier-Stokes), edges depth 2.  Readers find the values of their halo
//   region s in the layer opposite(s) of neighbour nbr[b][s], so every halo
//   read of a block face is one contiguous run.
#pragma once
#include <cstdint>

namespace atns {

constexpr int kNumSlots = 18;

// Slot direction table (matches the slot numbering of atns.h).
__host__ __device__ inline void slot_dir(int s, int d[3]) {
  const signed char t[18][3] = {{-1, 0, 0}, {1, 0, 0},  {0, -1, 0},  {0, 1, 0},  {0, 0, -1}, {0, 0, 1},
                                {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},  {1, 1, 0},  {-1, 0, -1}, {1, 0, -1},
                                {-1, 0, 1}, {1, 0, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}, {0, 1, 1}};
  d[0] = t[s][0];
  d[1] = t[s][1];
  d[2] = t[s][2];
}

// Slot index from per-axis signs (-1, 0, +1); -1 for the centre or a corner.
__host__ __device__ inline int slot_index(int sx, int sy, int sz) {
  const int nz = (sx != 0) + (sy != 0) + (sz != 0);
  if (nz == 1) {
    if (sx) return sx < 0 ? 0 : 1;
    if (sy) return sy < 0 ? 2 : 3;
    return sz < 0 ? 4 : 5;
  }
  if (nz == 2) {
    if (sz == 0) return 6 + (sx > 0) + 2 * (sy > 0);
    if (sy == 0) return 10 + (sx > 0) + 2 * (sz > 0);
    return 14 + (sy > 0) + 2 * (sz > 0);
  }
  return -1;
}

__host__ __device__ inline int slot_opposite(int s) {
  int d[3];
  slot_dir(s, d);
  return slot_index(-d[0], -d[1], -d[2]);
}

struct BlockDev {
  int o[3];                  // origin (global index of local (0,0,0))
  int s[3];                  // size
  int nbr[kNumSlots];        // neighbour block in each slot direction
  long long lay[kNumSlots];  // offset of this block's layer for slot s (-1: unused)
  long long hoff[kNumSlots]; // offset of this block's halo region s in a
                             // stage-halo buffer (-1: unused)
  long long roff[kNumSlots]; // offset in a ring slot of the neighbour's layer
                             // that feeds halo region s (-1: unused)
};

// One reader-side halo region: block b's halo in slot direction s, which is
// the layer opposite(s) of neighbour nbr[b][s] (same extents and order).
struct HaloRegion {
  long long dst;   // offset in a stage-halo buffer
  long long src;   // offset of the neighbour's layer in a ring slot
  int npts;        // points per variable
  int kidx;        // index of the delay: b * kNumSlots + s
};

// A chunk of up to kHaloChunk consecutive points of one region.
constexpr int kHaloChunk = 256;
struct HaloWork {
  int region;
  int start;
};

// Delay rule of a context for halo kernels that draw the step's delays
// themselves (draw != 0).
struct DelayDraw {
  int draw;
  int nblocks;
  int algo;
  unsigned long long seed;
};

struct TileDev {
  int blk;                  // block id
  short x0, y0, z0;         // tile origin, block-local
  short nx, ny, nz;         // tile extent (nx == 0: padding tile, no work)
};

// Free-running asynchronous steps (one persistent workgroup per block).
// Block b publishes prog[b] = m once ring level m of its boundary layers is
// written; a reader at step n takes from neighbour q the newest published
// level m = prog[q], i.e. the delay k = max(0, n - m), and waits while
// k > L - 1.  A wait longer than spin_limit polls sets *abort, and every
// workgroup then leaves.  log receives the realized delays,
// [step][block][slot] (-1 for unused slots).
struct AsyncArgs {
  int* prog;
  int* abort;
  int8_t* log;
  const HaloRegion* regions;
  const int* reg_begin;     // [nb + 1]: block b owns regions reg_begin[b] ..
  const TileDev* tiles;     // block-major tile list
  const int* tile_begin;    // [nb + 1]: block b owns tiles tile_begin[b] ..
  const double* W;          // halo weights [s][L][C]
  long long n0;             // step of the state at entry
  int nsteps;
  int nb;
  int D;
  int L;
  int stale;                // AS: the stale level instead of the AT sum
  long long slot_stride;
  long long spin_limit;
};

// A tile of one member of a batch.
struct BatchTile {
  int inst;      // member index
  TileDev t;
};

// Stage epilogue kinds.
enum StageKind {
  kRhsOnly = 0,   // Yout = R
  kRK4First = 1,  // acc = cA dt R     ; Yout = Y + cB dt R        (Y == U^n)
  kRK4Mid = 2,    // acc += cA dt R    ; Yout = U0 + cB dt R
                  //   (fold: acc = U0 + (acc + cA dt R))
  kRK4Last = 3,   // Yout = acc + cA dt R                          (Yout == U)
  kLSFirst = 4,   // Q = dt R          ; Yout = Y + cB Q           (A_1 = 0)
  kLSMid = 5      // Q = cA Q + dt R   ; Yout = Y + cB Q
};

enum HaloMode { kHaloSync = 0, kHaloStale = 1, kHaloAT = 2 };

template <typename T>
struct StageParams {
  const T* Y;          // stage input, read with the stencil
  const T* U0;         // RK4: U^n (pointwise)
  T* Yout;             // next stage input / final state
  T* acc;              // RK4 accumulator / LSERK Q register
  T* ring;             // ring base
  const T* hbuf;       // this stage's halo values (reader-side layout)
  const BlockDev* blocks;
  const TileDev* tiles;
  int n[3];              // global sizes
  long long field;       // nx*ny*nz, the variable stride
  long long slot_stride; // elements per ring slot
  int D;                 // ring depth
  int slot_now;          // n % D
  int halo;              // HaloMode for this stage
  // When nstep is set (graph-captured steps), n is read from this device
  // counter: slot_now = n % D and halo = (n >= C) ? async_halo : kHaloSync.
  const long long* nstep;
  int async_halo;
  // Set only for the last stage of a captured step: the workgroup that
  // finishes last (counted in *done) advances *step_end by one.
  long long* step_end;
  unsigned int* done;
  int L;
  int C;                 // delayed levels of the AT scheme (5 AT4, 3 AT2)
  int H;                 // halo depth (faces)
  int ndim;
  // Central difference of Eq. 2 from d1 = f(+1) - f(-1), d2 = f(+2) - f(-2):
  // (w1 d1 - w2 d2) * dscale, with w1 = 8, w2 = 1, dscale = 1/(12 h_d) for
  // CD4 and w1 = 1, w2 = 0, dscale = 1/(2 h_d) for CD2 (cd2 != 0).
  int cd2;
  double dscale[3];
  double gamma;
  double mach2_gamma;    // gamma * M^2          (T = gamma M^2 p / rho)
  double kappa;          // 1/((gamma-1) M^2 Pr)
  double inv_re;
  double dt;
  double cA;             // epilogue coefficients (see stage kinds)
  double cB;
  // Classical RK4 accumulates dt sum_j b_j R_j in acc starting from zero
  // and adds U^n once, in the last middle stage (fold != 0), which reads U^n
  // anyway: two roundings of state-sized sums per step instead of four, at
  // no extra traffic.
  int fold;
  // Compensated classical RK4 (comp != null, single-context steps): the
  // accumulator holds the step's increments only (fold stays 0) and the last
  // stage forms U^{n+1} = U^n + (increments + comp) with the sum's rounding
  // error kept in comp for the next step (TwoSum), so the state is carried
  // to about twice its precision.  U0 is U^n in the last stage too.
  T* comp;
  int ring_write;        // write the boundary layers of the result
  // Halo assembly inside the first stage of a graph-captured step (fuse_halo
  // != 0): before its plane loop, each tile computes, for the halo points it
  // reads, the values of all S stages (weights W, delays drawn by dd) into
  // the stage-halo buffers, in place of a separate halo kernel.
  int fuse_halo;
  int S;
  const double* W;
  DelayDraw dd;
};

// One pass of the tenth-order filter along axis dir: every block filters its
// lines of `in` into `out` (distinct buffers).  Halo points beyond a face
// come from `in` at the periodic neighbour position (synchronous) or from
// the filter-halo slot `fhalo` of the stage-halo buffer (delayed halos, same
// region layout as the stage halos).
template <typename T>
struct FilterArgs {
  const T* in;
  T* out;
  const BlockDev* blocks;
  const T* fhalo;        // filter-halo slot, or null when the context has none
  const double* inv;     // forward-elimination factors, rows 0..kFilterMaxLen-1
  const double* cp;
  int n[3];
  long long field;
  int H;                 // face depth of the halo regions
  int dir;
  int halo;              // HaloMode of the step
  // graph-captured steps: the step counter already advanced by the last
  // stage, so the step is *nstep - 1 and halo = (step >= C) ? async_halo :
  // kHaloSync
  const long long* nstep;
  int C;
  int async_halo;
  double ah[6];          // a_0, a_1/2, ..., a_5/2
  double alpha;
  // fused kernel: the ring the filtered boundary layers go to, its slot
  // (or, with nstep, *nstep mod D) and the slot size
  T* ring;
  long long slot_stride;
  int D;
  int slot;
};

}  // namespace atns
