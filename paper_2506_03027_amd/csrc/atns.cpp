// C ABI of the AT compressible-flow library: context, layout, scheduling.
#include "atns.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "coeffs.hpp"
#include "launch.hpp"
#include "layout.hpp"
#include "mlp.hpp"

using namespace atns;

struct atns_ctx {
  atns_config cfg{};
  std::vector<int> split[3];
  hipStream_t stream = nullptr;
  int device = 0;
  int n[3] = {1, 1, 1};
  double h[3] = {1, 1, 1};
  int H = 2;
  RKScheme rk{};
  int C = 5;                         // delayed levels of the AT scheme
  int nb = 0;
  std::vector<BlockDev> blocks;
  std::vector<TileDev> tiles;
  std::vector<HaloRegion> regions;
  std::vector<HaloWork> work;
  size_t esz = 4;
  long long field = 0;
  // RK registers: RK4 uses X[cur] = U, X[1-cur] = Ya, X[2] = Yb,
  // X[3] = acc (cur changes only with fused stage pairs, whose last stage
  // writes the new state to X[1-cur]); LSERK uses X[cur] = U, X[1-cur] =
  // the other stage buffer, X[3] = Q.
  void* X[4] = {nullptr, nullptr, nullptr, nullptr};
  int cur = 0;
  void* ring = nullptr;
  int D = 0;
  long long slot_stride = 0;
  BlockDev* d_blocks = nullptr;
  TileDev* d_tiles = nullptr;
  int8_t* d_delays = nullptr;
  int8_t* d_probe = nullptr;
  int8_t* d_inject = nullptr;
  int64_t inject0 = 0;
  int inject_n = 0;
  double* d_W = nullptr;
  void* hbuf = nullptr;              // stage halos: stages (+1 filter) x slot_stride
  double* d_finv = nullptr;          // filter: forward-elimination factors
  double* d_fcp = nullptr;
  double fah[6] = {0, 0, 0, 0, 0, 0};   // filter: a_0, a_1/2, ..., a_5/2
  void* comp = nullptr;              // compensated RK4: rounding error carried per point
  bool comp_on = false;
  bool fused_filter = true;          // filter steps with delayed halos in one kernel
  HaloRegion* d_regions = nullptr;
  HaloWork* d_work = nullptr;
  int nwork = 0;
  int tile[3] = {16, 16, 16};        // stage-kernel tile shape TX, TY, TZ
  // learned halo correction
  std::vector<FaceInfo> faceinfo;    // per halo region (faces meaningful)
  std::vector<int> face_regions;     // ids of face regions
  std::vector<HaloWork> face_chunks; // 16-point chunks of face regions
  FaceInfo* d_faceinfo = nullptr;
  int* d_face_regions = nullptr;
  HaloWork* d_face_chunks = nullptr;
  double* d_W0at = nullptr;          // AT stage-0 weights [L][C] (sampler target)
  MlpNet net{nullptr, nullptr, nullptr, nullptr};
  float* d_adam_m = nullptr;
  float* d_adam_v = nullptr;
  int adam_t = 0;
  float* d_grad = nullptr;
  float* d_part = nullptr;           // per-workgroup partial gradients
  float* d_loss_part = nullptr;
  float* d_loss = nullptr;
  float* d_X = nullptr;              // training batch
  float* d_Y = nullptr;
  int batch_cap = 0;
  unsigned long long* d_counters = nullptr;
  float mlp_s[5] = {1, 1, 1, 1, 1};
  float mlp_r[5] = {1, 1, 1, 1, 1};
  double mlp_tau = 1e30;
  bool mlp_on = false;
  bool mlp_ready = false;
  // graph-captured asynchronous steps
  long long* d_nstep = nullptr;      // device copy of the step number
  hipStream_t gstream = nullptr;     // capture/launch stream when `stream` is the null stream
  hipGraphExec_t gexec[2] = {nullptr, nullptr};   // per LSERK register parity
  bool use_graph = true;
  bool nstep_synced = false;
  uint64_t graph_gen = 0;   // bumped whenever captured step parameters go stale
  unsigned int* d_done = nullptr;   // workgroups done in the last stage of a captured step
  hipEvent_t order_ev = nullptr;
  double* d_partials = nullptr;
  double* d_diag = nullptr;
  int nparts = kDiagMaxParts;
  double dt = 0.0;
  int64_t step = 0;
  bool state_set = false;
  bool fuse = false;                 // classical RK4 stages 1-2 and 3-4 fused in pairs
  bool halo_fusion = false;          // halo assembly inside the first stage (graph steps)
  bool batch_member = false;         // stepped by a batch (its kernels never fuse halos)
  // free-running asynchronous steps: progress counters, abort flag, the
  // block-major tile list (for tiles async_tiles) and per-block ranges
  int* d_prog = nullptr;
  int* d_abort = nullptr;
  TileDev* d_btiles = nullptr;
  int* d_tile_begin = nullptr;
  int* d_reg_begin = nullptr;
  void* d_async_ps = nullptr;
  int async_tiles[3] = {0, 0, 0};
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;   // reusable events
  size_t ev_used = 0;                // events recorded since the last read
  std::vector<int> ev_launches;      // stage launches between each event pair
  std::string err;
};

namespace {

std::string g_err;

atns_status fail(atns_ctx* c, atns_status s, const std::string& msg) {
  if (c) c->err = msg;
  g_err = msg;
  return s;
}

// Entry points never let a C++ exception cross the C ABI (an uncaught one
// would end the caller's process with std::terminate): host allocation
// failures become ATNS_ENOMEM, anything else ATNS_EHIP, with the message.
template <class F>
atns_status guard_body(F&& f, std::string* err) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    if (err) *err = "host allocation failed";
    g_err = "host allocation failed";
    return ATNS_ENOMEM;
  } catch (const std::exception& e) {
    const std::string m = std::string("host exception: ") + e.what();
    if (err) *err = m;
    g_err = m;
    return ATNS_EHIP;
  } catch (...) {
    if (err) *err = "host exception";
    g_err = "host exception";
    return ATNS_EHIP;
  }
}
template <class F>
atns_status guarded(const atns_ctx* c, F&& f) {
  return guard_body(std::forward<F>(f), c ? &const_cast<atns_ctx*>(c)->err : nullptr);
}
template <class F>
atns_status guarded(std::nullptr_t, F&& f) {
  return guard_body(std::forward<F>(f), nullptr);
}

#define HIP_TRY(ctx, expr)                                                                  \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(ctx, ATNS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
  } while (0)

bool slot_used(const atns_ctx* c, int s) {
  int d[3];
  slot_dir(s, d);
  if (c->cfg.ndim == 2 && d[2] != 0) return false;
  const int nz = (d[0] != 0) + (d[1] != 0) + (d[2] != 0);
  return nz == 1 || (nz == 2 && c->cfg.physics == ATNS_NS);
}

// Face depth of the halo regions and ring layers: 2 (Euler CD4), 4
// (Navier-Stokes: gradients, then flux derivatives), 5 with the filter (its
// right-hand side reaches five points).
int halo_depth(const atns_config* cfg) {
  if (cfg->physics != ATNS_NS) return 2;
  return cfg->filter ? 5 : 4;
}

atns_status validate(const atns_config* cfg, std::vector<int> split[3], atns_ctx* c) {
  if (!cfg) return fail(c, ATNS_EINVAL, "null config");
  if (cfg->ndim != 2 && cfg->ndim != 3) return fail(c, ATNS_EINVAL, "ndim must be 2 or 3");
  if (cfg->physics != ATNS_EULER && cfg->physics != ATNS_NS) return fail(c, ATNS_EINVAL, "bad physics");
  if (cfg->rk != ATNS_RK4 && cfg->rk != ATNS_LSERK4 && cfg->rk != ATNS_LSERK2)
    return fail(c, ATNS_EINVAL, "bad rk");
  if (cfg->mode != ATNS_SA && cfg->mode != ATNS_AS && cfg->mode != ATNS_AT)
    return fail(c, ATNS_EINVAL, "bad mode");
  if (cfg->algo != ATNS_CAA && cfg->algo != ATNS_SAA) return fail(c, ATNS_EINVAL, "bad algo");
  if (cfg->precision != ATNS_F32 && cfg->precision != ATNS_F64) return fail(c, ATNS_EINVAL, "bad precision");
  if (cfg->L < 1 || cfg->L > 16) return fail(c, ATNS_EINVAL, "L must be in 1..16");
  if (!(cfg->gamma > 1.0)) return fail(c, ATNS_EINVAL, "gamma must exceed 1");
  if (cfg->physics == ATNS_NS && (!(cfg->mach > 0) || !(cfg->re > 0) || !(cfg->pr > 0)))
    return fail(c, ATNS_EINVAL, "Navier-Stokes needs mach, re, pr > 0");
  if (cfg->filter != 0 && cfg->filter != 1) return fail(c, ATNS_EINVAL, "filter must be 0 or 1");
  if (cfg->filter) {
    if (cfg->physics != ATNS_NS) return fail(c, ATNS_EINVAL, "the filter is built for Navier-Stokes contexts");
    if (!(cfg->filter_alpha > -0.5 && cfg->filter_alpha <= 0.5))
      return fail(c, ATNS_EINVAL, "filter_alpha must lie in (-0.5, 0.5]");
  }
  const int H = halo_depth(cfg);
  for (int d = 0; d < 3; ++d) {
    if (cfg->n[d] < 1 || cfg->nblk[d] < 1 || cfg->nblk[d] > cfg->n[d])
      return fail(c, ATNS_EINVAL, "bad grid or block count");
    if (!(cfg->len[d] > 0)) return fail(c, ATNS_EINVAL, "box lengths must be positive");
    if (cfg->n[d] > 32767) return fail(c, ATNS_EINVAL, "grid too large in one direction");
    split[d].clear();
    if (cfg->split[d]) {
      long long tot = 0;
      for (int i = 0; i < cfg->nblk[d]; ++i) {
        split[d].push_back(cfg->split[d][i]);
        tot += cfg->split[d][i];
      }
      if (tot != cfg->n[d]) return fail(c, ATNS_EINVAL, "split does not sum to n");
    } else {
      const int base = cfg->n[d] / cfg->nblk[d], rem = cfg->n[d] % cfg->nblk[d];
      for (int i = 0; i < cfg->nblk[d]; ++i) split[d].push_back(base + (i < rem ? 1 : 0));
    }
    const bool active = d < cfg->ndim;
    for (int s : split[d]) {
      if (s < 1) return fail(c, ATNS_EINVAL, "empty block");
      if (active && s < H) return fail(c, ATNS_EINVAL, "block smaller than the halo depth");
      if (active && cfg->filter && s > kFilterMaxLen)
        return fail(c, ATNS_EINVAL, "block longer than the filter's line limit");
    }
  }
  if (cfg->ndim == 2 && (cfg->n[2] != 1 || cfg->nblk[2] != 1))
    return fail(c, ATNS_EINVAL, "2D needs nz == 1 and one block in z");
  // the Navier-Stokes stage kernel addresses a field with 32-bit offsets
  if (cfg->physics == ATNS_NS && 5.0 * cfg->n[0] * cfg->n[1] * cfg->n[2] >= 2147483648.0)
    return fail(c, ATNS_EINVAL, "Navier-Stokes grid too large: 5 nx ny nz must stay below 2^31");
  return ATNS_OK;
}

void build_layout(atns_ctx* c) {
  const atns_config& cfg = c->cfg;
  const int nbx = cfg.nblk[0], nby = cfg.nblk[1], nbz = cfg.nblk[2];
  std::vector<int> start[3];
  for (int d = 0; d < 3; ++d) {
    int s = 0;
    for (int v : c->split[d]) {
      start[d].push_back(s);
      s += v;
    }
  }
  c->nb = nbx * nby * nbz;
  c->blocks.assign(c->nb, BlockDev{});
  auto bid = [&](int ix, int iy, int iz) {
    ix = (ix + nbx) % nbx;
    iy = (iy + nby) % nby;
    iz = (iz + nbz) % nbz;
    return (iz * nby + iy) * nbx + ix;
  };
  long long off = 0;
  for (int iz = 0; iz < nbz; ++iz)
    for (int iy = 0; iy < nby; ++iy)
      for (int ix = 0; ix < nbx; ++ix) {
        BlockDev& B = c->blocks[bid(ix, iy, iz)];
        const int idx[3] = {ix, iy, iz};
        for (int d = 0; d < 3; ++d) {
          B.o[d] = start[d][idx[d]];
          B.s[d] = c->split[d][idx[d]];
        }
        for (int s = 0; s < kNumSlots; ++s) {
          int dir[3];
          slot_dir(s, dir);
          B.nbr[s] = bid(ix + dir[0], iy + dir[1], iz + dir[2]);
          B.lay[s] = -1;
        }
      }
  // ring layers, block-major so a block's layers are adjacent
  for (int b = 0; b < c->nb; ++b) {
    BlockDev& B = c->blocks[b];
    for (int s = 0; s < kNumSlots; ++s) {
      if (!slot_used(c, s)) continue;
      int dir[3];
      slot_dir(s, dir);
      const int dep = s < 6 ? c->H : 2;
      long long cnt = 5;
      for (int d = 0; d < 3; ++d) cnt *= dir[d] ? dep : B.s[d];
      B.lay[s] = off;
      off += cnt;
    }
  }
  c->slot_stride = off;
  // reader-side halo offsets: region s of block b mirrors layer opposite(s)
  // of its neighbour, so the per-stage halo buffer has the same total size
  long long hoff = 0;
  for (int b = 0; b < c->nb; ++b) {
    BlockDev& B = c->blocks[b];
    for (int s = 0; s < kNumSlots; ++s) {
      B.hoff[s] = -1;
      B.roff[s] = -1;
      if (!slot_used(c, s)) continue;
      int dir[3];
      slot_dir(s, dir);
      const int dep = s < 6 ? c->H : 2;
      long long cnt = 1;
      for (int d = 0; d < 3; ++d) cnt *= dir[d] ? dep : B.s[d];
      B.hoff[s] = hoff;
      HaloRegion r;
      r.dst = hoff;
      r.src = c->blocks[B.nbr[s]].lay[slot_opposite(s)];
      B.roff[s] = r.src;
      r.npts = (int)cnt;
      r.kidx = b * kNumSlots + s;
      const int rid = (int)c->regions.size();
      c->regions.push_back(r);
      for (int st = 0; st < (int)cnt; st += kHaloChunk) c->work.push_back(HaloWork{rid, st});
      FaceInfo fi;
      fi.axis = dir[0] ? 0 : (dir[1] ? 1 : 2);
      for (int d = 0; d < 3; ++d) fi.ext[d] = dir[d] ? dep : B.s[d];
      c->faceinfo.push_back(fi);
      if (s < 6) {
        c->face_regions.push_back(rid);
        for (int st = 0; st < (int)cnt; st += kMlpChunk) c->face_chunks.push_back(HaloWork{rid, st});
      }
      hoff += 5 * cnt;
    }
  }
}

void build_tiles(atns_ctx* c, int TX, int TY, int TZ) {
  std::vector<TileDev> nat;
  for (int b = 0; b < c->nb; ++b) {
    const BlockDev& B = c->blocks[b];
    for (int z0 = 0; z0 < B.s[2]; z0 += TZ)
      for (int y0 = 0; y0 < B.s[1]; y0 += TY)
        for (int x0 = 0; x0 < B.s[0]; x0 += TX) {
          TileDev t;
          t.blk = b;
          t.x0 = (short)x0;
          t.y0 = (short)y0;
          t.z0 = (short)z0;
          t.nx = (short)std::min(TX, B.s[0] - x0);
          t.ny = (short)std::min(TY, B.s[1] - y0);
          t.nz = (short)std::min(TZ, B.s[2] - z0);
          nat.push_back(t);
        }
  }
  // XCD-aware order: workgroup w runs on XCD w % 8, so give XCD x the
  // contiguous chunk x of the natural (block-major) order.
  const int nx = 8;
  const size_t chunk = (nat.size() + nx - 1) / nx;
  c->tiles.assign(chunk * nx, TileDev{0, 0, 0, 0, 0, 0, 0});
  for (size_t j = 0; j < nat.size(); ++j) {
    const size_t x = j / chunk, pos = j % chunk;
    c->tiles[pos * nx + x] = nat[j];
  }
}

// (TX, TY) column shapes the stage kernels are instantiated for.  The
// single-precision Navier-Stokes kernel runs one thread per tile column and
// also takes 32 x 16; the double-precision one runs one thread per point of
// the tile plus a 4-point apron, whose LDS caps it at the first three.
constexpr int kNumEulerShapes = 5;
constexpr int kEulerShapes[kNumEulerShapes][2] = {{16, 16}, {32, 8}, {16, 8}, {64, 8}, {32, 16}};
constexpr int kNumNsShapes = 4;
constexpr int kNsShapes[kNumNsShapes][2] = {{16, 16}, {32, 8}, {16, 8}, {32, 16}};

// esz: bytes per value of the context's precision
int num_shapes(int physics, size_t esz) {
  return physics == ATNS_NS ? (esz == 4 ? kNumNsShapes : kNumNsShapes - 1) : kNumEulerShapes;
}
const int* shape_at(int physics, int i) { return physics == ATNS_NS ? kNsShapes[i] : kEulerShapes[i]; }

bool shape_supported(int physics, size_t esz, int tx, int ty) {
  for (int i = 0; i < num_shapes(physics, esz); ++i)
    if (shape_at(physics, i)[0] == tx && shape_at(physics, i)[1] == ty) return true;
  return false;
}

size_t count_tiles(const atns_ctx* c, int tx, int ty, int tz) {
  size_t n = 0;
  for (const BlockDev& B : c->blocks)
    n += (size_t)((B.s[0] + tx - 1) / tx) * ((B.s[1] + ty - 1) / ty) * ((B.s[2] + tz - 1) / tz);
  return n;
}

// Default shape before any tuning: 16 x 16 columns, and the longest column
// (32, 16, 8 or 4 planes) that still gives about eight workgroups per CU.
void default_tiles(atns_ctx* c) {
  c->tile[0] = 16;
  c->tile[1] = 16;
  int tz = 4;
  for (int cand : {32, 16, 8})
    if (count_tiles(c, 16, 16, cand) >= 2048) {
      tz = cand;
      break;
    }
  c->tile[2] = c->cfg.ndim == 2 ? 1 : tz;
}

void drop_graphs(atns_ctx* c);

atns_status upload_tiles(atns_ctx* c) {
  drop_graphs(c);
  build_tiles(c, c->tile[0], c->tile[1], c->tile[2]);
  if (c->d_tiles) (void)hipFree(c->d_tiles);
  c->d_tiles = nullptr;
  if (hipMalloc((void**)&c->d_tiles, c->tiles.size() * sizeof(TileDev)) != hipSuccess)
    return fail(c, ATNS_ENOMEM, "tile table allocation failed");
  HIP_TRY(c, hipMemcpy(c->d_tiles, c->tiles.data(), c->tiles.size() * sizeof(TileDev), hipMemcpyHostToDevice));
  return ATNS_OK;
}

template <typename T>
StageParams<T> base_params(const atns_ctx* c) {
  StageParams<T> p{};
  p.ring = (T*)c->ring;
  p.blocks = c->d_blocks;
  p.tiles = c->d_tiles;
  for (int d = 0; d < 3; ++d) {
    p.n[d] = c->n[d];
    p.dscale[d] = c->cfg.rk == ATNS_LSERK2 ? 1.0 / (2.0 * c->h[d]) : 1.0 / (12.0 * c->h[d]);
  }
  p.field = c->field;
  p.slot_stride = c->slot_stride;
  p.D = c->D;
  p.L = c->cfg.L;
  p.C = c->C;
  p.cd2 = c->cfg.rk == ATNS_LSERK2 ? 1 : 0;
  p.H = c->H;
  p.ndim = c->cfg.ndim;
  p.gamma = c->cfg.gamma;
  p.mach2_gamma = c->cfg.gamma * c->cfg.mach * c->cfg.mach;
  if (c->cfg.physics == ATNS_NS) {
    p.kappa = 1.0 / ((c->cfg.gamma - 1.0) * c->cfg.mach * c->cfg.mach * c->cfg.pr);
    p.inv_re = 1.0 / c->cfg.re;
  }
  p.dt = c->dt;
  return p;
}

hipError_t next_event(atns_ctx* c, hipEvent_t* ev) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    c->ev_pool.push_back(e);
  }
  *ev = c->ev_pool[c->ev_used++];
  return hipSuccess;
}

// Profiled runs of stage-kernel launches: one HIP event before the first
// launch of a run and one after its last, with nothing else enqueued in
// between, so the measured time is the launches' own plus the short gaps
// between back-to-back kernels on one stream.
hipError_t prof_begin(atns_ctx* c, hipStream_t s) {
  if (!c->profiling) return hipSuccess;
  hipEvent_t e;
  const hipError_t r = next_event(c, &e);
  return r == hipSuccess ? hipEventRecord(e, s) : r;
}

hipError_t prof_end(atns_ctx* c, hipStream_t s, int launches) {
  if (!c->profiling) return hipSuccess;
  hipEvent_t e;
  const hipError_t r = next_event(c, &e);
  if (r != hipSuccess) return r;
  c->ev_launches.push_back(launches);
  return hipEventRecord(e, s);
}

template <typename T>
hipError_t launch_stage(atns_ctx* c, const StageParams<T>& p, int kind) {
  return (c->cfg.physics == ATNS_NS)
             ? launch_ns_stage<T>(p, (int)c->tiles.size(), kind, c->tile[0], c->tile[1], c->stream)
             : launch_euler_stage<T>(p, (int)c->tiles.size(), kind, c->tile[0], c->tile[1], c->stream);
}

// Whether the RK4 stages run as two fused pairs: 3-D Euler, classical RK4,
// single precision, and a tile shape the pair kernel is built for.
bool pairs_apply(const atns_ctx* c) {
  if (!c->fuse || c->cfg.physics != ATNS_EULER || c->cfg.ndim != 3 || c->cfg.rk != ATNS_RK4 || c->esz != 4 ||
      c->comp_on)
    return false;
  const int tx = c->tile[0], ty = c->tile[1];
  return (tx == 16 && ty == 16) || (tx == 32 && ty == 8) || (tx == 16 && ty == 8) || (tx == 32 && ty == 16);
}

// Whether graph-captured steps assemble the stage halos inside the first
// stage kernel instead of a separate halo kernel: Euler with delayed halos,
// without the learned-halo correction (which works on assembled halos) and
// without the stage pairs.
bool fuse_halos(const atns_ctx* c) {
  return c->halo_fusion && !c->batch_member && c->cfg.physics == ATNS_EULER && c->cfg.mode != ATNS_SA &&
         !c->mlp_on && !pairs_apply(c) && c->hbuf != nullptr;
}

template <typename T>
hipError_t launch_pair(atns_ctx* c, const StageParams<T>& pA, const StageParams<T>& pB, int pair, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value)
    return launch_euler_pair<float>(pA, pB, (int)c->tiles.size(), pair, c->tile[0], c->tile[1], s);
  return hipErrorInvalidValue;
}

bool is_async(const atns_ctx* c, int64_t step) { return c->cfg.mode != ATNS_SA && step >= c->C; }

// Slots of the stage-halo buffer: one per stage, and the filter's halo at
// the new level when the filter is on.
int halo_slots(const atns_ctx* c) { return c->rk.stages + (c->cfg.filter ? 1 : 0); }

atns_status draw_delays(atns_ctx* c, int64_t step, int8_t* dst) {
  const int8_t* inj = nullptr;
  if (c->inject_n > 0 && step >= c->inject0 && step < c->inject0 + c->inject_n)
    inj = c->d_inject + (size_t)(step - c->inject0) * c->nb * kNumSlots;
  HIP_TRY(c, launch_delays(dst, inj, step, c->nb, c->cfg.L, c->C, c->cfg.seed, c->cfg.algo, c->stream));
  return ATNS_OK;
}

template <typename T>
MlpFeatArgs<T> feat_args(const atns_ctx* c) {
  MlpFeatArgs<T> fa{};
  fa.ring = (const T*)c->ring;
  fa.slot_stride = c->slot_stride;
  fa.D = c->D;
  fa.slot_now = c->D ? (int)(c->step % c->D) : 0;
  fa.L = c->cfg.L;
  for (int v = 0; v < 5; ++v) {
    fa.inv_s[v] = 1.f / c->mlp_s[v];
    fa.inv_r[v] = 1.f / c->mlp_r[v];
    fa.r[v] = c->mlp_r[v];
  }
  fa.tau2 = (float)std::min(c->mlp_tau * c->mlp_tau, 1e30);
  return fa;
}

// Delay draw and stage-halo assembly of the current step (asynchronous steps).
template <typename T>
atns_status prepare_halos(atns_ctx* c) {
  atns_status st = draw_delays(c, c->step, c->d_delays);
  if (st != ATNS_OK) return st;
  HIP_TRY(c, launch_halo<T>((const T*)c->ring, (T*)c->hbuf, c->d_regions, c->d_work, (int)c->work.size(),
                            c->d_delays, c->d_W, c->slot_stride, c->slot_stride, c->D,
                            (int)(c->step % c->D), c->cfg.L, halo_slots(c), c->cfg.mode == ATNS_AS,
                            c->stream));
  if (c->mlp_on && c->cfg.mode == ATNS_AT) {
    MlpFeatArgs<T> fa = feat_args<T>(c);
    HIP_TRY(c, mlp_halo<T>(fa, c->net, c->d_regions, c->d_faceinfo, c->d_face_chunks,
                           (long long)c->face_chunks.size(), c->d_delays, (T*)c->hbuf, c->slot_stride,
                           c->rk.stages, c->d_counters, c->stream));
  }
  return ATNS_OK;
}

hipStream_t work_stream(const atns_ctx* c) { return c->stream ? c->stream : c->gstream; }

// Executable graphs are destroyed only once every launch of them has
// finished: a queued launch still reads the kernel arguments the graph owns.
void drop_graphs(atns_ctx* c) {
  c->graph_gen += 1;
  bool any = false;
  for (hipGraphExec_t g : c->gexec) any = any || g != nullptr;
  if (!any) return;
  (void)hipStreamSynchronize(work_stream(c));
  for (hipGraphExec_t& g : c->gexec)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// Stage parameters of stage e of an asynchronous step whose step number is
// read on the device (graph-captured steps).
// fused: the parameters for the fused stage pairs, where the last stage
// writes the new state to X[1-cur] (the pair kernels never touch Ya).
template <typename T>
StageParams<T> graph_stage_params(const atns_ctx* c, int e, int* kind, bool fused) {
  const RKScheme& rk = c->rk;
  StageParams<T> p = base_params<T>(c);
  p.nstep = c->d_nstep;
  p.async_halo = c->cfg.mode == ATNS_SA ? kHaloSync : (c->cfg.mode == ATNS_AS ? kHaloStale : kHaloAT);
  p.halo = kHaloSync;
  p.hbuf = c->hbuf ? (const T*)c->hbuf + (size_t)e * c->slot_stride : nullptr;
  // with the filter on, the ring receives the filtered field after the passes
  p.ring_write = (c->ring != nullptr) && (e == rk.stages - 1) && !c->cfg.filter;
  if (e == 0 && fuse_halos(c)) {
    p.fuse_halo = 1;
    p.S = rk.stages;
    p.W = c->d_W;
    p.dd = DelayDraw{1, c->nb, c->cfg.algo == ATNS_SAA ? 1 : 0, (unsigned long long)c->cfg.seed};
  }
  if (e == rk.stages - 1) {   // the last stage also advances the step counter
    p.step_end = c->d_nstep;
    p.done = c->d_done;
  }
  if (!rk.low_storage) {
    T* U = (T*)c->X[c->cur];
    T* Ya = (T*)c->X[1 - c->cur];
    T* Yb = (T*)c->X[2];
    p.U0 = U;
    p.acc = (T*)c->X[3];
    const T* ins[4] = {U, Ya, Yb, Ya};
    T* outs[4] = {Ya, Yb, Ya, fused ? Ya : U};
    p.Y = ins[e];
    p.Yout = outs[e];
    *kind = e == 0 ? kRK4First : (e == 3 ? kRK4Last : kRK4Mid);
    p.cA = rk.b[e];
    p.cB = e < 3 ? rk.a[e + 1][e] : 0.0;
    // U^n joins the accumulator in the last middle stage, or, compensated,
    // the last stage adds it with its carried rounding error
    p.fold = (e == 2 && !c->comp_on) ? 1 : 0;
    p.comp = c->comp_on ? (T*)c->comp : nullptr;
  } else {
    const int cur = (c->cur + e) & 1;
    p.Y = (const T*)c->X[cur];
    p.Yout = (T*)c->X[1 - cur];
    p.acc = (T*)c->X[3];
    *kind = e == 0 ? kLSFirst : kLSMid;
    p.cA = rk.A[e];
    p.cB = rk.B[e];
  }
  return p;
}

// Enqueue the halo work of one asynchronous step with the device step counter.
template <typename T>
atns_status enqueue_graph_halos(atns_ctx* c, hipStream_t s) {
  if (c->cfg.mode == ATNS_SA || fuse_halos(c)) return ATNS_OK;   // fused: the first stage does it
  // the halo kernel draws the step's delays itself (no injection here)
  const DelayDraw dd{1, c->nb, c->cfg.algo == ATNS_SAA ? 1 : 0, (unsigned long long)c->cfg.seed};
  HIP_TRY(c, launch_halo<T>((const T*)c->ring, (T*)c->hbuf, c->d_regions, c->d_work, (int)c->work.size(),
                            c->d_delays, c->d_W, c->slot_stride, c->slot_stride, c->D, 0, c->cfg.L,
                            halo_slots(c), c->cfg.mode == ATNS_AS, s, c->d_nstep, dd));
  if (c->mlp_on && c->cfg.mode == ATNS_AT) {
    MlpFeatArgs<T> fa = feat_args<T>(c);
    fa.nstep = c->d_nstep;
    HIP_TRY(c, mlp_halo<T>(fa, c->net, c->d_regions, c->d_faceinfo, c->d_face_chunks,
                           (long long)c->face_chunks.size(), c->d_delays, (T*)c->hbuf, c->slot_stride,
                           c->rk.stages, c->d_counters, s));
  }
  return ATNS_OK;
}

// The filter passes on the state in X[fin] (x: X[fin] -> X[1-fin], y: ->
// X[2], z: -> X[fin]; 2-D: X[fin] -> X[1-fin] -> X[fin]; the other RK
// registers are free after the last stage), then the ring write of the
// filtered field into slot `slot` (or, with nstep, the slot of *nstep).
// halo: the step's HaloMode (ignored with nstep, which the kernels read).
template <typename T>
atns_status enqueue_filter(atns_ctx* c, int fin, int halo, const long long* nstep, int slot, hipStream_t s) {
  T* U = (T*)c->X[fin];
  T* bufs3[4] = {U, (T*)c->X[1 - fin], (T*)c->X[2], U};
  T* bufs2[3] = {U, (T*)c->X[1 - fin], U};
  T** bufs = c->cfg.ndim == 3 ? bufs3 : bufs2;
  FilterArgs<T> f{};
  f.blocks = c->d_blocks;
  f.fhalo = c->hbuf ? (const T*)c->hbuf + (size_t)c->rk.stages * c->slot_stride : nullptr;
  f.inv = c->d_finv;
  f.cp = c->d_fcp;
  for (int i = 0; i < 3; ++i) f.n[i] = c->n[i];
  f.field = c->field;
  f.H = c->H;
  f.halo = halo;
  f.nstep = nstep;
  f.C = c->C;
  f.async_halo = c->cfg.mode == ATNS_SA ? kHaloSync : (c->cfg.mode == ATNS_AS ? kHaloStale : kHaloAT);
  for (int m = 0; m < 6; ++m) f.ah[m] = c->fah[m];
  f.alpha = c->cfg.filter_alpha;
  // Steps with delayed halos filter each block in one workgroup per variable
  // (every block a cube of a size the fused kernel is built for).  Captured
  // steps are the asynchronous ones (step >= C), so they always take it.
  const int side = c->blocks.empty() ? 0 : c->blocks[0].s[0];
  bool fused = c->cfg.ndim == 3 && c->ring && f.fhalo && c->cfg.mode != ATNS_SA && c->fused_filter &&
               filter_fused_fits(side, (int)sizeof(T)) && (nstep || halo != kHaloSync);
  for (const BlockDev& B : c->blocks) fused = fused && B.s[0] == side && B.s[1] == side && B.s[2] == side;
  if (fused) {
    f.in = U;
    f.out = U;
    f.ring = (T*)c->ring;
    f.slot_stride = c->slot_stride;
    f.D = c->D;
    f.slot = slot;
    HIP_TRY(c, launch_filter_fused<T>(f, c->nb, side, s));
    return ATNS_OK;
  }
  for (int d = 0; d < c->cfg.ndim; ++d) {
    f.in = bufs[d];
    f.out = bufs[d + 1];
    f.dir = d;
    const int pa = d == 0 ? 1 : 0, qa = d == 2 ? 1 : 2;
    int max_lines = 1, max_len = 1, min_len = kFilterMaxLen;
    for (const BlockDev& B : c->blocks) {
      max_lines = std::max(max_lines, B.s[pa] * B.s[qa]);
      max_len = std::max(max_len, B.s[d]);
      min_len = std::min(min_len, B.s[d]);
    }
    HIP_TRY(c, launch_filter_pass<T>(f, c->nb, max_lines, min_len, max_len, s));
  }
  if (c->ring) HIP_TRY(c, launch_ring_fill<T>(base_params<T>(c), U, slot, c->nb, s, nstep));
  return ATNS_OK;
}

// One captured step: halos (with the delay draw) and the s stage kernels;
// the last stage kernel advances the device step counter when it finishes.
template <typename T>
atns_status capture_step(atns_ctx* c, hipGraphExec_t* out) {
  hipStream_t s = work_stream(c);
  hipGraph_t graph = nullptr;
  HIP_TRY(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  atns_status st = enqueue_graph_halos<T>(c, s);
  const bool pairs = pairs_apply(c);
  StageParams<T> ps[4];
  for (int e = 0; st == ATNS_OK && e < c->rk.stages; ++e) {
    int kind = 0;
    const StageParams<T> p = graph_stage_params<T>(c, e, &kind, pairs);
    hipError_t r = hipSuccess;
    if (pairs) {
      ps[e] = p;
      if constexpr (std::is_same<T, float>::value) {
        if (e == 1 || e == 3)
          r = launch_euler_pair<float>(ps[e - 1], ps[e], (int)c->tiles.size(), e / 2, c->tile[0], c->tile[1], s);
      }
    } else {
      r = (c->cfg.physics == ATNS_NS)
              ? launch_ns_stage<T>(p, (int)c->tiles.size(), kind, c->tile[0], c->tile[1], s)
              : launch_euler_stage<T>(p, (int)c->tiles.size(), kind, c->tile[0], c->tile[1], s);
    }
    if (r != hipSuccess) st = fail(c, ATNS_EHIP, std::string("stage launch in capture: ") + hipGetErrorString(r));
  }
  if (st == ATNS_OK && c->cfg.filter) {
    // the last stage has advanced the counter: the passes and the ring
    // write read the step as *nstep - 1 and the slot as *nstep mod D
    const int fin = c->rk.low_storage ? ((c->cur + c->rk.stages) & 1) : c->cur;
    st = enqueue_filter<T>(c, fin, kHaloSync, c->d_nstep, 0, s);
  }
  const hipError_t ec = hipStreamEndCapture(s, &graph);
  if (st != ATNS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (ec != hipSuccess) return fail(c, ATNS_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
  const hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return fail(c, ATNS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  return ATNS_OK;
}

// Work enqueued on `from` so far precedes later work on `to`.
atns_status order_streams(atns_ctx* c, hipStream_t from, hipStream_t to) {
  if (from == to) return ATNS_OK;
  HIP_TRY(c, hipEventRecord(c->order_ev, from));
  HIP_TRY(c, hipStreamWaitEvent(to, c->order_ev, 0));
  return ATNS_OK;
}

template <typename T>
atns_status do_steps_impl(atns_ctx* c, int nsteps, bool* on_graph) {
  const RKScheme& rk = c->rk;
  for (int it = 0; it < nsteps; ++it) {
    const bool async = is_async(c, c->step);
    const bool graphable = async && c->use_graph && !c->profiling && c->inject_n == 0;
    hipStream_t s = work_stream(c);
    if (graphable) {
      const int par = c->cur;
      if (!c->gexec[par]) {
        atns_status st = capture_step<T>(c, &c->gexec[par]);
        if (st != ATNS_OK) return st;
      }
      if (!*on_graph) {
        atns_status st = order_streams(c, c->stream, s);
        if (st != ATNS_OK) return st;
        *on_graph = true;
      }
      if (!c->nstep_synced) {
        HIP_TRY(c, launch_step_set(c->d_nstep, c->step, s));
        c->nstep_synced = true;
      }
      HIP_TRY(c, hipGraphLaunch(c->gexec[par], s));
      if ((rk.low_storage && (rk.stages & 1)) || pairs_apply(c)) c->cur = 1 - c->cur;
      c->step += 1;
      continue;
    }
    if (*on_graph) {
      atns_status st = order_streams(c, s, c->stream);
      if (st != ATNS_OK) return st;
      *on_graph = false;
    }
    c->nstep_synced = false;
    if (async) {
      atns_status st = prepare_halos<T>(c);
      if (st != ATNS_OK) return st;
    }
    StageParams<T> p = base_params<T>(c);
    p.halo = !async ? kHaloSync : (c->cfg.mode == ATNS_AS ? kHaloStale : kHaloAT);
    p.slot_now = c->D ? (int)(c->step % c->D) : 0;
    const bool pairs = pairs_apply(c);
    StageParams<T> ps[4];
    HIP_TRY(c, prof_begin(c, c->stream));
    for (int e = 0; e < rk.stages; ++e) {
      p.hbuf = c->hbuf ? (const T*)c->hbuf + (size_t)e * c->slot_stride : nullptr;
      p.ring_write = (c->ring != nullptr) && (e == rk.stages - 1) && !c->cfg.filter;
      int kind;
      if (!rk.low_storage) {
        T* U = (T*)c->X[c->cur];
        T* Ya = (T*)c->X[1 - c->cur];
        T* Yb = (T*)c->X[2];
        p.U0 = U;
        p.acc = (T*)c->X[3];
        const T* ins[4] = {U, Ya, Yb, Ya};
        T* outs[4] = {Ya, Yb, Ya, pairs ? Ya : U};
        p.Y = ins[e];
        p.Yout = outs[e];
        kind = e == 0 ? kRK4First : (e == 3 ? kRK4Last : kRK4Mid);
        p.cA = rk.b[e];
        p.cB = e < 3 ? rk.a[e + 1][e] : 0.0;
        // U^n joins the accumulator in the last middle stage, or, compensated,
        // the last stage adds it with its carried rounding error
        p.fold = (e == 2 && !c->comp_on) ? 1 : 0;
        p.comp = c->comp_on ? (T*)c->comp : nullptr;
      } else {
        p.Y = (const T*)c->X[c->cur];
        p.Yout = (T*)c->X[1 - c->cur];
        p.acc = (T*)c->X[3];
        kind = e == 0 ? kLSFirst : kLSMid;
        p.cA = rk.A[e];
        p.cB = rk.B[e];
      }
      if (pairs) {
        ps[e] = p;
        if (e == 1 || e == 3) HIP_TRY(c, launch_pair<T>(c, ps[e - 1], ps[e], e / 2, c->stream));
      } else {
        HIP_TRY(c, launch_stage<T>(c, p, kind));
      }
      if (rk.low_storage) c->cur = 1 - c->cur;
    }
    HIP_TRY(c, prof_end(c, c->stream, pairs ? rk.stages / 2 : rk.stages));
    if (pairs) c->cur = 1 - c->cur;   // the new state went to X[1 - cur]
    if (c->cfg.filter) {
      atns_status st = enqueue_filter<T>(c, c->cur, p.halo, nullptr, c->D ? (int)((c->step + 1) % c->D) : 0,
                                         c->stream);
      if (st != ATNS_OK) return st;
    }
    c->step += 1;
  }
  return ATNS_OK;
}

template <typename T>
atns_status do_steps(atns_ctx* c, int nsteps) {
  bool on_graph = false;
  atns_status st = do_steps_impl<T>(c, nsteps, &on_graph);
  if (on_graph) {
    const atns_status s2 = order_streams(c, work_stream(c), c->stream);
    if (st == ATNS_OK) st = s2;
  }
  return st;
}

void* state_ptr(const atns_ctx* c) { return c->X[c->cur]; }

void release(atns_ctx* c) {
  drop_graphs(c);
  if (c->gstream) (void)hipStreamDestroy(c->gstream);
  c->gstream = nullptr;
  if (c->order_ev) (void)hipEventDestroy(c->order_ev);
  c->order_ev = nullptr;
  if (c->d_nstep) (void)hipFree(c->d_nstep);
  c->d_nstep = nullptr;
  if (c->d_done) (void)hipFree(c->d_done);
  c->d_done = nullptr;
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  c->ev_pool.clear();
  for (void*& x : c->X)
    if (x) {
      (void)hipFree(x);
      x = nullptr;
    }
  void* ptrs[] = {c->ring, c->d_blocks, c->d_tiles, c->d_delays, c->d_probe, c->d_inject, c->d_W,
                  c->d_partials, c->d_diag, c->hbuf, c->d_regions, c->d_work, c->d_faceinfo,
                  c->d_face_regions, c->d_face_chunks, c->d_W0at, c->net.params, c->net.w1, c->net.w2,
                  c->net.w3, c->d_adam_m, c->d_adam_v, c->d_grad, c->d_part, c->d_loss_part, c->d_loss,
                  c->d_X, c->d_Y, c->d_counters, c->d_prog, c->d_abort, c->d_btiles, c->d_tile_begin,
                  c->d_reg_begin, c->d_async_ps, c->d_finv, c->d_fcp, c->comp};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  c->ring = nullptr;
}

}  // namespace

extern "C" {

const char* atns_version(void) { return "atns 0.1 gfx950"; }

const char* atns_last_error(const atns_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

atns_status atns_create(const atns_config* cfg, void* stream, atns_ctx** out) {
  return guarded(nullptr, [&]() -> atns_status {
    if (!out) return fail(nullptr, ATNS_EINVAL, "null output pointer");
    *out = nullptr;
    auto* c = new atns_ctx();
    std::vector<int> split[3];
    atns_status st = validate(cfg, split, c);
    if (st != ATNS_OK) {
      delete c;
      return st;
    }
    c->cfg = *cfg;
    for (int d = 0; d < 3; ++d) {
      c->split[d] = split[d];
      c->cfg.split[d] = nullptr;
      c->n[d] = cfg->n[d];
      c->h[d] = cfg->len[d] / cfg->n[d];
    }
    c->stream = (hipStream_t)stream;
    c->H = halo_depth(cfg);
    c->rk = make_rk(cfg->rk);
    c->C = levels(cfg->rk);
    c->esz = cfg->precision == ATNS_F64 ? 8 : 4;
    c->field = (long long)c->n[0] * c->n[1] * c->n[2];
    build_layout(c);
    default_tiles(c);
    build_tiles(c, c->tile[0], c->tile[1], c->tile[2]);
    // SA keeps a delayed-level ring only when L > 1 (history for the learned
    // halo's training samples); the asynchronous modes always do.
    // SA keeps C + L levels (training history); the asynchronous modes keep
    // C + 2L - 1, so that free-running steps (atns_step_async), where a
    // neighbour may run L - 1 steps ahead of a reader, never overwrite a level
    // the reader still needs.  Scheduled delays need only C + L.
    c->D = cfg->mode == ATNS_SA ? (cfg->L <= 1 ? 0 : c->C + cfg->L) : c->C + 2 * cfg->L - 1;

    auto fail_free = [&](atns_status s, const std::string& m) {
      release(c);
      g_err = m;
      delete c;
      return s;
    };
    if (hipGetDevice(&c->device) != hipSuccess) return fail_free(ATNS_EHIP, "no HIP device");
    if (hipMalloc((void**)&c->d_nstep, sizeof(long long)) != hipSuccess ||
        hipMalloc((void**)&c->d_done, sizeof(unsigned int)) != hipSuccess ||
        hipMemset(c->d_done, 0, sizeof(unsigned int)) != hipSuccess)
      return fail_free(ATNS_ENOMEM, "counter allocation failed");
    if (!c->stream && hipStreamCreate(&c->gstream) != hipSuccess)
      return fail_free(ATNS_EHIP, "stream creation failed");
    if (hipEventCreateWithFlags(&c->order_ev, hipEventDisableTiming) != hipSuccess)
      return fail_free(ATNS_EHIP, "event creation failed");
    const size_t fbytes = (size_t)c->field * 5 * c->esz;
    for (int i = 0; i < 4; ++i)
      if (hipMalloc(&c->X[i], fbytes) != hipSuccess) return fail_free(ATNS_ENOMEM, "state allocation failed");
    if (c->D) {
      if (hipMalloc(&c->ring, (size_t)c->slot_stride * c->D * c->esz) != hipSuccess)
        return fail_free(ATNS_ENOMEM, "ring allocation failed");
      if (cfg->mode != ATNS_SA &&
          hipMalloc(&c->hbuf, (size_t)c->slot_stride * halo_slots(c) * c->esz) != hipSuccess)
        return fail_free(ATNS_ENOMEM, "halo buffer allocation failed");
      {
        const std::vector<double> W0 = halo_weights(cfg->rk, ATNS_AT, cfg->L);   // stage 0 = first L*C entries
        if (hipMalloc((void**)&c->d_W0at, (size_t)cfg->L * c->C * sizeof(double)) != hipSuccess ||
            hipMemcpy(c->d_W0at, W0.data(), (size_t)cfg->L * c->C * sizeof(double), hipMemcpyHostToDevice) !=
                hipSuccess)
          return fail_free(ATNS_EHIP, "weight table upload failed");
        if (hipMalloc((void**)&c->d_faceinfo, c->faceinfo.size() * sizeof(FaceInfo)) != hipSuccess ||
            hipMemcpy(c->d_faceinfo, c->faceinfo.data(), c->faceinfo.size() * sizeof(FaceInfo),
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMalloc((void**)&c->d_face_regions, c->face_regions.size() * sizeof(int)) != hipSuccess ||
            hipMemcpy(c->d_face_regions, c->face_regions.data(), c->face_regions.size() * sizeof(int),
                      hipMemcpyHostToDevice) != hipSuccess ||
            hipMalloc((void**)&c->d_face_chunks, c->face_chunks.size() * sizeof(HaloWork)) != hipSuccess ||
            hipMemcpy(c->d_face_chunks, c->face_chunks.data(), c->face_chunks.size() * sizeof(HaloWork),
                      hipMemcpyHostToDevice) != hipSuccess)
          return fail_free(ATNS_EHIP, "face table upload failed");
      }
      if (hipMalloc((void**)&c->d_regions, c->regions.size() * sizeof(HaloRegion)) != hipSuccess ||
          hipMalloc((void**)&c->d_work, c->work.size() * sizeof(HaloWork)) != hipSuccess ||
          hipMemcpy(c->d_regions, c->regions.data(), c->regions.size() * sizeof(HaloRegion),
                    hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(c->d_work, c->work.data(), c->work.size() * sizeof(HaloWork), hipMemcpyHostToDevice) !=
              hipSuccess)
        return fail_free(ATNS_EHIP, "halo table upload failed");
      std::vector<double> W = halo_weights(cfg->rk, cfg->mode == ATNS_AS ? ATNS_AS : ATNS_AT, cfg->L);
      if (cfg->filter) {   // the filter-halo row follows the stage rows
        const std::vector<double> Wf = filter_halo_weights(cfg->rk, cfg->mode == ATNS_AS ? ATNS_AS : ATNS_AT, cfg->L);
        W.insert(W.end(), Wf.begin(), Wf.end());
      }
      if (hipMalloc((void**)&c->d_W, W.size() * sizeof(double)) != hipSuccess ||
          hipMemcpy(c->d_W, W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return fail_free(ATNS_EHIP, "weight table upload failed");
    }
    if (cfg->filter) {
      const std::vector<double> a = filter_coefficients(cfg->filter_alpha);
      for (int m = 0; m < 6; ++m) c->fah[m] = m == 0 ? a[0] : 0.5 * a[m];
      std::vector<double> inv, cp;
      filter_thomas(cfg->filter_alpha, kFilterMaxLen, inv, cp);
      if (hipMalloc((void**)&c->d_finv, kFilterMaxLen * sizeof(double)) != hipSuccess ||
          hipMalloc((void**)&c->d_fcp, kFilterMaxLen * sizeof(double)) != hipSuccess ||
          hipMemcpy(c->d_finv, inv.data(), kFilterMaxLen * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(c->d_fcp, cp.data(), kFilterMaxLen * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return fail_free(ATNS_EHIP, "filter table upload failed");
    }
    const size_t dcount = (size_t)c->nb * kNumSlots;
    if (hipMalloc((void**)&c->d_blocks, c->blocks.size() * sizeof(BlockDev)) != hipSuccess ||
        hipMalloc((void**)&c->d_tiles, c->tiles.size() * sizeof(TileDev)) != hipSuccess ||
        hipMalloc((void**)&c->d_delays, dcount) != hipSuccess || hipMalloc((void**)&c->d_probe, dcount) != hipSuccess ||
        hipMalloc((void**)&c->d_partials, (size_t)c->nparts * 7 * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&c->d_diag, 7 * sizeof(double)) != hipSuccess)
      return fail_free(ATNS_ENOMEM, "table allocation failed");
    if (hipMemcpy(c->d_blocks, c->blocks.data(), c->blocks.size() * sizeof(BlockDev), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(c->d_tiles, c->tiles.data(), c->tiles.size() * sizeof(TileDev), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemset(c->d_delays, 0, dcount) != hipSuccess)
      return fail_free(ATNS_EHIP, "table upload failed");
    *out = c;
    return ATNS_OK;
  });
}

atns_status atns_destroy(atns_ctx* ctx) {
  return guarded(ctx, [&]() -> atns_status {
    if (!ctx) return ATNS_OK;
    (void)hipStreamSynchronize(ctx->stream);
    release(ctx);
    delete ctx;
    return ATNS_OK;
  });
}

}  // extern "C"

namespace {

// The state now in state_ptr(c) becomes the state of `step`: its boundary
// layers go into the ring slot of that step.
atns_status adopt_state(atns_ctx* c, int64_t step) {
  c->step = step;
  c->state_set = true;
  c->nstep_synced = false;
  if (c->comp) HIP_TRY(c, hipMemsetAsync(c->comp, 0, (size_t)c->field * 5 * c->esz, c->stream));
  if (c->ring) {
    const int slot = (int)(step % c->D);
    if (c->esz == 4) {
      StageParams<float> p = base_params<float>(c);
      HIP_TRY(c, launch_ring_fill<float>(p, (const float*)state_ptr(c), slot, c->nb, c->stream));
    } else {
      StageParams<double> p = base_params<double>(c);
      HIP_TRY(c, launch_ring_fill<double>(p, (const double*)state_ptr(c), slot, c->nb, c->stream));
    }
  }
  return ATNS_OK;
}

// Fingerprint of everything a restart record depends on (FNV-1a).
uint64_t config_fingerprint(const atns_ctx* c) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  const atns_config& g = c->cfg;
  mix(&g.ndim, sizeof g.ndim);
  mix(g.n, sizeof g.n);
  mix(g.len, sizeof g.len);
  mix(&g.physics, sizeof g.physics);
  mix(&g.gamma, sizeof g.gamma);
  mix(&g.mach, sizeof g.mach);
  mix(&g.re, sizeof g.re);
  mix(&g.pr, sizeof g.pr);
  mix(&g.rk, sizeof g.rk);
  mix(&g.mode, sizeof g.mode);
  mix(&g.algo, sizeof g.algo);
  mix(&g.L, sizeof g.L);
  mix(&g.seed, sizeof g.seed);
  mix(&g.precision, sizeof g.precision);
  mix(&g.filter, sizeof g.filter);
  if (g.filter) mix(&g.filter_alpha, sizeof g.filter_alpha);
  for (const BlockDev& B : c->blocks) {
    mix(B.o, sizeof B.o);
    mix(B.s, sizeof B.s);
  }
  return h;
}

struct CkptHeader {
  char magic[8];
  uint64_t fingerprint;
  int64_t step;
  double dt;
  uint64_t state_bytes, ring_bytes;
};
const char kCkptMagic[8] = {'A', 'T', 'N', 'S', 'C', 'K', 'P', '1'};

}  // namespace

extern "C" {

atns_status atns_set_state(atns_ctx* c, const void* dev_U, int64_t step) {
  return guarded(c, [&]() -> atns_status {
    if (!c || !dev_U) return fail(c, ATNS_EINVAL, "null argument");
    if (step < 0) return fail(c, ATNS_EINVAL, "negative step");
    HIP_TRY(c, hipMemcpyAsync(state_ptr(c), dev_U, (size_t)c->field * 5 * c->esz, hipMemcpyDeviceToDevice,
                              c->stream));
    return adopt_state(c, step);
  });
}

atns_status atns_init_case(atns_ctx* c, int32_t case_id, const double* params, int32_t np, int64_t step) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    if (step < 0) return fail(c, ATNS_EINVAL, "negative step");
    if (np < 0 || (np > 0 && !params)) return fail(c, ATNS_EINVAL, "bad parameter list");
    // vortex parameters, in order, with their defaults: t, beta, mach, xc, yc
    double vp[5] = {0.0, 5.0, 0.5, 5.0, 5.0};
    if (case_id == ATNS_CASE_VORTEX) {
      if (np > 5) return fail(c, ATNS_EINVAL, "the vortex takes at most 5 parameters");
      for (int i = 0; i < np; ++i) vp[i] = params[i];
    } else if (case_id == ATNS_CASE_TGV) {
      if (np != 0) return fail(c, ATNS_EINVAL, "the Taylor-Green case takes no parameters");
      if (c->cfg.ndim != 3) return fail(c, ATNS_EINVAL, "the Taylor-Green case is three-dimensional");
      vp[2] = c->cfg.mach;
    } else {
      return fail(c, ATNS_EINVAL, "unknown case");
    }
    const int kind = case_id == ATNS_CASE_VORTEX ? 0 : 1;
    const hipError_t e =
        c->esz == 4 ? launch_init_case<float>((float*)state_ptr(c), c->n, c->h, c->cfg.len, kind, c->cfg.ndim,
                                              c->cfg.gamma, vp[2], vp[1], vp[0], vp[3], vp[4], c->stream)
                    : launch_init_case<double>((double*)state_ptr(c), c->n, c->h, c->cfg.len, kind, c->cfg.ndim,
                                               c->cfg.gamma, vp[2], vp[1], vp[0], vp[3], vp[4], c->stream);
    if (e != hipSuccess) return fail(c, ATNS_EHIP, std::string("init_case: ") + hipGetErrorString(e));
    return adopt_state(c, step);
  });
}

atns_status atns_checkpoint(atns_ctx* c, void* host_blob, size_t* bytes) {
  return guarded(c, [&]() -> atns_status {
    if (!c || !bytes) return fail(c, ATNS_EINVAL, "null argument");
    const size_t sb = (size_t)c->field * 5 * c->esz;
    const size_t rb = c->ring ? (size_t)c->slot_stride * c->D * c->esz : 0;
    const size_t need = sizeof(CkptHeader) + sb + rb;
    if (!host_blob) {
      *bytes = need;
      return ATNS_OK;
    }
    if (*bytes < need) return fail(c, ATNS_EINVAL, "checkpoint buffer too small");
    if (!c->state_set) return fail(c, ATNS_ESTATE, "no state to checkpoint");
    CkptHeader h;
    std::memcpy(h.magic, kCkptMagic, 8);
    h.fingerprint = config_fingerprint(c);
    h.step = c->step;
    h.dt = c->dt;
    h.state_bytes = sb;
    h.ring_bytes = rb;
    char* out = (char*)host_blob;
    std::memcpy(out, &h, sizeof h);
    HIP_TRY(c, hipMemcpyAsync(out + sizeof h, state_ptr(c), sb, hipMemcpyDeviceToHost, c->stream));
    if (rb) HIP_TRY(c, hipMemcpyAsync(out + sizeof h + sb, c->ring, rb, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *bytes = need;
    return ATNS_OK;
  });
}

atns_status atns_restore(atns_ctx* c, const void* host_blob, size_t bytes) {
  return guarded(c, [&]() -> atns_status {
    if (!c || !host_blob) return fail(c, ATNS_EINVAL, "null argument");
    CkptHeader h;
    if (bytes < sizeof h) return fail(c, ATNS_EINVAL, "not a restart record");
    std::memcpy(&h, host_blob, sizeof h);
    const size_t sb = (size_t)c->field * 5 * c->esz;
    const size_t rb = c->ring ? (size_t)c->slot_stride * c->D * c->esz : 0;
    if (std::memcmp(h.magic, kCkptMagic, 8) != 0) return fail(c, ATNS_EINVAL, "not a restart record");
    if (h.fingerprint != config_fingerprint(c) || h.state_bytes != sb || h.ring_bytes != rb)
      return fail(c, ATNS_EINVAL, "restart record of a different configuration");
    if (bytes < sizeof h + sb + rb) return fail(c, ATNS_EINVAL, "truncated restart record");
    const char* in = (const char*)host_blob;
    HIP_TRY(c, hipMemcpyAsync(state_ptr(c), in + sizeof h, sb, hipMemcpyHostToDevice, c->stream));
    if (rb) HIP_TRY(c, hipMemcpyAsync(c->ring, in + sizeof h + sb, rb, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (h.dt > 0 && h.dt != c->dt) drop_graphs(c);
    if (h.dt > 0) c->dt = h.dt;
    c->step = h.step;
    c->state_set = true;
    c->nstep_synced = false;
    return ATNS_OK;
  });
}

atns_status atns_get_state(const atns_ctx* c, void* dst, int32_t on_host) {
  return guarded(c, [&]() -> atns_status {
    if (!c || !dst) return fail(const_cast<atns_ctx*>(c), ATNS_EINVAL, "null argument");
    atns_ctx* m = const_cast<atns_ctx*>(c);
    const size_t bytes = (size_t)c->field * 5 * c->esz;
    if (on_host) {
      HIP_TRY(m, hipMemcpyAsync(dst, state_ptr(c), bytes, hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(m, hipStreamSynchronize(c->stream));
    } else {
      HIP_TRY(m, hipMemcpyAsync(dst, state_ptr(c), bytes, hipMemcpyDeviceToDevice, c->stream));
    }
    return ATNS_OK;
  });
}

atns_status atns_get_step(const atns_ctx* c, int64_t* step) {
  return guarded(c, [&]() -> atns_status {
    if (!c || !step) return fail(const_cast<atns_ctx*>(c), ATNS_EINVAL, "null argument");
    *step = c->step;
    return ATNS_OK;
  });
}

atns_status atns_set_dt(atns_ctx* c, double dt) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(c, ATNS_EINVAL, "dt must be positive and finite");
    if (dt != c->dt) drop_graphs(c);
    c->dt = dt;
    return ATNS_OK;
  });
}

atns_status atns_set_delays(atns_ctx* c, int64_t step0, int32_t nsteps, const int8_t* host_k) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    if (nsteps < 0 || (nsteps > 0 && !host_k)) return fail(c, ATNS_EINVAL, "bad delay injection");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->d_inject) {
      HIP_TRY(c, hipFree(c->d_inject));
      c->d_inject = nullptr;
    }
    c->inject_n = 0;
    if (nsteps == 0) return ATNS_OK;
    const size_t bytes = (size_t)nsteps * c->nb * kNumSlots;
    if (hipMalloc((void**)&c->d_inject, bytes) != hipSuccess) return fail(c, ATNS_ENOMEM, "inject allocation");
    HIP_TRY(c, hipMemcpy(c->d_inject, host_k, bytes, hipMemcpyHostToDevice));
    c->inject0 = step0;
    c->inject_n = nsteps;
    return ATNS_OK;
  });
}

atns_status atns_get_delays(atns_ctx* c, int64_t step, int8_t* host_k, int32_t* synchronous) {
  return guarded(c, [&]() -> atns_status {
    if (!c || !host_k) return fail(c, ATNS_EINVAL, "null argument");
    const size_t cnt = (size_t)c->nb * kNumSlots;
    if (!is_async(c, step)) {
      std::memset(host_k, 0, cnt);
      if (synchronous) *synchronous = 1;
      return ATNS_OK;
    }
    atns_status st = draw_delays(c, step, c->d_probe);
    if (st != ATNS_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(host_k, c->d_probe, cnt, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (synchronous) *synchronous = 0;
    return ATNS_OK;
  });
}

atns_status atns_rhs(atns_ctx* c, int32_t stage, void* dev_R) {
  return guarded(c, [&]() -> atns_status {
    if (!c || !dev_R) return fail(c, ATNS_EINVAL, "null argument");
    if (stage < 0 || stage >= c->rk.stages) return fail(c, ATNS_EINVAL, "stage outside 0..s-1");
    if (!c->state_set) return fail(c, ATNS_ESTATE, "state not set");
    const bool async = is_async(c, c->step);
    auto go = [&](auto tag) -> atns_status {
      using T = decltype(tag);
      if (async) {
        atns_status st = prepare_halos<T>(c);
        if (st != ATNS_OK) return st;
      }
      StageParams<T> p = base_params<T>(c);
      p.halo = !async ? kHaloSync : (c->cfg.mode == ATNS_AS ? kHaloStale : kHaloAT);
      p.slot_now = c->D ? (int)(c->step % c->D) : 0;
      p.hbuf = c->hbuf ? (const T*)c->hbuf + (size_t)stage * c->slot_stride : nullptr;
      p.ring_write = 0;
      p.Y = (const T*)state_ptr(c);
      p.Yout = (T*)dev_R;
      HIP_TRY(c, prof_begin(c, c->stream));
      HIP_TRY(c, launch_stage<T>(c, p, kRhsOnly));
      HIP_TRY(c, prof_end(c, c->stream, 1));
      return ATNS_OK;
    };
    return c->esz == 4 ? go(float{}) : go(double{});
  });
}

atns_status atns_set_fusion(atns_ctx* c, int32_t on) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    c->fuse = on != 0;
    drop_graphs(c);
    return ATNS_OK;
  });
}

atns_status atns_set_compensation(atns_ctx* c, int32_t on) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    if (on && c->cfg.rk != ATNS_RK4) return fail(c, ATNS_EINVAL, "compensated steps are built for classical RK4");
    if (on && c->cfg.filter) return fail(c, ATNS_EINVAL, "compensated steps are not combined with the filter");
    if (on && !c->comp) {
      const size_t bytes = (size_t)c->field * 5 * c->esz;
      if (hipMalloc(&c->comp, bytes) != hipSuccess) return fail(c, ATNS_ENOMEM, "compensation allocation failed");
      HIP_TRY(c, hipMemsetAsync(c->comp, 0, bytes, c->stream));
    }
    c->comp_on = on != 0;
    drop_graphs(c);
    return ATNS_OK;
  });
}

atns_status atns_set_halo_fusion(atns_ctx* c, int32_t on) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    c->halo_fusion = on != 0;
    drop_graphs(c);
    return ATNS_OK;
  });
}

atns_status atns_set_filter_fusion(atns_ctx* c, int32_t on) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    c->fused_filter = on != 0;
    drop_graphs(c);
    return ATNS_OK;
  });
}

atns_status atns_rk_step(atns_ctx* c, int32_t nsteps) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    if (nsteps < 0) return fail(c, ATNS_EINVAL, "negative step count");
    if (!c->state_set) return fail(c, ATNS_ESTATE, "state not set");
    if (!(c->dt > 0)) return fail(c, ATNS_ESTATE, "dt not set");
    return c->esz == 4 ? do_steps<float>(c, nsteps) : do_steps<double>(c, nsteps);
  });
}

}  // extern "C"

namespace {

// Device tables of the free-running kernel for the current tile shape.
atns_status async_tables(atns_ctx* c) {
  if (c->d_btiles && c->async_tiles[0] == c->tile[0] && c->async_tiles[1] == c->tile[1] &&
      c->async_tiles[2] == c->tile[2])
    return ATNS_OK;
  std::vector<TileDev> bt;
  std::vector<int> tb(1, 0), rb(1, 0);
  for (int b = 0; b < c->nb; ++b) {
    const BlockDev& B = c->blocks[b];
    for (int z0 = 0; z0 < B.s[2]; z0 += c->tile[2])
      for (int y0 = 0; y0 < B.s[1]; y0 += c->tile[1])
        for (int x0 = 0; x0 < B.s[0]; x0 += c->tile[0]) {
          TileDev t;
          t.blk = b;
          t.x0 = (short)x0;
          t.y0 = (short)y0;
          t.z0 = (short)z0;
          t.nx = (short)std::min(c->tile[0], B.s[0] - x0);
          t.ny = (short)std::min(c->tile[1], B.s[1] - y0);
          t.nz = (short)std::min(c->tile[2], B.s[2] - z0);
          bt.push_back(t);
        }
    tb.push_back((int)bt.size());
  }
  // regions are stored block by block (build_layout)
  int r = 0;
  for (int b = 0; b < c->nb; ++b) {
    while (r < (int)c->regions.size() && c->regions[r].kidx / kNumSlots == b) ++r;
    rb.push_back(r);
  }
  void* ptrs[] = {c->d_btiles, c->d_tile_begin, c->d_reg_begin};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  c->d_btiles = nullptr;
  c->d_tile_begin = c->d_reg_begin = nullptr;
  if (hipMalloc((void**)&c->d_btiles, bt.size() * sizeof(TileDev)) != hipSuccess ||
      hipMalloc((void**)&c->d_tile_begin, tb.size() * sizeof(int)) != hipSuccess ||
      hipMalloc((void**)&c->d_reg_begin, rb.size() * sizeof(int)) != hipSuccess)
    return fail(c, ATNS_ENOMEM, "free-running tables allocation failed");
  HIP_TRY(c, hipMemcpy(c->d_btiles, bt.data(), bt.size() * sizeof(TileDev), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->d_tile_begin, tb.data(), tb.size() * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(c, hipMemcpy(c->d_reg_begin, rb.data(), rb.size() * sizeof(int), hipMemcpyHostToDevice));
  for (int d = 0; d < 3; ++d) c->async_tiles[d] = c->tile[d];
  return ATNS_OK;
}

template <typename T>
atns_status step_async_impl(atns_ctx* c, int nsteps, long long spin_limit, int8_t* dev_log) {
  const int stages = c->rk.stages;
  AsyncArgs a{};
  int per_cu = 0, cus = 0;
  const bool ns = c->cfg.physics == ATNS_NS;
  HIP_TRY(c, ns ? launch_ns_async<T>(nullptr, a, stages, c->tile[0], c->tile[1], c->stream, &per_cu)
                : launch_euler_async<T>(nullptr, a, stages, c->tile[0], c->tile[1], c->stream, &per_cu));
  HIP_TRY(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
  if ((long long)per_cu * cus < c->nb)
    return fail(c, ATNS_EINVAL, "more blocks than workgroups that fit on the device at once (" +
                                    std::to_string((long long)per_cu * cus) + ")");
  atns_status st = async_tables(c);
  if (st != ATNS_OK) return st;
  if (!c->d_prog) {
    if (hipMalloc((void**)&c->d_prog, c->nb * sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&c->d_abort, sizeof(int)) != hipSuccess ||
        hipMalloc(&c->d_async_ps, 4 * sizeof(StageParams<T>)) != hipSuccess)
      return fail(c, ATNS_ENOMEM, "free-running state allocation failed");
  }
  std::vector<StageParams<T>> ps(stages);
  for (int e = 0; e < stages; ++e) {
    int kind = 0;
    ps[e] = graph_stage_params<T>(c, e, &kind, false);
    ps[e].fuse_halo = 0;   // the persistent kernel assembles its own halos
    ps[e].nstep = nullptr;
    ps[e].step_end = nullptr;
    ps[e].done = nullptr;
    ps[e].halo = c->cfg.mode == ATNS_AS ? kHaloStale : kHaloAT;
  }
  const std::vector<int> prog(c->nb, (int)c->step);
  const int zero = 0;
  HIP_TRY(c, hipMemcpyAsync(c->d_async_ps, ps.data(), stages * sizeof(StageParams<T>), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_prog, prog.data(), c->nb * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->d_abort, &zero, sizeof(int), hipMemcpyHostToDevice, c->stream));
  a.prog = c->d_prog;
  a.abort = c->d_abort;
  a.log = dev_log;
  a.regions = c->d_regions;
  a.reg_begin = c->d_reg_begin;
  a.tiles = c->d_btiles;
  a.tile_begin = c->d_tile_begin;
  a.W = c->d_W;
  a.n0 = c->step;
  a.nsteps = nsteps;
  a.nb = c->nb;
  a.D = c->D;
  a.L = c->cfg.L;
  a.stale = c->cfg.mode == ATNS_AS ? 1 : 0;
  a.slot_stride = c->slot_stride;
  a.spin_limit = spin_limit;
  const StageParams<T>* dps = (const StageParams<T>*)c->d_async_ps;
  HIP_TRY(c, ns ? launch_ns_async<T>(dps, a, stages, c->tile[0], c->tile[1], c->stream, nullptr)
                : launch_euler_async<T>(dps, a, stages, c->tile[0], c->tile[1], c->stream, nullptr));
  int aborted = 0;
  HIP_TRY(c, hipMemcpyAsync(&aborted, c->d_abort, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->nstep_synced = false;
  if (aborted) {
    c->state_set = false;
    return fail(c, ATNS_ESTATE, "a wait for a neighbour exceeded spin_limit polls; the blocks stopped at "
                                "different steps, so the state must be set again");
  }
  c->step += nsteps;
  return ATNS_OK;
}

}  // namespace

extern "C" {

atns_status atns_step_async(atns_ctx* c, int32_t nsteps, int64_t spin_limit, int8_t* dev_log) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    if (nsteps < 0 || (nsteps > 0 && !dev_log) || spin_limit < 1)
      return fail(c, ATNS_EINVAL, "need nsteps >= 0, a delay log for nsteps > 0 and spin_limit >= 1");
    if (c->cfg.physics == ATNS_NS && c->cfg.ndim != 3)
      return fail(c, ATNS_EINVAL, "free-running Navier-Stokes steps are built for 3-D contexts");
    if (c->cfg.mode == ATNS_SA) return fail(c, ATNS_EINVAL, "free-running steps need mode ATNS_AT or ATNS_AS");
    if (c->rk.stages != 4 && c->rk.stages != 2)
      return fail(c, ATNS_EINVAL, "free-running steps need ATNS_RK4 or ATNS_LSERK2");
    if (c->mlp_on) return fail(c, ATNS_EINVAL, "the learned halo is not applied in free-running steps");
    if (c->cfg.filter) return fail(c, ATNS_EINVAL, "the filter is not applied in free-running steps");
  if (c->comp_on) return fail(c, ATNS_EINVAL, "compensated steps are not built for free-running steps");
    if (!c->state_set) return fail(c, ATNS_ESTATE, "state not set");
    if (!(c->dt > 0)) return fail(c, ATNS_ESTATE, "dt not set");
    if (c->step < c->C + c->cfg.L - 1) return fail(c, ATNS_ESTATE, "history shorter than C + L - 1 levels");
    if (nsteps == 0) return ATNS_OK;
    return c->esz == 4 ? step_async_impl<float>(c, nsteps, spin_limit, dev_log)
                       : step_async_impl<double>(c, nsteps, spin_limit, dev_log);
  });
}

atns_status atns_reduce(atns_ctx* c, double* host_out) {
  return guarded(c, [&]() -> atns_status {
    if (!c || !host_out) return fail(c, ATNS_EINVAL, "null argument");
    if (!c->state_set) return fail(c, ATNS_ESTATE, "state not set");
    // the reduction kernel indexes the five fields with 32-bit offsets
    if (5 * c->field >= (1ll << 31)) return fail(c, ATNS_EINVAL, "grid too large for the reduction (5 n^3 >= 2^31)");
    double inv12h[3];
    for (int d = 0; d < 3; ++d) inv12h[d] = 1.0 / (12.0 * c->h[d]);
    const double dV = c->h[0] * c->h[1] * (c->cfg.ndim == 3 ? c->h[2] : c->cfg.len[2]);
    if (c->esz == 4) {
      HIP_TRY(c, launch_diag<float>((const float*)state_ptr(c), c->n, c->cfg.ndim, inv12h, dV, c->d_partials,
                                    c->nparts, c->d_diag, c->stream));
    } else {
      HIP_TRY(c, launch_diag<double>((const double*)state_ptr(c), c->n, c->cfg.ndim, inv12h, dV, c->d_partials,
                                     c->nparts, c->d_diag, c->stream));
    }
    HIP_TRY(c, hipMemcpyAsync(host_out, c->d_diag, 7 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < 7; ++i)
      if (!std::isfinite(host_out[i])) return fail(c, ATNS_ENONFINITE, "non-finite diagnostic");
    return ATNS_OK;
  });
}

atns_status atns_reduce_noalloc(const void* dev_U, int32_t precision, int32_t ndim, const int32_t* n,
                                const double* len, double* dev_out, void* stream) {
  return guarded(nullptr, [&]() -> atns_status {
    if (!dev_U || !n || !len || !dev_out) return fail(nullptr, ATNS_EINVAL, "null argument");
    if (precision != ATNS_F32 && precision != ATNS_F64) return fail(nullptr, ATNS_EINVAL, "bad precision");
    if (ndim != 2 && ndim != 3) return fail(nullptr, ATNS_EINVAL, "ndim must be 2 or 3");
    if (ndim == 2 && n[2] != 1) return fail(nullptr, ATNS_EINVAL, "2D needs nz == 1");
    for (int d = 0; d < 3; ++d) {
      if (n[d] < 1 || !(len[d] > 0)) return fail(nullptr, ATNS_EINVAL, "bad grid or box length");
      if (d < ndim && n[d] < 5) return fail(nullptr, ATNS_EINVAL, "the CD4 vorticity needs 5 points per axis");
    }
    if (5.0 * n[0] * n[1] * n[2] >= 2147483648.0)
      return fail(nullptr, ATNS_EINVAL, "grid too large for the reduction (5 nx ny nz >= 2^31)");
    double inv12h[3], h[3];
    for (int d = 0; d < 3; ++d) {
      h[d] = len[d] / n[d];
      inv12h[d] = 1.0 / (12.0 * h[d]);
    }
    const double dV = h[0] * h[1] * (ndim == 3 ? h[2] : len[2]);
    const int nn[3] = {n[0], n[1], n[2]};
    const hipError_t e =
        precision == ATNS_F32
            ? launch_diag_noalloc<float>((const float*)dev_U, nn, ndim, inv12h, dV, dev_out, (hipStream_t)stream)
            : launch_diag_noalloc<double>((const double*)dev_U, nn, ndim, inv12h, dV, dev_out, (hipStream_t)stream);
    if (e != hipSuccess) return fail(nullptr, ATNS_EHIP, std::string("atns_reduce_noalloc: ") + hipGetErrorString(e));
    return ATNS_OK;
  });
}

atns_status atns_get_layout(const atns_ctx* c, int32_t* nblocks, int32_t* ring_depth) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(nullptr, ATNS_EINVAL, "null context");
    if (nblocks) *nblocks = c->nb;
    if (ring_depth) *ring_depth = c->D;
    return ATNS_OK;
  });
}

atns_status atns_set_graphs(atns_ctx* c, int32_t on) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    HIP_TRY(c, hipDeviceSynchronize());
    c->use_graph = on != 0;
    if (!c->use_graph) drop_graphs(c);
    return ATNS_OK;
  });
}

atns_status atns_profile_enable(atns_ctx* c, int32_t on) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->profiling = on != 0;
    c->ev_used = 0;
    c->ev_launches.clear();
    return ATNS_OK;
  });
}

atns_status atns_profile_read(atns_ctx* c, int64_t* launches, double* total_ms) {
  return guarded(c, [&]() -> atns_status {
    if (!c || !launches || !total_ms) return fail(c, ATNS_EINVAL, "null argument");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double tot = 0.0;
    int64_t n = 0;
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
      float ms = 0.f;
      HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_pool[i], c->ev_pool[i + 1]));
      tot += ms;
      n += c->ev_launches[i / 2];
    }
    *launches = n;
    *total_ms = tot;
    c->ev_used = 0;
    c->ev_launches.clear();
    return ATNS_OK;
  });
}

atns_status atns_set_tiles(atns_ctx* c, int32_t tx, int32_t ty, int32_t tz) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    if (!shape_supported(c->cfg.physics, c->esz, tx, ty) || tz < 1 || tz > 32767)
      return fail(c, ATNS_EINVAL, "unsupported tile shape");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->tile[0] = tx;
    c->tile[1] = ty;
    c->tile[2] = c->cfg.ndim == 2 ? 1 : tz;
    return upload_tiles(c);
  });
}

atns_status atns_get_tiles(const atns_ctx* c, int32_t* tx, int32_t* ty, int32_t* tz) {
  return guarded(c, [&]() -> atns_status {
    if (!c || !tx || !ty || !tz) return fail(const_cast<atns_ctx*>(c), ATNS_EINVAL, "null argument");
    *tx = c->tile[0];
    *ty = c->tile[1];
    *tz = c->tile[2];
    return ATNS_OK;
  });
}

}  // extern "C"

namespace {

std::string tune_key(const atns_ctx* c) {
  // blocks of one size class tune alike: key on the first block's shape,
  // the block count, the physics, precision and dimension
  char buf[256];
  const BlockDev& B = c->blocks[0];
  std::snprintf(buf, sizeof buf, "gfx950/phys%d/prec%d/ndim%d/blk%dx%dx%d/nb%d", c->cfg.physics,
                c->cfg.precision, c->cfg.ndim, B.s[0], B.s[1], B.s[2], c->nb);
  return buf;
}

bool cache_lookup(const char* path, const std::string& key, int out[3]) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char k[256];
  int a, b, d;
  bool found = false;
  while (std::fscanf(f, "%255s %d %d %d", k, &a, &b, &d) == 4)
    if (key == k) {
      out[0] = a;
      out[1] = b;
      out[2] = d;
      found = true;
    }
  std::fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, const int v[3]) {
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d\n", key.c_str(), v[0], v[1], v[2]);
  std::fclose(f);
}

// Parameters of RK stage e of a timing probe on the current state, writing
// only what is dead at a step boundary: the stage registers and the
// accumulator (RK4), or Q and the spare buffer (LSERK4).  The last stage's
// output goes to a stage register instead of the state, and its ring write to
// slot (n + 1) mod D, whose level n + 1 - D no stage of step n reads.
// Contexts with delayed halos read the stage-halo buffer, as their
// asynchronous steps do (probe_halos fills it).
template <typename T>
StageParams<T> probe_stage(atns_ctx* c, int e, int* kind_out) {
  const RKScheme& rk = c->rk;
  StageParams<T> p = base_params<T>(c);
  p.halo = kHaloSync;
  if (c->hbuf) {
    p.halo = c->cfg.mode == ATNS_AS ? kHaloStale : kHaloAT;
    p.hbuf = (const T*)c->hbuf + (size_t)e * c->slot_stride;
  }
  p.slot_now = c->D ? (int)(c->step % c->D) : 0;
  p.ring_write = (c->ring != nullptr) && (e == rk.stages - 1);
  int kind;
  if (!rk.low_storage) {
    T* U = (T*)c->X[c->cur];
    T* Ya = (T*)c->X[1 - c->cur];
    T* Yb = (T*)c->X[2];
    p.U0 = U;
    p.acc = (T*)c->X[3];
    const T* ins[4] = {U, Ya, Yb, Ya};
    T* outs[4] = {Ya, Yb, Ya, Yb};   // the last stage into Yb, not U
    p.Y = ins[e];
    p.Yout = outs[e];
    kind = e == 0 ? kRK4First : (e == 3 ? kRK4Last : kRK4Mid);
    p.cA = rk.b[e];
    p.cB = e < 3 ? rk.a[e + 1][e] : 0.0;
    p.fold = e == 2 ? 1 : 0;   // U^n joins the accumulator in the last middle stage
  } else {
    // the state buffer is only ever read; the stages alternate between
    // the spare buffer and X[2], which low-storage schemes do not use
    void* spare[2] = {c->X[1 - c->cur], c->X[2]};
    p.Y = (const T*)(e == 0 ? c->X[c->cur] : spare[(e - 1) & 1]);
    p.Yout = (T*)spare[e & 1];
    p.acc = (T*)c->X[3];
    kind = e == 0 ? kLSFirst : kLSMid;
    p.cA = rk.A[e];
    p.cB = rk.B[e];
  }
  *kind_out = kind;
  return p;
}

// The stage-halo buffer of the current step, for timing probes of contexts
// with delayed halos.  The buffer is rewritten at the start of every
// asynchronous step, so it is dead at a step boundary.
template <typename T>
atns_status probe_halos(atns_ctx* c) {
  return c->hbuf ? prepare_halos<T>(c) : ATNS_OK;
}

template <typename T>
atns_status time_shape(atns_ctx* c, int reps, float* ms_out) {
  // One step's mix of stage kernels -- first, middle and last RK stage, the
  // last with its ring write -- as timing probes.
  atns_status st = probe_halos<T>(c);
  if (st != ATNS_OK) return st;
  std::vector<std::pair<StageParams<T>, int>> seq;
  for (int e = 0; e < c->rk.stages; ++e) {
    int kind;
    StageParams<T> p = probe_stage<T>(c, e, &kind);
    seq.push_back({p, kind});
  }
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  for (auto& q : seq) HIP_TRY(c, launch_stage<T>(c, q.first, q.second));   // warm
  HIP_TRY(c, hipEventRecord(e0, c->stream));
  for (int r = 0; r < reps; ++r)
    for (auto& q : seq) HIP_TRY(c, launch_stage<T>(c, q.first, q.second));
  HIP_TRY(c, hipEventRecord(e1, c->stream));
  HIP_TRY(c, hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms_out = ms / reps;
  return ATNS_OK;
}

}  // namespace

extern "C" {

atns_status atns_autotune(atns_ctx* c, int32_t reps, const char* cache_path, int32_t* best) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    if (!c->state_set) return fail(c, ATNS_ESTATE, "state not set");
    if (reps < 1) return fail(c, ATNS_EINVAL, "reps must be positive");
    const std::string key = tune_key(c);
    int pick[3];
    // entries naming a shape the library does not provide are ignored
    const bool cached = cache_lookup(cache_path, key, pick) && shape_supported(c->cfg.physics, c->esz, pick[0], pick[1]) &&
                        pick[2] >= 1 && pick[2] <= 32767;
    if (!cached) {
      const bool ns = c->cfg.physics == ATNS_NS;
      const int tzs[] = {4, 8, 16, 32};
      float best_ms = 1e30f;
      pick[0] = c->tile[0];
      pick[1] = c->tile[1];
      pick[2] = c->tile[2];
      for (int i = 0; i < num_shapes(c->cfg.physics, c->esz); ++i)
        for (int tz : tzs) {
          if (c->cfg.ndim == 2 && tz != 4) continue;
          if (ns && tz < 8) continue;   // 8 extra planes per column: short ones waste work
          const int tx = shape_at(c->cfg.physics, i)[0], ty = shape_at(c->cfg.physics, i)[1];
          atns_status st = atns_set_tiles(c, tx, ty, tz);
          if (st != ATNS_OK) return st;
          float ms = 0.f;
          st = c->esz == 4 ? time_shape<float>(c, reps, &ms) : time_shape<double>(c, reps, &ms);
          if (st != ATNS_OK) return st;
          if (ms < best_ms) {
            best_ms = ms;
            pick[0] = tx;
            pick[1] = ty;
            pick[2] = c->tile[2];
          }
        }
      cache_store(cache_path, key, pick);
    }
    atns_status st = atns_set_tiles(c, pick[0], pick[1], pick[2]);
    if (st != ATNS_OK) return st;
    if (best) {
      best[0] = pick[0];
      best[1] = pick[1];
      best[2] = pick[2];
    }
    return ATNS_OK;
  });
}

namespace {

atns_status mlp_alloc(atns_ctx* c) {
  if (c->net.params) return ATNS_OK;
  const size_t pb = kMlpParams * sizeof(float);
  if (hipMalloc((void**)&c->net.params, pb) != hipSuccess ||
      hipMalloc((void**)&c->net.w1, kMlpH * kMlpIn * 2) != hipSuccess ||
      hipMalloc((void**)&c->net.w2, kMlpH * kMlpH * 2) != hipSuccess ||
      hipMalloc((void**)&c->net.w3, kMlpOut * kMlpH * 2) != hipSuccess ||
      hipMalloc((void**)&c->d_adam_m, pb) != hipSuccess || hipMalloc((void**)&c->d_adam_v, pb) != hipSuccess ||
      hipMalloc((void**)&c->d_grad, pb) != hipSuccess || hipMalloc((void**)&c->d_loss, sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&c->d_counters, 2 * sizeof(unsigned long long)) != hipSuccess)
    return fail(c, ATNS_ENOMEM, "MLP allocation failed");
  HIP_TRY(c, hipMemsetAsync(c->d_adam_m, 0, pb, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_adam_v, 0, pb, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->d_counters, 0, 2 * sizeof(unsigned long long), c->stream));
  return ATNS_OK;
}

atns_status mlp_batch(atns_ctx* c, int n) {
  const int nparts = (n + 63) / 64;
  if (n <= c->batch_cap) return ATNS_OK;
  for (float** p : {&c->d_part, &c->d_loss_part, &c->d_X, &c->d_Y})
    if (*p) {
      (void)hipFree(*p);
      *p = nullptr;
    }
  if (hipMalloc((void**)&c->d_part, (size_t)nparts * kMlpParams * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&c->d_loss_part, (size_t)nparts * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&c->d_X, (size_t)n * kMlpIn * sizeof(float)) != hipSuccess ||
      hipMalloc((void**)&c->d_Y, (size_t)n * 8 * sizeof(float)) != hipSuccess)
    return fail(c, ATNS_ENOMEM, "MLP batch allocation failed");
  c->batch_cap = n;
  return ATNS_OK;
}

atns_status mlp_need(atns_ctx* c) {
  if (!c) return fail(c, ATNS_EINVAL, "null context");
  if (!c->mlp_ready) return fail(c, ATNS_ESTATE, "MLP parameters not set");
  return ATNS_OK;
}

atns_status sample_into(atns_ctx* c, int n, uint64_t seed, float* X, float* Y) {
  if (!c->ring) return fail(c, ATNS_ESTATE, "no delayed-level history (SA with L = 1)");
  if (c->face_regions.empty()) return fail(c, ATNS_ESTATE, "no face halos");
  if (c->C != kMaxC) return fail(c, ATNS_EINVAL, "the learned halo works with AT4 (C = 5 levels)");
  if (c->step < c->C + c->cfg.L - 1) return fail(c, ATNS_ESTATE, "history shorter than C + L - 1 levels");
  if (c->esz == 4) {
    MlpFeatArgs<float> fa = feat_args<float>(c);
    HIP_TRY(c, mlp_sample<float>(fa, c->d_regions, c->d_faceinfo, c->d_face_regions, (int)c->face_regions.size(),
                                 c->d_W0at, seed, n, X, Y, c->stream));
  } else {
    MlpFeatArgs<double> fa = feat_args<double>(c);
    HIP_TRY(c, mlp_sample<double>(fa, c->d_regions, c->d_faceinfo, c->d_face_regions,
                                  (int)c->face_regions.size(), c->d_W0at, seed, n, X, Y, c->stream));
  }
  return ATNS_OK;
}

}  // namespace

atns_status atns_mlp_set_params(atns_ctx* c, const float* host_params) {
  return guarded(c, [&]() -> atns_status {
    if (!c || !host_params) return fail(c, ATNS_EINVAL, "null argument");
    atns_status st = mlp_alloc(c);
    if (st != ATNS_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(c->net.params, host_params, kMlpParams * sizeof(float), hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, mlp_pack(c->net, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->d_adam_m, 0, kMlpParams * sizeof(float), c->stream));
    HIP_TRY(c, hipMemsetAsync(c->d_adam_v, 0, kMlpParams * sizeof(float), c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->adam_t = 0;
    c->mlp_ready = true;
    return ATNS_OK;
  });
}

atns_status atns_mlp_get_params(atns_ctx* c, float* host_params) {
  return guarded(c, [&]() -> atns_status {
    atns_status st = mlp_need(c);
    if (st != ATNS_OK) return st;
    if (!host_params) return fail(c, ATNS_EINVAL, "null argument");
    HIP_TRY(c, hipMemcpyAsync(host_params, c->net.params, kMlpParams * sizeof(float), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return ATNS_OK;
  });
}

atns_status atns_mlp_set_scales(atns_ctx* c, const float* feat_scale, const float* targ_scale) {
  return guarded(c, [&]() -> atns_status {
    if (!c || !feat_scale || !targ_scale) return fail(c, ATNS_EINVAL, "null argument");
    for (int v = 0; v < 5; ++v)
      if (!(feat_scale[v] > 0) || !(targ_scale[v] > 0) || !std::isfinite(feat_scale[v]) ||
          !std::isfinite(targ_scale[v]))
        return fail(c, ATNS_EINVAL, "scales must be positive and finite");
    for (int v = 0; v < 5; ++v) {
      c->mlp_s[v] = feat_scale[v];
      c->mlp_r[v] = targ_scale[v];
    }
    drop_graphs(c);
    return ATNS_OK;
  });
}

atns_status atns_mlp_forward(atns_ctx* c, const float* dev_X, int32_t n, float* dev_out) {
  return guarded(c, [&]() -> atns_status {
    atns_status st = mlp_need(c);
    if (st != ATNS_OK) return st;
    if (!dev_X || !dev_out || n < 1) return fail(c, ATNS_EINVAL, "bad forward arguments");
    HIP_TRY(c, mlp_forward(c->net, dev_X, n, dev_out, c->stream));
    return ATNS_OK;
  });
}

atns_status atns_mlp_grad(atns_ctx* c, const float* dev_X, const float* dev_Y, int32_t n, float* dev_grad,
                          double* host_loss) {
  return guarded(c, [&]() -> atns_status {
    atns_status st = mlp_need(c);
    if (st != ATNS_OK) return st;
    if (!dev_X || !dev_Y || !dev_grad || n < 1) return fail(c, ATNS_EINVAL, "bad gradient arguments");
    st = mlp_batch(c, n);
    if (st != ATNS_OK) return st;
    HIP_TRY(c, mlp_grad(c->net, dev_X, dev_Y, n, c->d_part, c->d_loss_part, dev_grad, c->d_loss, c->stream));
    if (host_loss) {
      float l = 0.f;
      HIP_TRY(c, hipMemcpyAsync(&l, c->d_loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
      HIP_TRY(c, hipStreamSynchronize(c->stream));
      *host_loss = l;
    }
    return ATNS_OK;
  });
}

atns_status atns_mlp_sample(atns_ctx* c, int32_t n, uint64_t seed, float* dev_X, float* dev_Y) {
  return guarded(c, [&]() -> atns_status {
    if (!c || !dev_X || !dev_Y || n < 1) return fail(c, ATNS_EINVAL, "bad sample arguments");
    return sample_into(c, n, seed, dev_X, dev_Y);
  });
}

atns_status atns_mlp_train(atns_ctx* c, int32_t iters, int32_t batch, double lr, uint64_t seed, double* losses) {
  return guarded(c, [&]() -> atns_status {
    atns_status st = mlp_need(c);
    if (st != ATNS_OK) return st;
    if (iters < 1 || batch < 64 || !(lr > 0)) return fail(c, ATNS_EINVAL, "bad training arguments");
    st = mlp_batch(c, batch);
    if (st != ATNS_OK) return st;
    std::vector<float> lv(iters);
    for (int i = 0; i < iters; ++i) {
      st = sample_into(c, batch, seed + (uint64_t)i * 0x632BE59BD9B4E019ull, c->d_X, c->d_Y);
      if (st != ATNS_OK) return st;
      HIP_TRY(c, mlp_grad(c->net, c->d_X, c->d_Y, batch, c->d_part, c->d_loss_part, c->d_grad, c->d_loss,
                          c->stream));
      if (losses) HIP_TRY(c, hipMemcpyAsync(&lv[i], c->d_loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
      c->adam_t += 1;
      HIP_TRY(c, mlp_adam(c->net, c->d_adam_m, c->d_adam_v, c->d_grad, (float)lr, c->adam_t, c->stream));
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (losses)
      for (int i = 0; i < iters; ++i) losses[i] = lv[i];
    return ATNS_OK;
  });
}

atns_status atns_mlp_enable(atns_ctx* c, int32_t on, double tau) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    if (on && !c->mlp_ready) return fail(c, ATNS_ESTATE, "MLP parameters not set");
    if (on && c->cfg.mode != ATNS_AT) return fail(c, ATNS_EINVAL, "the learned halo needs mode ATNS_AT");
    if (on && c->C != kMaxC) return fail(c, ATNS_EINVAL, "the learned halo works with AT4 (C = 5 levels)");
    if (on && c->cfg.filter) return fail(c, ATNS_EINVAL, "the learned halo is not combined with the filter");
    if (!(tau >= 0)) return fail(c, ATNS_EINVAL, "tau must be non-negative");
    c->mlp_on = on != 0;
    c->mlp_tau = tau;
    drop_graphs(c);
    return ATNS_OK;
  });
}

atns_status atns_mlp_stats(atns_ctx* c, int64_t* applied, int64_t* fallback) {
  return guarded(c, [&]() -> atns_status {
    if (!c || !applied || !fallback) return fail(c, ATNS_EINVAL, "null argument");
    if (!c->d_counters) {
      *applied = *fallback = 0;
      return ATNS_OK;
    }
    unsigned long long h[2] = {0, 0};
    HIP_TRY(c, hipMemcpyAsync(h, c->d_counters, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->d_counters, 0, sizeof h, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *applied = (int64_t)h[0];
    *fallback = (int64_t)h[1];
    return ATNS_OK;
  });
}

atns_status atns_hbm_probe(const void* dev_src, void* dev_dst, int64_t bytes, void* stream) {
  return guarded(nullptr, [&]() -> atns_status {
    if (!dev_src || !dev_dst || bytes < 16 || bytes % 16 != 0)
      return fail(nullptr, ATNS_EINVAL, "probe needs device buffers and a positive multiple of 16 bytes");
    const hipError_t e = launch_copy_probe(dev_src, dev_dst, bytes, (hipStream_t)stream);
    if (e != hipSuccess) return fail(nullptr, ATNS_EHIP, std::string("copy probe: ") + hipGetErrorString(e));
    return ATNS_OK;
  });
}

atns_status atns_filter_state(atns_ctx* c) {
  return guarded(c, [&]() -> atns_status {
    if (!c) return fail(c, ATNS_EINVAL, "null context");
    if (!c->cfg.filter) return fail(c, ATNS_EINVAL, "the context has no filter");
    if (!c->state_set) return fail(c, ATNS_ESTATE, "state not set");
    const int slot = c->D ? (int)(c->step % c->D) : 0;
    return c->esz == 4 ? enqueue_filter<float>(c, c->cur, kHaloSync, nullptr, slot, c->stream)
                       : enqueue_filter<double>(c, c->cur, kHaloSync, nullptr, slot, c->stream);
  });
}

atns_status atns_host_filter_coefficients(double alpha, double* a6) {
  return guarded(nullptr, [&]() -> atns_status {
    if (!a6 || !(alpha > -0.5 && alpha <= 0.5)) return fail(nullptr, ATNS_EINVAL, "bad filter request");
    const std::vector<double> a = filter_coefficients(alpha);
    for (int m = 0; m < 6; ++m) a6[m] = a[m];
    return ATNS_OK;
  });
}

atns_status atns_host_weights(int32_t rk, int32_t mode, int32_t L, double* out) {
  return guarded(nullptr, [&]() -> atns_status {
    if (!out || L < 1 || L > 16 || (rk != ATNS_RK4 && rk != ATNS_LSERK4 && rk != ATNS_LSERK2) ||
        (mode != ATNS_AT && mode != ATNS_AS))
      return fail(nullptr, ATNS_EINVAL, "bad weight-table request");
    const std::vector<double> W = halo_weights(rk, mode, L);
    std::memcpy(out, W.data(), W.size() * sizeof(double));
    return ATNS_OK;
  });
}

atns_status atns_host_delays(int32_t algo, int32_t rk, int64_t n, int32_t nblocks, int32_t L, uint64_t seed,
                             int8_t* out, int32_t* synchronous) {
  return guarded(nullptr, [&]() -> atns_status {
    if (!out || nblocks < 1 || L < 1 || L > 16 || (algo != ATNS_CAA && algo != ATNS_SAA) || n < 0 ||
        (rk != ATNS_RK4 && rk != ATNS_LSERK4 && rk != ATNS_LSERK2))
      return fail(nullptr, ATNS_EINVAL, "bad delay request");
    const bool async = step_delays(algo, n, nblocks, L, levels(rk), seed, nullptr, out);
    if (synchronous) *synchronous = async ? 0 : 1;
    return ATNS_OK;
  });
}

}  // extern "C"

// ============================================================================
// Batches: many independent instances advanced together.
// ============================================================================
struct atns_batch {
  std::vector<atns_ctx*> m;
  hipStream_t user = nullptr;
  hipStream_t s[2] = {nullptr, nullptr};   // Euler chain, Navier-Stokes chain
  hipEvent_t fork = nullptr, join = nullptr, order = nullptr;
  int shape[2][3] = {{16, 16, 8}, {16, 16, 32}};
  std::vector<BatchTile> tl[2];
  BatchTile* d_tl[2] = {nullptr, nullptr};
  int grid[2] = {0, 0};
  void* d_ps = nullptr;                    // StageParams<T>[stages][n]
  long long** d_cnt = nullptr;             // member step counters
  hipGraphExec_t gexec = nullptr;
  std::vector<uint64_t> gen;   // member graph_gen at capture
  int esz = 4;
  int stages = 4;
  std::string err;
};

namespace {

template <class F>
atns_status guarded(const atns_batch* b, F&& f) {
  return guard_body(std::forward<F>(f), b ? &const_cast<atns_batch*>(b)->err : nullptr);
}

atns_status bfail(atns_batch* b, atns_status s, const std::string& msg) {
  if (b) b->err = msg;
  g_err = msg;
  return s;
}

#define BHIP(b, expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return bfail(b, ATNS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

void batch_drop_graph(atns_batch* b) {
  if (!b->gexec) return;
  (void)hipStreamSynchronize(b->s[0]);   // see drop_graphs
  (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
}

// Combined tile list of the members of one physics, XCD-ordered.
atns_status batch_tiles(atns_batch* b, int ph) {
  batch_drop_graph(b);
  std::vector<BatchTile> nat;
  for (int i = 0; i < (int)b->m.size(); ++i) {
    atns_ctx* c = b->m[i];
    if ((c->cfg.physics == ATNS_NS) != (ph == 1)) continue;
    c->tile[0] = b->shape[ph][0];
    c->tile[1] = b->shape[ph][1];
    c->tile[2] = b->shape[ph][2];
    atns_status st = upload_tiles(c);   // the member's own list stays consistent
    if (st != ATNS_OK) return bfail(b, st, c->err);
    for (const TileDev& t : c->tiles)
      if (t.nx > 0) nat.push_back(BatchTile{i, t});
  }
  const size_t chunk = (nat.size() + 7) / 8;
  b->tl[ph].assign(chunk * 8, BatchTile{0, TileDev{0, 0, 0, 0, 0, 0, 0}});
  for (size_t j = 0; j < nat.size(); ++j) b->tl[ph][(j % chunk) * 8 + j / chunk] = nat[j];
  if (b->d_tl[ph]) (void)hipFree(b->d_tl[ph]);
  b->d_tl[ph] = nullptr;
  if (!b->tl[ph].empty()) {
    if (hipMalloc((void**)&b->d_tl[ph], b->tl[ph].size() * sizeof(BatchTile)) != hipSuccess)
      return bfail(b, ATNS_ENOMEM, "batch tile allocation failed");
    BHIP(b, hipMemcpy(b->d_tl[ph], b->tl[ph].data(), b->tl[ph].size() * sizeof(BatchTile), hipMemcpyHostToDevice));
  }
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->m[0]->device);
  // as many persistent workgroups as fit on the device at once (occupancy of
  // the batch kernel of this shape and precision)
  int per_cu = 0;
  const int tx = b->shape[ph][0], ty = b->shape[ph][1];
  hipError_t e;
  if (b->esz == 4)
    e = ph == 1 ? launch_ns_batch<float>(nullptr, nullptr, 0, 0, 0, tx, ty, nullptr, &per_cu)
                : launch_euler_batch<float>(nullptr, nullptr, 0, 0, 0, tx, ty, nullptr, &per_cu);
  else
    e = ph == 1 ? launch_ns_batch<double>(nullptr, nullptr, 0, 0, 0, tx, ty, nullptr, &per_cu)
                : launch_euler_batch<double>(nullptr, nullptr, 0, 0, 0, tx, ty, nullptr, &per_cu);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  b->grid[ph] = (int)std::min<size_t>(b->tl[ph].size(), (size_t)cus * per_cu);
  return ATNS_OK;
}

template <typename T>
atns_status batch_params(atns_batch* b) {
  const int n = (int)b->m.size();
  std::vector<StageParams<T>> ps((size_t)b->stages * n);
  for (int e = 0; e < b->stages; ++e)
    for (int i = 0; i < n; ++i) {
      int kind = 0;
      ps[(size_t)e * n + i] = graph_stage_params<T>(b->m[i], e, &kind, false);
    }
  if (!b->d_ps && hipMalloc(&b->d_ps, ps.size() * sizeof(StageParams<T>)) != hipSuccess)
    return bfail(b, ATNS_ENOMEM, "batch parameter allocation failed");
  BHIP(b, hipMemcpy(b->d_ps, ps.data(), ps.size() * sizeof(StageParams<T>), hipMemcpyHostToDevice));
  return ATNS_OK;
}

template <typename T>
atns_status batch_capture(atns_batch* b) {
  atns_status st = batch_params<T>(b);
  if (st != ATNS_OK) return st;
  const int n = (int)b->m.size();
  hipGraph_t graph = nullptr;
  BHIP(b, hipStreamBeginCapture(b->s[0], hipStreamCaptureModeThreadLocal));
  auto body = [&]() -> atns_status {
    BHIP(b, hipEventRecord(b->fork, b->s[0]));
    BHIP(b, hipStreamWaitEvent(b->s[1], b->fork, 0));
    for (int ph = 0; ph < 2; ++ph) {
      hipStream_t s = b->s[ph];
      for (int i = 0; i < n; ++i) {
        atns_ctx* c = b->m[i];
        if ((c->cfg.physics == ATNS_NS) != (ph == 1)) continue;
        atns_status r = enqueue_graph_halos<T>(c, s);
        if (r != ATNS_OK) return bfail(b, r, c->err);
      }
      if (b->tl[ph].empty()) continue;
      for (int e = 0; e < b->stages; ++e) {
        const StageParams<T>* pe = (const StageParams<T>*)b->d_ps + (size_t)e * n;
        const int kind = e == 0 ? kRK4First : (e == b->stages - 1 ? kRK4Last : kRK4Mid);
        const hipError_t r =
            ph == 0 ? launch_euler_batch<T>(pe, b->d_tl[0], (int)b->tl[0].size(), b->grid[0], kind, b->shape[0][0],
                                           b->shape[0][1], s)
                    : launch_ns_batch<T>(pe, b->d_tl[1], (int)b->tl[1].size(), b->grid[1], kind, b->shape[1][0],
                                        b->shape[1][1], s);
        if (r != hipSuccess) return bfail(b, ATNS_EHIP, std::string("batch stage launch: ") + hipGetErrorString(r));
      }
    }
    BHIP(b, hipEventRecord(b->join, b->s[1]));
    BHIP(b, hipStreamWaitEvent(b->s[0], b->join, 0));
    BHIP(b, launch_step_inc(b->d_cnt, n, b->s[0]));
    return ATNS_OK;
  };
  st = body();
  const hipError_t ec = hipStreamEndCapture(b->s[0], &graph);
  if (st != ATNS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (ec != hipSuccess) return bfail(b, ATNS_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
  const hipError_t ei = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return bfail(b, ATNS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  b->gen.clear();
  for (atns_ctx* c : b->m) b->gen.push_back(c->graph_gen);
  return ATNS_OK;
}

// Orders everything enqueued so far on stream `from` before later work on `to`.
atns_status batch_order(atns_batch* b, hipStream_t from, hipStream_t to) {
  BHIP(b, hipEventRecord(b->order, from));
  BHIP(b, hipStreamWaitEvent(to, b->order, 0));
  return ATNS_OK;
}

template <typename T>
atns_status batch_steps(atns_batch* b, int nsteps) {
  bool on_graph = false;   // the last work of this call went to the graph stream
  atns_status st = ATNS_OK;
  for (int it = 0; it < nsteps && st == ATNS_OK; ++it) {
    const int64_t step = b->m[0]->step;
    bool eager = step < kMaxC;   // members use RK4 (C = 5)
    for (atns_ctx* c : b->m) {
      if (c->step != step) return bfail(b, ATNS_ESTATE, "members are not at the same step");
      if (!c->state_set || !(c->dt > 0)) return bfail(b, ATNS_ESTATE, "member state or dt not set");
      if (c->inject_n > 0 || c->profiling) eager = true;
    }
    if (eager) {
      if (on_graph && (st = batch_order(b, b->s[0], b->user)) != ATNS_OK) break;
      on_graph = false;
      for (atns_ctx* c : b->m) {
        st = atns_rk_step(c, 1);
        if (st != ATNS_OK) return bfail(b, st, c->err);
      }
      continue;
    }
    // A member whose dt, tiles or learned-halo settings changed since the
    // capture invalidates the batch graph too.
    for (size_t i = 0; b->gexec && i < b->m.size(); ++i)
      if (b->m[i]->graph_gen != b->gen[i]) batch_drop_graph(b);
    if (!b->gexec && (st = batch_capture<T>(b)) != ATNS_OK) break;
    if (!on_graph) {
      // Member work (state uploads, eager steps) precedes the graph; the
      // device step counters are written from the host's step numbers.
      if ((st = batch_order(b, b->user, b->s[0])) != ATNS_OK) break;
      for (atns_ctx* c : b->m) BHIP(b, launch_step_set(c->d_nstep, c->step, b->s[0]));
      on_graph = true;
    }
    BHIP(b, hipGraphLaunch(b->gexec, b->s[0]));
    for (atns_ctx* c : b->m) {
      c->step += 1;
      c->nstep_synced = false;
    }
  }
  if (on_graph) {
    const atns_status s2 = batch_order(b, b->s[0], b->user);
    if (st == ATNS_OK) st = s2;
  }
  return st;
}

void batch_release(atns_batch* b) {
  batch_drop_graph(b);
  for (atns_ctx* c : b->m) atns_destroy(c);
  b->m.clear();
  for (BatchTile*& t : b->d_tl)
    if (t) {
      (void)hipFree(t);
      t = nullptr;
    }
  if (b->d_ps) (void)hipFree(b->d_ps);
  if (b->d_cnt) (void)hipFree(b->d_cnt);
  for (hipStream_t& s : b->s)
    if (s) (void)hipStreamDestroy(s);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->join) (void)hipEventDestroy(b->join);
  if (b->order) (void)hipEventDestroy(b->order);
}

}  // namespace

extern "C" {

atns_status atns_batch_create(const atns_config* cfgs, int32_t n, void* stream, atns_batch** out) {
  return guarded(nullptr, [&]() -> atns_status {
    if (!out || !cfgs || n < 1) return bfail(nullptr, ATNS_EINVAL, "bad batch arguments");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
      if (cfgs[i].rk != ATNS_RK4) return bfail(nullptr, ATNS_EINVAL, "batch members use classical RK4");
      if (cfgs[i].precision != cfgs[0].precision) return bfail(nullptr, ATNS_EINVAL, "batch members share precision");
      if (cfgs[i].ndim != 3) return bfail(nullptr, ATNS_EINVAL, "batch members are three-dimensional");
      if (cfgs[i].filter) return bfail(nullptr, ATNS_EINVAL, "batch members run without the filter");
    }
    auto* b = new atns_batch();
    b->user = (hipStream_t)stream;
    b->esz = cfgs[0].precision == ATNS_F64 ? 8 : 4;
    for (int i = 0; i < n; ++i) {
      atns_ctx* c = nullptr;
      atns_status st = atns_create(&cfgs[i], stream, &c);
      if (st != ATNS_OK) {
        batch_release(b);
        delete b;
        return st;
      }
      c->batch_member = true;
      b->m.push_back(c);
    }
    auto bad = [&](atns_status s, const char* m) {
      batch_release(b);
      delete b;
      return bfail(nullptr, s, m);
    };
    if (hipStreamCreate(&b->s[0]) != hipSuccess || hipStreamCreate(&b->s[1]) != hipSuccess ||
        hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->order, hipEventDisableTiming) != hipSuccess)
      return bad(ATNS_EHIP, "batch stream creation failed");
    std::vector<long long*> cnt;
    for (atns_ctx* c : b->m) cnt.push_back(c->d_nstep);
    if (hipMalloc((void**)&b->d_cnt, cnt.size() * sizeof(long long*)) != hipSuccess ||
        hipMemcpy(b->d_cnt, cnt.data(), cnt.size() * sizeof(long long*), hipMemcpyHostToDevice) != hipSuccess)
      return bad(ATNS_EHIP, "batch counter table failed");
    for (int ph = 0; ph < 2; ++ph)
      if (batch_tiles(b, ph) != ATNS_OK) return bad(ATNS_EHIP, "batch tile table failed");
    *out = b;
    return ATNS_OK;
  });
}

atns_status atns_batch_destroy(atns_batch* b) {
  return guarded(b, [&]() -> atns_status {
    if (!b) return ATNS_OK;
    (void)hipDeviceSynchronize();
    batch_release(b);
    delete b;
    return ATNS_OK;
  });
}

const char* atns_batch_last_error(const atns_batch* b) { return b ? b->err.c_str() : g_err.c_str(); }

atns_status atns_batch_member(atns_batch* b, int32_t i, atns_ctx** ctx) {
  return guarded(b, [&]() -> atns_status {
    if (!b || !ctx || i < 0 || i >= (int)b->m.size()) return bfail(b, ATNS_EINVAL, "bad member index");
    *ctx = b->m[i];
    return ATNS_OK;
  });
}

atns_status atns_batch_set_tiles(atns_batch* b, int32_t physics, int32_t tx, int32_t ty, int32_t tz) {
  return guarded(b, [&]() -> atns_status {
    if (!b || (physics != ATNS_EULER && physics != ATNS_NS)) return bfail(b, ATNS_EINVAL, "bad physics");
    if (!shape_supported(physics, b->esz, tx, ty) || tz < 1) return bfail(b, ATNS_EINVAL, "unsupported tile shape");
    BHIP(b, hipDeviceSynchronize());
    const int ph = physics == ATNS_NS ? 1 : 0;
    b->shape[ph][0] = tx;
    b->shape[ph][1] = ty;
    b->shape[ph][2] = tz;
    return batch_tiles(b, ph);
  });
}

atns_status atns_batch_step(atns_batch* b, int32_t nsteps) {
  return guarded(b, [&]() -> atns_status {
    if (!b || nsteps < 0) return bfail(b, ATNS_EINVAL, "bad arguments");
    return b->esz == 4 ? batch_steps<float>(b, nsteps) : batch_steps<double>(b, nsteps);
  });
}

}  // extern "C"

namespace {

// Average time of one step's batch stage kernels (first, middle and last RK
// stage over the combined tile lists, with the current tiles and grids) of
// the physics in `mask` (bit 0 Euler, bit 1 Navier-Stokes; both: the two run
// concurrently on their own streams, as in a batch step), as timing probes
// that leave every member's state intact.
template <typename T>
atns_status batch_time(atns_batch* b, int mask, int reps, float* ms_out) {
  const int n = (int)b->m.size();
  for (int i = 0; i < n; ++i) {   // members with delayed halos: their stage-halo buffers
    const atns_status st = probe_halos<T>(b->m[i]);
    if (st != ATNS_OK) return bfail(b, st, b->m[i]->err);
  }
  BHIP(b, hipDeviceSynchronize());
  std::vector<StageParams<T>> ps((size_t)b->stages * n);
  std::vector<int> kinds(b->stages);
  for (int e = 0; e < b->stages; ++e)
    for (int i = 0; i < n; ++i) ps[(size_t)e * n + i] = probe_stage<T>(b->m[i], e, &kinds[e]);
  StageParams<T>* d = nullptr;
  BHIP(b, hipMalloc(&d, ps.size() * sizeof(StageParams<T>)));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto run = [&]() -> atns_status {
    BHIP(b, hipMemcpy(d, ps.data(), ps.size() * sizeof(StageParams<T>), hipMemcpyHostToDevice));
    BHIP(b, hipEventCreate(&e0));
    BHIP(b, hipEventCreate(&e1));
    auto pass = [&](int ph) -> hipError_t {
      for (int e = 0; e < b->stages; ++e) {
        const StageParams<T>* pe = d + (size_t)e * n;
        const hipError_t r =
            ph == 0 ? launch_euler_batch<T>(pe, b->d_tl[0], (int)b->tl[0].size(), b->grid[0], kinds[e],
                                           b->shape[0][0], b->shape[0][1], b->s[0])
                    : launch_ns_batch<T>(pe, b->d_tl[1], (int)b->tl[1].size(), b->grid[1], kinds[e],
                                        b->shape[1][0], b->shape[1][1], b->s[1]);
        if (r != hipSuccess) return r;
      }
      return hipSuccess;
    };
    auto passes = [&](int count) -> atns_status {
      BHIP(b, hipEventRecord(b->fork, b->s[0]));
      BHIP(b, hipStreamWaitEvent(b->s[1], b->fork, 0));
      for (int ph = 0; ph < 2; ++ph)
        if ((mask >> ph & 1) && !b->tl[ph].empty())
          for (int r = 0; r < count; ++r) BHIP(b, pass(ph));
      BHIP(b, hipEventRecord(b->join, b->s[1]));
      BHIP(b, hipStreamWaitEvent(b->s[0], b->join, 0));
      return ATNS_OK;
    };
    atns_status st = passes(1);   // warm
    if (st != ATNS_OK) return st;
    BHIP(b, hipEventRecord(e0, b->s[0]));
    if ((st = passes(reps)) != ATNS_OK) return st;
    BHIP(b, hipEventRecord(e1, b->s[0]));
    BHIP(b, hipEventSynchronize(e1));
    float ms = 0.f;
    BHIP(b, hipEventElapsedTime(&ms, e0, e1));
    *ms_out = ms / reps;
    return ATNS_OK;
  };
  const atns_status st = run();
  (void)hipDeviceSynchronize();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(d);
  return st;
}

}  // namespace

extern "C" {

atns_status atns_batch_autotune(atns_batch* b, int32_t reps, int32_t* best) {
  return guarded(b, [&]() -> atns_status {
    if (!b || reps < 1) return bfail(b, ATNS_EINVAL, "bad arguments");
    for (atns_ctx* c : b->m)
      if (!c->state_set) return bfail(b, ATNS_ESTATE, "member state not set");
    BHIP(b, hipDeviceSynchronize());
    // Every shape of each physics is timed with the batch kernels themselves
    // over the combined tile list of all members of that physics (timing
    // probes on the current states, which stay untouched).  The two physics
    // share the device during a batch step, so the three fastest shapes of
    // each are then timed in pairs, running concurrently, and the fastest pair
    // is kept.
    constexpr int kTop = 3;
    std::vector<std::array<int, 3>> top[2];
    auto timer = [&](int mask, float* ms) {
      return b->esz == 4 ? batch_time<float>(b, mask, reps, ms) : batch_time<double>(b, mask, reps, ms);
    };
    for (int ph = 0; ph < 2; ++ph) {
      const int phys = ph ? ATNS_NS : ATNS_EULER;
      if (b->tl[ph].empty()) {
        top[ph].push_back({b->shape[ph][0], b->shape[ph][1], b->shape[ph][2]});
        continue;
      }
      std::vector<std::pair<float, std::array<int, 3>>> timed;
      for (int i = 0; i < num_shapes(phys, b->esz); ++i)
        for (int tz : {4, 8, 16, 32}) {
          if (ph == 1 && tz < 8) continue;
          const int tx = shape_at(phys, i)[0], ty = shape_at(phys, i)[1];
          atns_status st = atns_batch_set_tiles(b, phys, tx, ty, tz);
          if (st != ATNS_OK) return st;
          float ms = 0.f;
          if ((st = timer(1 << ph, &ms)) != ATNS_OK) return st;
          timed.push_back({ms, {tx, ty, tz}});
        }
      std::stable_sort(timed.begin(), timed.end(),
                       [](const auto& x, const auto& y) { return x.first < y.first; });
      for (int i = 0; i < kTop && i < (int)timed.size(); ++i) top[ph].push_back(timed[i].second);
    }
    float best_ms = 1e30f;
    std::array<int, 3> pick[2] = {top[0][0], top[1][0]};
    for (const auto& eu : top[0])
      for (const auto& ns : top[1]) {
        atns_status st = atns_batch_set_tiles(b, ATNS_EULER, eu[0], eu[1], eu[2]);
        if (st == ATNS_OK) st = atns_batch_set_tiles(b, ATNS_NS, ns[0], ns[1], ns[2]);
        if (st != ATNS_OK) return st;
        float ms = 0.f;
        if ((st = timer(3, &ms)) != ATNS_OK) return st;
        if (ms < best_ms) {
          best_ms = ms;
          pick[0] = eu;
          pick[1] = ns;
        }
      }
    for (int ph = 0; ph < 2; ++ph) {
      const atns_status st = atns_batch_set_tiles(b, ph ? ATNS_NS : ATNS_EULER, pick[ph][0], pick[ph][1], pick[ph][2]);
      if (st != ATNS_OK) return st;
    }
    if (best)
      for (int ph = 0; ph < 2; ++ph)
        for (int d = 0; d < 3; ++d) best[ph * 3 + d] = b->shape[ph][d];
    return ATNS_OK;
  });
}

}  // extern "C"
