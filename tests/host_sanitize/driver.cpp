// Host-side exercise of the C ABI for AddressSanitizer / UndefinedBehavior-
// Sanitizer builds (only the host code is instrumented; device code is
// built as usual).  Calls only include/atns.h.
//
//   driver cpu   validation and error paths, host tables, null arguments;
//                contexts fail at the device query without a GPU
//   driver gpu   whole lifecycles on the device: graph-captured steps,
//                tile changes (graph drop and re-capture), checkpoint and
//                restore, the filter, and a batch stepped, re-tiled, tuned
//                and stepped again
//
// Prints one line per stage and "driver ok" at the end; any unexpected
// status ends it with exit code 1 (sanitizer findings end it themselves).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include <unistd.h>

#include <hip/hip_runtime_api.h>

#include "atns.h"

static int g_fail = 0;

#define EXPECT(cond, what)                                                  \
  do {                                                                      \
    if (!(cond)) {                                                          \
      std::printf("FAILED: %s (line %d)\n", what, __LINE__);                \
      g_fail = 1;                                                           \
    }                                                                       \
  } while (0)

static atns_config base_config() {
  atns_config c;
  std::memset(&c, 0, sizeof c);
  c.ndim = 3;
  for (int d = 0; d < 3; ++d) {
    c.n[d] = 32;
    c.len[d] = 2.0 * M_PI;
    c.nblk[d] = 2;
  }
  c.physics = ATNS_NS;
  c.gamma = 1.4;
  c.mach = 0.1;
  c.re = 1600.0;
  c.pr = 0.71;
  c.rk = ATNS_RK4;
  c.mode = ATNS_AT;
  c.algo = ATNS_SAA;
  c.L = 4;
  c.seed = 3;
  c.precision = ATNS_F32;
  return c;
}

static void cpu_paths() {
  // invalid configurations: rejected before any device call
  atns_ctx* ctx = nullptr;
  atns_config c = base_config();
  c.L = 0;
  EXPECT(atns_create(&c, nullptr, &ctx) == ATNS_EINVAL && !ctx, "L = 0 rejected");
  c = base_config();
  c.nblk[0] = 16;   // 2-point blocks
  EXPECT(atns_create(&c, nullptr, &ctx) == ATNS_EINVAL, "thin blocks rejected");
  c = base_config();
  int32_t split[2] = {10, 10};
  c.split[0] = split;
  EXPECT(atns_create(&c, nullptr, &ctx) == ATNS_EINVAL, "split not summing to n rejected");
  c = base_config();
  c.filter = 1;
  c.filter_alpha = 0.7;
  EXPECT(atns_create(&c, nullptr, &ctx) == ATNS_EINVAL, "filter alpha rejected");
  c = base_config();
  c.ndim = 2;
  EXPECT(atns_create(&c, nullptr, &ctx) == ATNS_EINVAL, "2-D with nz != 1 rejected");
  EXPECT(atns_create(nullptr, nullptr, &ctx) == ATNS_EINVAL, "null config");
  EXPECT(atns_create(&c, nullptr, nullptr) == ATNS_EINVAL, "null output");
  std::printf("validation ok\n");

  // host tables
  std::vector<double> W(5 * 16 * 5);
  for (int rk : {ATNS_RK4, ATNS_LSERK4, ATNS_LSERK2})
    for (int L : {1, 4, 5, 16}) EXPECT(atns_host_weights(rk, ATNS_AT, L, W.data()) == ATNS_OK, "weights");
  EXPECT(atns_host_weights(ATNS_RK4, ATNS_AT, 17, W.data()) == ATNS_EINVAL, "weights L = 17");
  std::vector<int8_t> k(64 * ATNS_NSLOTS);
  int32_t sync = 0;
  for (int64_t n : {0, 4, 5, 123456789})
    EXPECT(atns_host_delays(ATNS_SAA, ATNS_RK4, n, 64, 5, 77, k.data(), &sync) == ATNS_OK, "delays");
  double a6[6];
  EXPECT(atns_host_filter_coefficients(0.499, a6) == ATNS_OK && std::fabs(a6[0] - 0.9995078125) < 1e-12,
         "filter coefficients");
  std::printf("host tables ok\n");

  // null handles on every entry point that takes one
  EXPECT(atns_destroy(nullptr) == ATNS_OK, "destroy null");
  EXPECT(atns_rk_step(nullptr, 1) == ATNS_EINVAL, "step null");
  EXPECT(atns_rhs(nullptr, 0, nullptr) == ATNS_EINVAL, "rhs null");
  EXPECT(atns_filter_state(nullptr) == ATNS_EINVAL, "filter null");
  EXPECT(atns_set_compensation(nullptr, 1) == ATNS_EINVAL, "compensation null");
  EXPECT(atns_set_filter_fusion(nullptr, 1) == ATNS_EINVAL, "filter fusion null");
  EXPECT(atns_set_dt(nullptr, 1.0) == ATNS_EINVAL, "dt null");
  size_t bytes = 0;
  EXPECT(atns_checkpoint(nullptr, nullptr, &bytes) == ATNS_EINVAL, "checkpoint null");
  EXPECT(atns_restore(nullptr, "x", 1) == ATNS_EINVAL, "restore null");
  EXPECT(atns_batch_create(nullptr, 0, nullptr, nullptr) == ATNS_EINVAL, "batch null");
  EXPECT(atns_batch_destroy(nullptr) == ATNS_OK, "batch destroy null");
  std::printf("null handles ok\n");

  // a valid context: without a device creation stops at the device query
  c = base_config();
  const atns_status st = atns_create(&c, nullptr, &ctx);
  EXPECT(st == ATNS_OK || st == ATNS_EHIP, "valid config");
  if (st == ATNS_OK) atns_destroy(ctx);
  atns_config bc[2] = {base_config(), base_config()};
  bc[1].physics = ATNS_EULER;
  atns_batch* b = nullptr;
  const atns_status sb = atns_batch_create(bc, 2, nullptr, &b);
  EXPECT(sb == ATNS_OK || sb == ATNS_EHIP, "valid batch");
  if (sb == ATNS_OK) atns_batch_destroy(b);
  std::printf("contexts ok\n");
}

static void check(atns_status s, const char* what, const atns_ctx* c) {
  if (s != ATNS_OK) {
    std::printf("FAILED: %s: %d %s\n", what, (int)s, atns_last_error(c));
    g_fail = 1;
  }
}

static atns_ctx* make_ctx(const atns_config& cfg, double dt) {
  atns_ctx* c = nullptr;
  check(atns_create(&cfg, nullptr, &c), "create", nullptr);
  if (!c) return nullptr;
  check(atns_init_case(c, ATNS_CASE_TGV, nullptr, 0, 0), "init_case", c);
  check(atns_set_dt(c, dt), "set_dt", c);
  return c;
}

static void gpu_paths() {
  const double dt = 2e-3;
  // one context through graph steps, tile changes and restart
  atns_config cfg = base_config();
  atns_ctx* c = make_ctx(cfg, dt);
  if (!c) return;
  check(atns_rk_step(c, 8), "steps", c);
  check(atns_set_tiles(c, 32, 8, 16), "tiles", c);
  check(atns_rk_step(c, 3), "steps after tiles", c);
  size_t bytes = 0;
  check(atns_checkpoint(c, nullptr, &bytes), "checkpoint size", c);
  std::vector<char> blob(bytes);
  check(atns_checkpoint(c, blob.data(), &bytes), "checkpoint", c);
  check(atns_rk_step(c, 2), "steps", c);
  check(atns_restore(c, blob.data(), bytes), "restore", c);
  check(atns_set_graphs(c, 0), "graphs off", c);
  check(atns_rk_step(c, 2), "eager steps", c);
  check(atns_set_graphs(c, 1), "graphs on", c);
  check(atns_rk_step(c, 2), "graph steps", c);
  void* R = nullptr;
  (void)hipMalloc(&R, (size_t)5 * 32 * 32 * 32 * sizeof(float));
  check(atns_rhs(c, 2, R), "rhs", c);
  double diag[ATNS_NDIAG];
  check(atns_reduce(c, diag), "reduce", c);
  int32_t best[3];
  check(atns_autotune(c, 1, nullptr, best), "autotune", c);
  check(atns_rk_step(c, 2), "steps after tuning", c);
  check(atns_set_compensation(c, 1), "compensation on", c);
  check(atns_rk_step(c, 3), "compensated steps", c);
  check(atns_set_compensation(c, 0), "compensation off", c);
  (void)hipFree(R);
  check(atns_destroy(c), "destroy", nullptr);
  std::printf("context lifecycle ok\n");

  // the filter
  cfg = base_config();
  cfg.filter = 1;
  cfg.filter_alpha = 0.499;
  c = make_ctx(cfg, dt);
  if (c) {
    check(atns_filter_state(c), "filter", c);
    check(atns_rk_step(c, 9), "filtered steps", c);
    check(atns_set_filter_fusion(c, 0), "filter fusion off", c);
    check(atns_rk_step(c, 2), "filtered steps, per-axis passes", c);
    check(atns_destroy(c), "destroy", nullptr);
  }
  std::printf("filter ok\n");

  // a batch: warm-up, graph steps, re-tiling, tuning, more steps
  std::vector<atns_config> bc(4, base_config());
  bc[1].physics = ATNS_EULER;
  bc[3].physics = ATNS_EULER;
  bc[2].n[0] = 48;
  bc[2].nblk[0] = 3;
  bc[3].L = 2;
  atns_batch* b = nullptr;
  atns_status s = atns_batch_create(bc.data(), 4, nullptr, &b);
  if (s != ATNS_OK) {
    std::printf("FAILED: batch create %d %s\n", (int)s, atns_batch_last_error(nullptr));
    g_fail = 1;
    return;
  }
  for (int i = 0; i < 4; ++i) {
    atns_ctx* m = nullptr;
    check(atns_batch_member(b, i, &m) == ATNS_OK ? ATNS_OK : ATNS_EINVAL, "member", nullptr);
    check(atns_init_case(m, bc[i].physics == ATNS_NS ? ATNS_CASE_TGV : ATNS_CASE_VORTEX, nullptr, 0, 0), "member init", m);
    check(atns_set_dt(m, dt), "member dt", m);
  }
  auto bcheck = [&](atns_status st, const char* what) {
    if (st != ATNS_OK) {
      std::printf("FAILED: %s: %d %s\n", what, (int)st, atns_batch_last_error(b));
      g_fail = 1;
    }
  };
  bcheck(atns_batch_step(b, 8), "batch steps");
  bcheck(atns_batch_set_tiles(b, ATNS_NS, 32, 8, 16), "batch tiles");
  bcheck(atns_batch_step(b, 3), "batch steps after tiles");
  int32_t bb[6];
  bcheck(atns_batch_autotune(b, 1, bb), "batch autotune");
  bcheck(atns_batch_step(b, 3), "batch steps after tuning");
  bcheck(atns_batch_destroy(b), "batch destroy");
  std::printf("batch lifecycle ok\n");
}

int main(int argc, char** argv) {
  std::setvbuf(stdout, nullptr, _IONBF, 0);
  if (argc < 2 || (std::strcmp(argv[1], "cpu") && std::strcmp(argv[1], "gpu"))) {
    std::printf("usage: driver cpu|gpu\n");
    return 2;
  }
  cpu_paths();
  if (!std::strcmp(argv[1], "gpu")) gpu_paths();
  std::printf(g_fail ? "driver FAILED\n" : "driver ok\n");
  // Leave without the static destructors: the HIP runtime's own teardown
  // frees device-runtime memory after ROCm's sanitizer allocator has been
  // told the runtime is gone, which trips a check inside that allocator.
  // Every context and batch was destroyed above.
  _exit(g_fail);
}
