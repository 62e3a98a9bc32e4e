// Host-side tables of the AT method: RK coefficients, per-stage halo
// weights and the delay schedules.  Plain C++, no device code.
#pragma once
#include <cstdint>
#include <vector>

namespace atns {

constexpr int kMaxC = 5;       // most delayed levels of any scheme (AT4)
constexpr int kSlots = 18;     // 6 faces + 12 edges

// Delayed levels C of the AT scheme paired with an integrator: AT4,
// (d, q, r) = (1, 4, 1), C = 5 with RK4 and LSERK4; AT2, (1, 2, 1), C = 3
// with LSERK2 (Table 1).
int levels(int rk);

struct RKScheme {
  int stages;                  // s
  // Classical RK4: stage e input Y_e = U + dt * sum_{j<e} a[e][j] k_j,
  // U^{n+1} = U + dt * sum b_j k_j.  LSERK (Eq. 3): A[m], B[m], m = 0..s-1.
  double a[5][5];
  double b[5];
  double A[5];
  double B[5];
  bool low_storage;
};

RKScheme make_rk(int rk);      // rk: ATNS_RK4, ATNS_LSERK4 or ATNS_LSERK2

// W[e][k][l], e < s, k < L, l < C = levels(rk).  mode: ATNS_AT or ATNS_AS.
std::vector<double> halo_weights(int rk, int mode, int L);

// Tenth-order Pade filter (Sec. 2): alpha f^[i-1] + f^[i] + alpha f^[i+1]
// = sum_{m=0..5} (a_m/2)(f[i+m] + f[i-m]).  The six a_m solve T(pi) = 0 and
// sum_m a_m m^{2p} = [p == 0] + 2 alpha for p = 0..4 (the w^0..w^8 Taylor
// coefficients of numerator and denominator of the transfer function
// agree).  Returns a_0..a_5.
std::vector<double> filter_coefficients(double alpha);

// Weights [k][l] (k < L, l < C = levels(rk)) of the C delayed levels
// U^{n-k-l} that give a filter halo value at level n+1: AT the Lagrange
// extrapolation of Eqs. 14-15 at delay k+1, AS the newest level.
std::vector<double> filter_halo_weights(int rk, int mode, int L);

// Forward-elimination factors of the block filter's tridiagonal system (1
// on the diagonal, alpha beside it), rows 0..n-1: inv[0] = 1, cp[0] = alpha,
// inv[i] = 1 / (1 - alpha cp[i-1]), cp[i] = alpha inv[i].  The factors of
// row i do not depend on the line length, so one table serves every block.
void filter_thomas(double alpha, int n, std::vector<double>& inv, std::vector<double>& cp);

// SplitMix64 draw i of stream `seed`.
uint64_t splitmix64(uint64_t seed, uint64_t i);

// Delays of step n after the Alg. 3 guard (override may be null), for a
// scheme with C delayed levels.  Returns false (and zeros) for a synchronous
// step (n < C).
bool step_delays(int algo, int64_t n, int nblocks, int L, int C, uint64_t seed,
                 const int8_t* override_k, int8_t* out);

}  // namespace atns
