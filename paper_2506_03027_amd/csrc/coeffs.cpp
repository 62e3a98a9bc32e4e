// Host-side tables of the AT method.
//
// Halo weights.  A halo point holds C delayed levels U^{n-k-l}, l = 0..C-1,
// at times tau_l = -(k+l) (units of dt, relative to t_n).  Let p(tau) be
// their degree-(C-1) interpolant.  The AT buffer value at RK stage e is
//
//     Uhat^(e) = sum_j nu_j^e p^{(j)}(0),
//
// where nu_j^e are the coefficients of stage e's polynomial in z = lambda dt
// for the linear test equation (Sec. 3.1, Eqs. 9-10).  Stage 0 is the buffer
// extrapolation of Eqs. 14-15; later stages are what the buffer recursion of
// Eq. (8) produces when the temporal derivative of Eq. (12) (the weights
// that reproduce sum_j nu_j^e dt^j p^{(j+1)}(t_n)) replaces the spatial
// residual.  All arithmetic here is long double; the result is stored as
// double and applied in FP64 on the device.
#include "coeffs.hpp"

#include <cmath>
#include <cstring>
#include <utility>

#include "atns.h"

namespace atns {

int levels(int rk) { return rk == ATNS_LSERK2 ? 3 : 5; }

RKScheme make_rk(int rk) {
  RKScheme s{};
  if (rk == ATNS_LSERK2) {
    // Two-stage LSERK2, App. B: A = {0, -1/2}, B = {1/2, 1}
    s.stages = 2;
    s.low_storage = true;
    s.A[0] = 0.0;
    s.A[1] = -0.5;
    s.B[0] = 0.5;
    s.B[1] = 1.0;
  } else if (rk == ATNS_RK4) {
    s.stages = 4;
    s.low_storage = false;
    s.a[1][0] = 0.5;
    s.a[2][1] = 0.5;
    s.a[3][2] = 1.0;
    s.b[0] = 1.0 / 6.0;
    s.b[1] = 1.0 / 3.0;
    s.b[2] = 1.0 / 3.0;
    s.b[3] = 1.0 / 6.0;
  } else {
    // Five-stage LSERK4, App. B Table 4 (eight printed digits).
    static const double A[5] = {0.0, -0.4812317, -1.0495626, -1.6025296, -1.7782672};
    static const double B[5] = {0.09761835, 0.41225329, 0.44021696, 1.42631146, 0.19787605};
    s.stages = 5;
    s.low_storage = true;
    for (int m = 0; m < 5; ++m) {
      s.A[m] = A[m];
      s.B[m] = B[m];
    }
  }
  return s;
}

namespace {

using Poly = std::vector<long double>;  // ascending coefficients

Poly mul(const Poly& p, const Poly& q) {
  Poly r(p.size() + q.size() - 1, 0.0L);
  for (size_t i = 0; i < p.size(); ++i)
    for (size_t j = 0; j < q.size(); ++j) r[i + j] += p[i] * q[j];
  return r;
}

Poly add(const Poly& p, const Poly& q) {
  Poly r(std::max(p.size(), q.size()), 0.0L);
  for (size_t i = 0; i < p.size(); ++i) r[i] += p[i];
  for (size_t i = 0; i < q.size(); ++i) r[i] += q[i];
  return r;
}

Poly scale(const Poly& p, long double a) {
  Poly r(p);
  for (auto& c : r) c *= a;
  return r;
}

// Stage polynomials of the scheme (stage inputs e = 0..s-1).
std::vector<Poly> stage_polys(int rk) {
  std::vector<Poly> out;
  const Poly one{1.0L}, z{0.0L, 1.0L};
  if (rk == ATNS_RK4) {
    const long double a[4][4] = {{0, 0, 0, 0}, {0.5L, 0, 0, 0}, {0, 0.5L, 0, 0}, {0, 0, 1, 0}};
    for (int e = 0; e < 4; ++e) {
      Poly acc{0.0L};
      for (int j = 0; j < e; ++j) acc = add(acc, scale(out[j], a[e][j]));
      out.push_back(add(one, mul(z, acc)));
    }
    return out;
  }
  const RKScheme s = make_rk(rk);
  Poly U = one, Q{0.0L};
  out.push_back(U);
  for (int m = 0; m < s.stages - 1; ++m) {
    Q = add(scale(Q, s.A[m]), mul(z, U));
    U = add(U, scale(Q, s.B[m]));
    out.push_back(U);
  }
  return out;
}

// d^j/dtau^j of the Lagrange basis polynomial of level l (of C levels), at
// tau = 0.
long double basis_derivative(int k, int l, int j, int C) {
  Poly p{1.0L};
  long double denom = 1.0L;
  const long double tl = -(long double)(k + l);
  for (int m = 0; m < C; ++m) {
    if (m == l) continue;
    const long double tm = -(long double)(k + m);
    p = mul(p, Poly{-tm, 1.0L});
    denom *= (tl - tm);
  }
  if (j >= (int)p.size()) return 0.0L;
  long double fact = 1.0L;
  for (int i = 2; i <= j; ++i) fact *= i;
  return p[j] * fact / denom;
}

}  // namespace

std::vector<double> halo_weights(int rk, int mode, int L) {
  const int s = make_rk(rk).stages;
  const int C = levels(rk);
  std::vector<double> W((size_t)s * L * C, 0.0);
  const std::vector<Poly> nu = stage_polys(rk);
  for (int e = 0; e < s; ++e)
    for (int k = 0; k < L; ++k)
      for (int l = 0; l < C; ++l) {
        long double w = 0.0L;
        if (mode == ATNS_AT) {
          for (int j = 0; j < (int)nu[e].size() && j < C; ++j)
            w += nu[e][j] * basis_derivative(k, l, j, C);
        } else {
          w = (l == 0) ? 1.0L : 0.0L;
        }
        W[((size_t)e * L + k) * C + l] = (double)w;
      }
  return W;
}

std::vector<double> filter_coefficients(double alpha) {
  // 6 x 6 system, Gaussian elimination with partial pivoting in long double
  long double M[6][7];
  for (int p = 0; p < 5; ++p) {
    for (int m = 0; m < 6; ++m) {
      long double v = 1.0L;
      for (int q = 0; q < 2 * p; ++q) v *= (long double)m;
      M[p][m] = v;   // m^{2p}, with 0^0 = 1
    }
    M[p][6] = (p == 0 ? 1.0L : 0.0L) + 2.0L * (long double)alpha;
  }
  for (int m = 0; m < 6; ++m) M[5][m] = (m & 1) ? -1.0L : 1.0L;
  M[5][6] = 0.0L;
  for (int col = 0; col < 6; ++col) {
    int piv = col;
    for (int r = col + 1; r < 6; ++r)
      if (std::fabs((double)M[r][col]) > std::fabs((double)M[piv][col])) piv = r;
    for (int j = 0; j < 7; ++j) std::swap(M[col][j], M[piv][j]);
    for (int r = 0; r < 6; ++r) {
      if (r == col) continue;
      const long double f = M[r][col] / M[col][col];
      for (int j = col; j < 7; ++j) M[r][j] -= f * M[col][j];
    }
  }
  std::vector<double> a(6);
  for (int m = 0; m < 6; ++m) a[m] = (double)(M[m][6] / M[m][m]);
  return a;
}

std::vector<double> filter_halo_weights(int rk, int mode, int L) {
  const int C = levels(rk);
  std::vector<double> W((size_t)L * C, 0.0);
  for (int k = 0; k < L; ++k)
    for (int l = 0; l < C; ++l)
      W[(size_t)k * C + l] = mode == ATNS_AT ? (double)basis_derivative(k + 1, l, 0, C) : (l == 0 ? 1.0 : 0.0);
  return W;
}

void filter_thomas(double alpha, int n, std::vector<double>& inv, std::vector<double>& cp) {
  inv.assign(n, 1.0);
  cp.assign(n, alpha);
  long double c = alpha;
  for (int i = 1; i < n; ++i) {
    const long double m = 1.0L / (1.0L - (long double)alpha * c);
    c = (long double)alpha * m;
    inv[i] = (double)m;
    cp[i] = (double)c;
  }
}

// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output i of the generator
// seeded with `seed` is mix(seed + (i + 1) * golden).
uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

bool step_delays(int algo, int64_t n, int nblocks, int L, int C, uint64_t seed,
                 const int8_t* override_k, int8_t* out) {
  const size_t cnt = (size_t)nblocks * kSlots;
  if (n < C) {  // Alg. 2/3: the first C steps are synchronous
    std::memset(out, 0, cnt);
    return false;
  }
  for (int b = 0; b < nblocks; ++b)
    for (int v = 0; v < kSlots; ++v) {
      const size_t idx = (size_t)b * kSlots + v;
      int64_t k;
      if (override_k) {
        k = override_k[idx];
      } else if (algo == ATNS_CAA) {
        k = (n - C) % L;  // period-L refresh, delay 0 right after it
      } else {
        const uint64_t draw = ((uint64_t)n * (uint64_t)nblocks + (uint64_t)b) * kSlots + v;
        k = (int64_t)(splitmix64(seed, draw) % (uint64_t)L);
      }
      // Alg. 3 guard: too stale, or levels not (yet) available -> wait, k = 0
      if (k < 0 || k > L - 1 || k > n - C + 1) k = 0;
      out[idx] = (int8_t)k;
    }
  return true;
}

}  // namespace atns
