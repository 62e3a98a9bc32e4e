// Tenth-order Pade low-pass filter (Sec. 2), one axis per launch.
//
// Every block filters its own grid lines along the pass axis:
//
//   alpha f^[i-1] + f^[i] + alpha f^[i+1] = sum_{m=0..5} (a_m/2)(f[i+m] + f[i-m]),
//
// i = 0..n-1 over the block's points of the line, with f^[-1] and f^[n]
// replaced by the halo values f[-1], f[n] (so blocks solve independently)
// and the right-hand side reading halo points i = -5..-1 and n..n+4.  One
// thread per line walks it once forward (right-hand side from an 11-point
// register window, forward elimination into LDS) and once backward (back
// substitution, store).  Arithmetic in FP64; the result is rounded to T.
//
// Halo points come from the pass input at the periodic neighbour position
// (synchronous steps: the neighbours' current values) or from the
// filter-halo slot of the stage-halo buffer, assembled by halo_kernel from
// the delayed levels (AT: extrapolated to the new level; AS: the newest).
#include "kernels_common.hpp"
#include "launch.hpp"

namespace atns {

constexpr int kFilterLines = 64;   // lines (threads) per workgroup

template <typename T>
__global__ void __launch_bounds__(kFilterLines) filter_pass_kernel(const FilterArgs<T> f) {
  extern __shared__ double sD[];   // [len][kFilterLines] forward-eliminated values
  const BlockDev* __restrict__ B = f.blocks + blockIdx.y;
  const int d = f.dir;
  // the other two axes: p (fastest across threads) and q
  const int pa = d == 0 ? 1 : 0, qa = d == 2 ? 1 : 2;
  const int len = B->s[d];
  const int li = blockIdx.x * kFilterLines + threadIdx.x;
  if (li >= B->s[pa] * B->s[qa]) return;   // no barriers below
  int loc[3];
  loc[d] = 0;
  loc[pa] = li % B->s[pa];
  loc[qa] = li / B->s[pa];

  int halo = f.halo;
  if (f.nstep) halo = (*f.nstep - 1 >= f.C) ? f.async_halo : kHaloSync;
  const bool sync = halo == kHaloSync || f.fhalo == nullptr;

  const long long nxy = (long long)f.n[0] * f.n[1];
  const long long st = d == 0 ? 1 : (d == 1 ? f.n[0] : nxy);   // global stride along the line
  const long long g0 = (long long)(B->o[2] + loc[2]) * nxy + (long long)(B->o[1] + loc[1]) * f.n[0] +
                       (B->o[0] + loc[0]);
  // delayed halos: region of the low (-d) and high (+d) face, per-variable
  // stride, and this line's offset in a layer (x-faces [s_z][s_y][H],
  // y-faces [s_z][H][s_x], z-faces [H][s_y][s_x])
  const int H = f.H;
  long long lay_lo = 0, lay_hi = 0, vs = 0, lo0 = 0, lstep = 0;
  if (!sync) {
    lay_lo = B->hoff[2 * d];
    lay_hi = B->hoff[2 * d + 1];
    if (d == 0) {
      vs = (long long)B->s[2] * B->s[1] * H;
      lo0 = ((long long)loc[2] * B->s[1] + loc[1]) * H;
      lstep = 1;
    } else if (d == 1) {
      vs = (long long)B->s[2] * H * B->s[0];
      lo0 = (long long)loc[2] * H * B->s[0] + loc[0];
      lstep = B->s[0];
    } else {
      vs = (long long)H * B->s[1] * B->s[0];
      lo0 = (long long)loc[1] * B->s[0] + loc[0];
      lstep = (long long)B->s[1] * B->s[0];
    }
  }
  const int od = B->o[d], nd = f.n[d];
  const double al = f.alpha;

  for (int v = 0; v < 5; ++v) {
    const T* in = f.in + v * f.field;
    // value at line position i (-5 <= i < len + 5)
    auto at = [&](int i) -> double {
      if (i >= 0 && i < len) return (double)in[g0 + i * st];
      if (sync) return (double)in[g0 + (long long)(wrap(od + i, nd) - od) * st];
      if (i < 0) return (double)f.fhalo[lay_lo + v * vs + lo0 + (long long)(i + H) * lstep];
      return (double)f.fhalo[lay_hi + v * vs + lo0 + (long long)(i - len) * lstep];
    };
    double w[11];
#pragma unroll
    for (int j = 0; j < 11; ++j) w[j] = at(j - 5);
    double dp = 0.0;
    for (int i = 0; i < len; ++i) {
      double r = f.ah[0] * w[5];
#pragma unroll
      for (int m = 1; m < 6; ++m) r = fma(f.ah[m], w[5 + m] + w[5 - m], r);
      if (i == 0) r = fma(-al, w[4], r);
      if (i == len - 1) r = fma(-al, w[6], r);
      dp = (r - al * dp) * f.inv[i];
      sD[i * kFilterLines + threadIdx.x] = dp;
#pragma unroll
      for (int j = 0; j < 10; ++j) w[j] = w[j + 1];
      if (i + 1 < len) w[10] = at(i + 6);
    }
    T* out = f.out + v * f.field;
    double x = dp;
    out[g0 + (long long)(len - 1) * st] = (T)x;
    for (int i = len - 2; i >= 0; --i) {
      x = sD[i * kFilterLines + threadIdx.x] - f.cp[i] * x;
      out[g0 + i * st] = (T)x;
    }
  }
}

template <typename T>
hipError_t launch_filter_pass(const FilterArgs<T>& f, int nblocks, int max_lines, int max_len, hipStream_t s) {
  if (max_len < 1 || max_len > kFilterMaxLen || max_lines < 1) return hipErrorInvalidValue;
  dim3 grid((max_lines + kFilterLines - 1) / kFilterLines, nblocks), block(kFilterLines);
  const size_t lds = (size_t)max_len * kFilterLines * sizeof(double);
  filter_pass_kernel<T><<<grid, block, lds, s>>>(f);
  return hipGetLastError();
}
template hipError_t launch_filter_pass<float>(const FilterArgs<float>&, int, int, int, hipStream_t);
template hipError_t launch_filter_pass<double>(const FilterArgs<double>&, int, int, int, hipStream_t);

}  // namespace atns
