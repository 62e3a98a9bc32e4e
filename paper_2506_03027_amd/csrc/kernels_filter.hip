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
// With delayed halos no pass reads another block's values, so one workgroup
// can run all three passes of a block from an LDS copy (filter_fused_kernel).
#include <type_traits>

#include "kernels_common.hpp"
#include "launch.hpp"

namespace atns {

constexpr int kFilterLines = 64;   // lines (threads) per workgroup

// The line solve of one pass, the arithmetic of filter_pass_kernel in the
// same order: ph holds line positions -5 .. LEN+4 (the halo values at both
// ends); put(i, value) receives the filtered values from the last point to
// the first.
template <typename T, int LEN, typename Put>
__device__ __forceinline__ void filter_line(const T* ph, const FilterArgs<T>& f, Put&& put) {
  const double al = f.alpha;
  double dq[LEN];
  double dp = 0.0;
#pragma unroll
  for (int i = 0; i < LEN; ++i) {
    double r = f.ah[0] * (double)ph[i + 5];
#pragma unroll
    for (int m = 1; m < 6; ++m) r = fma(f.ah[m], (double)ph[i + 5 + m] + (double)ph[i + 5 - m], r);
    if (i == 0) r = fma(-al, (double)ph[4], r);
    if (i == LEN - 1) r = fma(-al, (double)ph[LEN + 5], r);
    dp = (r - al * dp) * f.inv[i];
    dq[i] = dp;
  }
  double x = 0.0;
#pragma unroll
  for (int i = LEN - 1; i >= 0; --i) {
    x = i == LEN - 1 ? dq[i] : dq[i] - f.cp[i] * x;
    put(i, (T)x);
  }
}

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

// The same pass when every block has LEN points along the pass axis: the
// line (with its ten halo values) and the forward-eliminated values live in
// registers, all of the line's loads are issued before any arithmetic, and
// the arithmetic is that of filter_pass_kernel, in the same order.  Along x,
// where a line is a row of contiguous values, the workgroup's 64 rows pass
// through LDS so that loads and stores run along rows.
template <typename T, int LEN, int DIR>
__global__ void __launch_bounds__(kFilterLines) filter_pass_fixed_kernel(const FilterArgs<T> f) {
  constexpr int RS = LEN + 1;                      // padded LDS row
  constexpr int TL = DIR == 0 ? kFilterLines * RS : 1;
  __shared__ T tile[TL];
  __shared__ int rowoff[kFilterLines];             // row starts relative to the first row
  const BlockDev* __restrict__ B = f.blocks + blockIdx.y;
  constexpr int d = DIR;
  const int pa = d == 0 ? 1 : 0, qa = d == 2 ? 1 : 2;
  const int lines = B->s[pa] * B->s[qa];
  const int l0 = blockIdx.x * kFilterLines;
  if (l0 >= lines) return;                         // whole workgroup
  // lanes past the block's last line work on that line and store nothing
  const bool act = l0 + (int)threadIdx.x < lines;
  const int li = act ? l0 + (int)threadIdx.x : lines - 1;
  int loc[3];
  loc[d] = 0;
  loc[pa] = li % B->s[pa];
  loc[qa] = li / B->s[pa];

  int halo = f.halo;
  if (f.nstep) halo = (*f.nstep - 1 >= f.C) ? f.async_halo : kHaloSync;
  const bool sync = halo == kHaloSync || f.fhalo == nullptr;

  const long long nxy = (long long)f.n[0] * f.n[1];
  const long long st = d == 0 ? 1 : (d == 1 ? f.n[0] : nxy);
  const long long g0 = (long long)(B->o[2] + loc[2]) * nxy + (long long)(B->o[1] + loc[1]) * f.n[0] +
                       (B->o[0] + loc[0]);
  const int rows = min(kFilterLines, lines - l0);  // rows of this workgroup (x pass)
  // x pass over single-precision rows that start on 16-byte boundaries: each
  // lane reads and writes its own row four values at a time; other x passes
  // stage the rows through LDS
  const bool vec4 = d == 0 && sizeof(T) == 4 && LEN % 4 == 0 && (B->o[0] & 3) == 0 && (f.n[0] & 3) == 0;
  const bool staged = d == 0 && !vec4;
  // x pass: the first row's start (the same for every lane) and each row's
  // offset from it, so the staging addresses are one base plus 32 bits
  const long long gfirst = (long long)(B->o[2] + l0 / B->s[1]) * nxy + (long long)(B->o[1] + l0 % B->s[1]) * f.n[0] +
                           B->o[0];
  if (staged) {
    rowoff[threadIdx.x] = (int)(g0 - gfirst);
    __syncthreads();
  }
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
    T ph[LEN + 10];   // line positions -5 .. LEN+4
    if constexpr (sizeof(T) == 4) {
      if (vec4) {
        using V4 = float __attribute__((ext_vector_type(4)));
        const V4* row = reinterpret_cast<const V4*>(in + g0);
#pragma unroll
        for (int q = 0; q < LEN / 4; ++q) {
          const V4 x4 = row[q];
          ph[5 + 4 * q] = x4.x;
          ph[6 + 4 * q] = x4.y;
          ph[7 + 4 * q] = x4.z;
          ph[8 + 4 * q] = x4.w;
        }
      }
    }
    if (staged) {
      // rows of this workgroup into LDS, each load instruction along rows
      __syncthreads();
      const T* in0 = in + gfirst;
      const int c = threadIdx.x % LEN;
#pragma unroll 8
      for (int k = 0; k < LEN; ++k) {
        const int r = k * (kFilterLines / LEN) + threadIdx.x / LEN;
        if (r < rows) tile[r * RS + c] = in0[rowoff[r] + c];
      }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < LEN + 10; ++j) {
      const int i = j - 5;
      if (i >= 0 && i < LEN) {
        if (!vec4) ph[j] = staged ? tile[threadIdx.x * RS + i] : in[g0 + i * st];
      } else if (sync)
        ph[j] = in[g0 + (long long)(wrap(od + i, nd) - od) * st];
      else if (i < 0)
        ph[j] = f.fhalo[lay_lo + v * vs + lo0 + (long long)(i + H) * lstep];
      else
        ph[j] = f.fhalo[lay_hi + v * vs + lo0 + (long long)(i - LEN) * lstep];
    }
    // the arithmetic of filter_line, written out so that the stores can sit
    // in the back substitution's own loop
    double dq[LEN];
    double dp = 0.0;
#pragma unroll
    for (int i = 0; i < LEN; ++i) {
      double r = f.ah[0] * (double)ph[i + 5];
#pragma unroll
      for (int m = 1; m < 6; ++m) r = fma(f.ah[m], (double)ph[i + 5 + m] + (double)ph[i + 5 - m], r);
      if (i == 0) r = fma(-al, (double)ph[4], r);
      if (i == LEN - 1) r = fma(-al, (double)ph[LEN + 5], r);
      dp = (r - al * dp) * f.inv[i];
      dq[i] = dp;
    }
    T* out = f.out + v * f.field;
    if (staged) __syncthreads();   // every lane has read its row from the tile
    double x = 0.0;
    T res[vec4 ? LEN : 1];
#pragma unroll
    for (int i = LEN - 1; i >= 0; --i) {
      x = i == LEN - 1 ? dq[i] : dq[i] - f.cp[i] * x;
      const T val = (T)x;
      if (vec4)
        res[i] = val;
      else if (staged)
        tile[threadIdx.x * RS + i] = val;
      else if (act)
        out[g0 + i * st] = val;
    }
    if constexpr (sizeof(T) == 4) {
      if (vec4 && act) {
        using V4 = float __attribute__((ext_vector_type(4)));
        V4* row = reinterpret_cast<V4*>(out + g0);
#pragma unroll
        for (int q = 0; q < LEN / 4; ++q) row[q] = V4{res[4 * q], res[4 * q + 1], res[4 * q + 2], res[4 * q + 3]};
      }
    }
    if (staged) {
      __syncthreads();
      T* out0 = out + gfirst;
      const int c = threadIdx.x % LEN;
#pragma unroll 8
      for (int k = 0; k < LEN; ++k) {
        const int r = k * (kFilterLines / LEN) + threadIdx.x / LEN;
        if (r < rows) out0[rowoff[r] + c] = tile[r * RS + c];
      }
    }
  }
}

// All three passes of one variable of one block, a cube of side LEN, with
// delayed halos: workgroup (v, b), one thread per line of each pass.  The
// block's values of variable v are read once into LDS (rows padded to
// LEN + 1, so that the lines of every axis fall in distinct banks), the x, y
// and z passes each solve the block's LEN^2 lines of their axis from LDS,
// with the halo values from the filter-halo slot (the next pass's are
// loaded while a pass computes), the z pass stores the result, and after a
// barrier the workgroup writes the block's boundary layers of variable v to
// the ring, layer by layer in storage order.
// Each line's arithmetic is filter_line, as in the per-axis passes, so the
// results are the same bits.
template <typename T, int LEN>
__global__ void __launch_bounds__(LEN * LEN) filter_fused_kernel(const FilterArgs<T> f) {
  constexpr int PY = LEN + 1, PZ = LEN * PY;
  __shared__ T sU[LEN * PZ];
  int halo = f.halo;
  if (f.nstep) halo = (*f.nstep - 1 >= f.C) ? f.async_halo : kHaloSync;
  if (halo == kHaloSync || f.fhalo == nullptr) return;   // the per-axis passes take this step
  const int v = blockIdx.x;
  const BlockDev* __restrict__ B = f.blocks + blockIdx.y;
  const int tid = threadIdx.x;
  const int a = tid % LEN, b = tid / LEN;   // the thread's line: (y, z), (x, z), (x, y)
  const int H = f.H;
  const long long nxy = (long long)f.n[0] * f.n[1];
  const long long n0 = f.n[0];
  const long long gb = v * f.field + (long long)B->o[2] * nxy + (long long)B->o[1] * n0 + B->o[0];
  // the halo values of the thread's line of pass d: positions -5..-1 of the
  // low face, LEN..LEN+4 of the high one.  Layers: x-faces [s_z][s_y][H],
  // y-faces [s_z][H][s_x], z-faces [H][s_y][s_x], variables outermost.
  auto halo_load = [&](auto dc, T hv[10]) {
    constexpr int d = decltype(dc)::value;
    constexpr int lstep = d == 0 ? 1 : (d == 1 ? LEN : LEN * LEN);
    const long long vs = (long long)LEN * LEN * H;
    const T* hlo = f.fhalo + B->hoff[2 * d] + v * vs;
    const T* hhi = f.fhalo + B->hoff[2 * d + 1] + v * vs;
    const int lo0 = d == 0 ? (b * LEN + a) * H : (d == 1 ? b * H * LEN + a : b * LEN + a);
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      hv[j] = hlo[lo0 + (j - 5 + H) * lstep];
      hv[5 + j] = hhi[lo0 + j * lstep];
    }
  };
  T hv[10];
  halo_load(std::integral_constant<int, 0>{}, hv);
  {
    // the block's values of variable v, each thread a row per load
    const T* in = f.in + gb;
    if constexpr (sizeof(T) == 4 && LEN % 4 == 0) {
      using V4 = float __attribute__((ext_vector_type(4)));
      constexpr int Q = LEN / 4;   // float4 per row
#pragma unroll
      for (int k = tid; k < LEN * LEN * Q; k += LEN * LEN) {
        const int q = k % Q, y = (k / Q) % LEN, z = k / (Q * LEN);
        const V4 x4 = *reinterpret_cast<const V4*>(in + z * nxy + y * n0 + 4 * q);
        T* d = sU + z * PZ + y * PY + 4 * q;
        d[0] = x4.x;
        d[1] = x4.y;
        d[2] = x4.z;
        d[3] = x4.w;
      }
    } else {
#pragma unroll
      for (int k = tid; k < LEN * LEN * LEN; k += LEN * LEN) {
        const int x = k % LEN, y = (k / LEN) % LEN, z = k / (LEN * LEN);
        sU[z * PZ + y * PY + x] = in[z * nxy + y * n0 + x];
      }
    }
  }
  __syncthreads();
  T* out = f.out + gb;
  auto pass = [&](auto dc) {
    constexpr int d = decltype(dc)::value;
    constexpr int sstep = d == 0 ? 1 : (d == 1 ? PY : PZ);   // LDS stride along the line
    const int s0 = d == 0 ? b * PZ + a * PY : (d == 1 ? b * PZ + a : b * PY + a);
    T ph[LEN + 10];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      ph[j] = hv[j];
      ph[LEN + 5 + j] = hv[5 + j];
    }
#pragma unroll
    for (int i = 0; i < LEN; ++i) ph[i + 5] = sU[s0 + i * sstep];
    if constexpr (d < 2) halo_load(std::integral_constant<int, d + 1>{}, hv);
    filter_line<T, LEN>(ph, f, [&](int i, T val) {
      sU[s0 + i * sstep] = val;
      if constexpr (d == 2) out[i * nxy + b * n0 + a] = val;
    });
    __syncthreads();
  };
  pass(std::integral_constant<int, 0>{});
  pass(std::integral_constant<int, 1>{});
  pass(std::integral_constant<int, 2>{});
  // the filtered boundary layers of variable v into the ring slot of the new
  // level, walking each layer in its storage order ([5][ez][ey][ex], faces H
  // deep, edges 2) so that every store is along contiguous memory
  T* slot = f.ring + (long long)(f.nstep ? (int)(*f.nstep % f.D) : f.slot) * f.slot_stride;
  for (int sl = 0; sl < kNumSlots; ++sl) {
    if (B->lay[sl] < 0) continue;
    int dir[3];
    slot_dir(sl, dir);
    const int dep = sl < 6 ? H : 2;
    int e[3], o[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      e[k] = dir[k] ? dep : LEN;
      o[k] = dir[k] > 0 ? LEN - dep : 0;
    }
    const int cnt = e[0] * e[1] * e[2];
    T* dst = slot + B->lay[sl] + (long long)v * cnt;
    // i / e as the high half of i * ceil(2^32 / e): exact for e <= 32 and
    // i < 2^27 (here i < LEN^3)
    const unsigned m0 = 0xFFFFFFFFu / (unsigned)e[0] + 1u, m1 = 0xFFFFFFFFu / (unsigned)e[1] + 1u;
    for (int idx = tid; idx < cnt; idx += LEN * LEN) {
      const unsigned r = __umulhi((unsigned)idx, m0);
      const unsigned iz = __umulhi(r, m1);
      const int ix = idx - (int)r * e[0], iy = (int)r - (int)iz * e[1];
      dst[idx] = sU[(o[2] + (int)iz) * PZ + (o[1] + iy) * PY + o[0] + ix];
    }
  }
}

template <typename T>
hipError_t launch_filter_fused(const FilterArgs<T>& f, int nblocks, int side, hipStream_t s) {
  if (!filter_fused_fits(side, (int)sizeof(T))) return hipErrorInvalidValue;
  dim3 grid(5, nblocks);
  if (side == 8) {
    filter_fused_kernel<T, 8><<<grid, 8 * 8, 0, s>>>(f);
  } else if (side == 16) {
    filter_fused_kernel<T, 16><<<grid, 16 * 16, 0, s>>>(f);
  } else {
    if constexpr (sizeof(T) == 4) filter_fused_kernel<T, 32><<<grid, 32 * 32, 0, s>>>(f);
  }
  return hipGetLastError();
}
template hipError_t launch_filter_fused<float>(const FilterArgs<float>&, int, int, hipStream_t);
template hipError_t launch_filter_fused<double>(const FilterArgs<double>&, int, int, hipStream_t);

template <typename T>
hipError_t launch_filter_pass(const FilterArgs<T>& f, int nblocks, int max_lines, int min_len, int max_len,
                              hipStream_t s) {
  if (max_len < 1 || max_len > kFilterMaxLen || max_lines < 1) return hipErrorInvalidValue;
  dim3 grid((max_lines + kFilterLines - 1) / kFilterLines, nblocks), block(kFilterLines);
  if (filter_pass_fixed(min_len, max_len)) {
#define ATNS_FILTER_FIXED(LEN)                                                             \
  do {                                                                                     \
    if (f.dir == 0)                                                                        \
      filter_pass_fixed_kernel<T, LEN, 0><<<grid, block, 0, s>>>(f);                       \
    else if (f.dir == 1)                                                                   \
      filter_pass_fixed_kernel<T, LEN, 1><<<grid, block, 0, s>>>(f);                       \
    else                                                                                   \
      filter_pass_fixed_kernel<T, LEN, 2><<<grid, block, 0, s>>>(f);                       \
  } while (0)
    if (max_len == 8)
      ATNS_FILTER_FIXED(8);
    else if (max_len == 16)
      ATNS_FILTER_FIXED(16);
    else
      ATNS_FILTER_FIXED(32);
#undef ATNS_FILTER_FIXED
    return hipGetLastError();
  }
  const size_t lds = (size_t)max_len * kFilterLines * sizeof(double);
  filter_pass_kernel<T><<<grid, block, lds, s>>>(f);
  return hipGetLastError();
}
template hipError_t launch_filter_pass<float>(const FilterArgs<float>&, int, int, int, int, hipStream_t);
template hipError_t launch_filter_pass<double>(const FilterArgs<double>&, int, int, int, int, hipStream_t);

}  // namespace atns
