// Learned halo correction: a 64-64-64-16 MLP on BF16 MFMA (FP32 accumulate).
//
// For a face halo point the network reads 60 features built from the delayed
// levels the AT extrapolation uses (4 newest levels x 5 variables x the point
// and its two neighbours along the face normal, relative to the newest level
// and scaled by s_v), plus k/(L-1), and predicts the extrapolation error in
// units of r_v.  The correction delta_v = r_v out_v is added to all stage
// halo values of the point unless |out|_2 > tau (then the AT value stays).
//
// Parameters (FP32 master, BF16 working copy), row-major [out][in]:
//   W1[64][64] b1[64] W2[64][64] b2[64] W3[16][64] b3[16]
//
// Every product runs on v_mfma_f32_16x16x32_bf16.  Lane l of a wave supplies
// A[m = l%16][k = 8(l/16) + j] and B[k = 8(l/16) + j][n = l%16], j = 0..7,
// and receives D[m = 4(l/16) + i][n = l%16], i = 0..3.  A wave works on 16
// samples at a time; operands are staged in LDS as BF16.
#include <hip/hip_runtime.h>

#include "kernels_common.hpp"
#include "mlp.hpp"

#include <algorithm>

namespace atns {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// Order this wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// FP32 -> BF16, round to nearest even (same rounding as the host reference).
__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

// C[16x16] += A[16 x K] B[K x 16] for one wave; operands in LDS as BF16 bit
// patterns with element (m,k) of A at A[m*sam + k*sak] and (k,n) of B at
// B[k*sbk + n*sbn].  K is a multiple of 32.
template <int K>
__device__ __forceinline__ f32x4 wave_gemm(const unsigned short* A, int sam, int sak, const unsigned short* B,
                                           int sbk, int sbn, f32x4 acc) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int kb = 0; kb < K / 32; ++kb) {
    bf16x8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = kb * 32 + 8 * g + j;
      unsigned short av = A[r * sam + k * sak];
      unsigned short bv = B[k * sbk + r * sbn];
      a[j] = __builtin_bit_cast(__bf16, av);
      b[j] = __builtin_bit_cast(__bf16, bv);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// The same product when both operands are contiguous along k (A row-major
// [16][lda], B given as rows of W, [16][ldb]): each lane's 8 consecutive k
// values of A and B are one 16-byte LDS read.  Rows must be 16-byte aligned.
template <int K>
__device__ __forceinline__ f32x4 wave_gemm_k(const unsigned short* A, int lda, const unsigned short* Bt, int ldb,
                                             f32x4 acc) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int kb = 0; kb < K / 32; ++kb) {
    const bf16x8 av = *reinterpret_cast<const bf16x8*>(A + r * lda + kb * 32 + 8 * g);
    const bf16x8 bv = *reinterpret_cast<const bf16x8*>(Bt + r * ldb + kb * 32 + 8 * g);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
  }
  return acc;
}

// Layer y = x W^T + b for 16 samples of one wave: x [16][nin] BF16 in LDS
// (row stride ldx), W [nout][nin] BF16 in LDS, b FP32.  Writes pre-activation
// z (FP32, [16][nout], row stride ldz) to LDS.
template <int NIN, int NOUT>
__device__ __forceinline__ void wave_layer(const unsigned short* x, int ldx, const unsigned short* W,
                                           const float* b, float* z, int ldz) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int nt = 0; nt < NOUT / 16; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    // B[k][n] = W[nt*16 + n][k]: rows of W, contiguous along k
    acc = wave_gemm_k<NIN>(x, ldx, W + nt * 16 * NIN, NIN, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) z[(4 * g + i) * ldz + nt * 16 + r] = acc[i] + b[nt * 16 + r];
  }
}

// Inference form of a hidden layer: h = BF16(ReLU(x W^T + b)) written
// straight from the accumulators (the FP32 pre-activations are kept only by
// the training path, which needs them).  Same values as wave_layer followed
// by the ReLU and the BF16 rounding.
template <int NIN, int NOUT>
__device__ __forceinline__ void wave_layer_relu(const unsigned short* x, int ldx, const unsigned short* W,
                                                const float* b, unsigned short* h, int ldh) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
#pragma unroll
  for (int nt = 0; nt < NOUT / 16; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = wave_gemm_k<NIN>(x, ldx, W + nt * 16 * NIN, NIN, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) h[(4 * g + i) * ldh + nt * 16 + r] = f2bf(fmaxf(acc[i] + b[nt * 16 + r], 0.f));
  }
}

// Shared-memory image of the network for one workgroup.
struct alignas(16) MlpLds {
  unsigned short W1[kMlpH * kMlpIn];
  unsigned short W2[kMlpH * kMlpH];
  unsigned short W3[kMlpOut * kMlpH];
  float b1[kMlpH], b2[kMlpH], b3[kMlpOut];
};

__device__ __forceinline__ void load_net(const MlpNet& net, MlpLds& L) {
  for (int i = threadIdx.x; i < kMlpH * kMlpIn; i += blockDim.x) L.W1[i] = net.w1[i];
  for (int i = threadIdx.x; i < kMlpH * kMlpH; i += blockDim.x) L.W2[i] = net.w2[i];
  for (int i = threadIdx.x; i < kMlpOut * kMlpH; i += blockDim.x) L.W3[i] = net.w3[i];
  for (int i = threadIdx.x; i < kMlpH; i += blockDim.x) {
    L.b1[i] = net.params[kOffB1 + i];
    L.b2[i] = net.params[kOffB2 + i];
  }
  for (int i = threadIdx.x; i < kMlpOut; i += blockDim.x) L.b3[i] = net.params[kOffB3 + i];
}

// Activations of 16 samples of one wave (row-major [16][width] slices).
struct Fwd {
  unsigned short* x;   // BF16 input [16][64]
  float* z1;           // pre-activations, FP32 [16][64]
  unsigned short* h1;  // BF16 ReLU(z1)
  float* z2;
  unsigned short* h2;
  float* o;            // outputs, FP32 [16][16]
};

// Per-wave scratch of the inference kernels.
struct alignas(16) WaveScratch {
  unsigned short x[16 * kMlpIn];
  float z1[16 * kMlpH];
  unsigned short h1[16 * kMlpH];
  float z2[16 * kMlpH];
  unsigned short h2[16 * kMlpH];
  float o[16 * kMlpOut];
  __device__ Fwd fwd() { return Fwd{x, z1, h1, z2, h2, o}; }
};

// Per-wave scratch of the halo inference: the input, reused for the second
// hidden layer once the first has read it, the first hidden layer and the
// outputs (5 KB per wave).
struct alignas(16) InferScratch {
  unsigned short x[16 * kMlpIn];   // input, then h2
  unsigned short h1[16 * kMlpH];
  float o[16 * kMlpOut];
};

__device__ __forceinline__ void wave_forward_infer(const MlpLds& L, InferScratch& S) {
  wave_layer_relu<kMlpIn, kMlpH>(S.x, kMlpIn, L.W1, L.b1, S.h1, kMlpH);
  wave_sync();
  wave_layer_relu<kMlpH, kMlpH>(S.h1, kMlpH, L.W2, L.b2, S.x, kMlpH);
  wave_sync();
  wave_layer<kMlpH, kMlpOut>(S.x, kMlpH, L.W3, L.b3, S.o, kMlpOut);
  wave_sync();
}

// Forward pass of the wave's 16 samples (x already staged).
__device__ __forceinline__ void wave_forward(const MlpLds& L, Fwd F) {
  const int lane = threadIdx.x & 63;
  wave_layer<kMlpIn, kMlpH>(F.x, kMlpIn, L.W1, L.b1, F.z1, kMlpH);
  wave_sync();
  for (int i = lane; i < 16 * kMlpH; i += 64) F.h1[i] = f2bf(fmaxf(F.z1[i], 0.f));
  wave_sync();
  wave_layer<kMlpH, kMlpH>(F.h1, kMlpH, L.W2, L.b2, F.z2, kMlpH);
  wave_sync();
  for (int i = lane; i < 16 * kMlpH; i += 64) F.h2[i] = f2bf(fmaxf(F.z2[i], 0.f));
  wave_sync();
  wave_layer<kMlpH, kMlpOut>(F.h2, kMlpH, L.W3, L.b3, F.o, kMlpOut);
  wave_sync();
}

// ----------------------------------------------------------------- features
// Feature f (< 60) of the face-halo point `pt` of region rg: level l, var v,
// normal offset j (f = (l*5 + v)*3 + j), relative to level 0 at the point.
template <typename T>
__device__ __forceinline__ void face_features(const MlpFeatArgs<T>& a, const HaloRegion& rg, const FaceInfo& fi,
                                              int pt, int k, float* out /*64*/) {
  // point coordinates in the region (extents ex, ey, ez) and its normal index
  int c[3];
  c[0] = pt % fi.ext[0];
  c[1] = (pt / fi.ext[0]) % fi.ext[1];
  c[2] = pt / (fi.ext[0] * fi.ext[1]);
  const int ax = fi.axis;
  const int depth = fi.ext[ax];
  int idx[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    int cc[3] = {c[0], c[1], c[2]};
    cc[ax] = min(max(c[ax] + j - 1, 0), depth - 1);
    idx[j] = (cc[2] * fi.ext[1] + cc[1]) * fi.ext[0] + cc[0];
  }
  float centre[5];
  const int snow = a.nstep ? (int)(*a.nstep % a.D) : a.slot_now;
  int sl0 = snow - k;
  sl0 += (sl0 < 0) ? a.D : 0;
  const T* base0 = a.ring + (long long)sl0 * a.slot_stride + rg.src;
#pragma unroll
  for (int v = 0; v < 5; ++v) centre[v] = (float)base0[(long long)v * rg.npts + idx[1]];
  int f = 0;
  for (int l = 0; l < 4; ++l) {
    int sl = snow - k - l;
    sl += (sl < 0) ? a.D : 0;
    const T* base = a.ring + (long long)sl * a.slot_stride + rg.src;
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int j = 0; j < 3; ++j) out[f++] = ((float)base[(long long)v * rg.npts + idx[j]] - centre[v]) * a.inv_s[v];
  }
  out[60] = (a.L > 1) ? (float)k / (float)(a.L - 1) : 0.f;
  out[61] = out[62] = out[63] = 0.f;
}

// ------------------------------------------------------------ halo inference
// Features of level l (15 values: 5 variables x normal offsets j-1, j, j+1,
// relative to level 0 at the point) of the face-halo point `pt`, written as
// BF16 at x[l*15 ..]; the same values as face_features().
template <typename T>
__device__ __forceinline__ void level_features(const MlpFeatArgs<T>& a, const HaloRegion& rg, const FaceInfo& fi,
                                               int pt, int k, int l, unsigned short* x) {
  // no arrays indexed by the (run-time) normal axis: they would live in scratch
  const int e0 = fi.ext[0], e1 = fi.ext[1], e2 = fi.ext[2];
  const int cx = pt % e0, cy = (pt / e0) % e1, cz = pt / (e0 * e1);
  const int ax = fi.axis;
  int idx[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int nx = ax == 0 ? min(max(cx + j - 1, 0), e0 - 1) : cx;
    const int ny = ax == 1 ? min(max(cy + j - 1, 0), e1 - 1) : cy;
    const int nz = ax == 2 ? min(max(cz + j - 1, 0), e2 - 1) : cz;
    idx[j] = (nz * e1 + ny) * e0 + nx;
  }
  const int snow = a.nstep ? (int)(*a.nstep % a.D) : a.slot_now;
  int sl0 = snow - k;
  sl0 += (sl0 < 0) ? a.D : 0;
  int sl = snow - k - l;
  sl += (sl < 0) ? a.D : 0;
  const T* base0 = a.ring + (long long)sl0 * a.slot_stride + rg.src;
  const T* base = a.ring + (long long)sl * a.slot_stride + rg.src;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const float centre = (float)base0[(long long)v * rg.npts + idx[1]];
#pragma unroll
    for (int j = 0; j < 3; ++j)
      x[l * 15 + v * 3 + j] = f2bf(((float)base[(long long)v * rg.npts + idx[j]] - centre) * a.inv_s[v]);
  }
}

// Persistent workgroups (the network is staged in LDS once); each wave takes
// chunks of 16 face-halo points: four lanes per point gather its features
// (one delayed level each, the point's own delay), the wave runs the forward
// pass on the matrix cores, and the lanes of accepted points add delta to
// every stage halo value of the point.  Applied / fallback counts are summed
// per wave and added once at the end.
template <typename T>
__global__ void __launch_bounds__(256) mlp_halo_kernel(MlpFeatArgs<T> a, MlpNet net, const HaloRegion* regions,
                                                        const FaceInfo* faces, const HaloWork* chunks,
                                                        long long nchunks, const int8_t* delays, T* hbuf,
                                                        long long halo_stride, int stages,
                                                        unsigned long long* counters) {
  __shared__ MlpLds L;
  __shared__ InferScratch S[4];
  load_net(net, L);
  __syncthreads();
  // the ring slot of level n, resolved once (not per point)
  MlpFeatArgs<T> af = a;
  if (af.nstep) {
    af.slot_now = (int)(*af.nstep % af.D);
    af.nstep = nullptr;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  InferScratch& W = S[wave];
  unsigned long long n_ok = 0, n_fb = 0;
  constexpr int kItems = (kMlpChunk * 5 + 63) / 64;   // (point, variable) items per lane
  for (long long c = (long long)blockIdx.x * 4 + wave; c < nchunks; c += (long long)gridDim.x * 4) {
    const HaloWork ck = chunks[c];
    const HaloRegion rg = regions[ck.region];
    const FaceInfo fi = faces[ck.region];
    const int k = (int)delays[rg.kidx];
    {
      const int p = lane & 15, l = lane >> 4;
      const int pt = ck.start + p;
      unsigned short* x = W.x + p * kMlpIn;
      if (pt < rg.npts) {
        level_features(af, rg, fi, pt, k, l, x);
      } else {
#pragma unroll
        for (int f = 0; f < 15; ++f) x[l * 15 + f] = 0;
      }
      if (l == 0) {
        x[60] = f2bf(pt < rg.npts && a.L > 1 ? (float)k / (float)(a.L - 1) : 0.f);
        x[61] = x[62] = x[63] = 0;
      }
    }
    // the stage halo values this lane may correct, loaded now so that their
    // latency hides behind the forward pass
    T hv[kItems][kMlpMaxStages];
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int j = lane + 64 * q;
      const int p = j % kMlpChunk, v = j / kMlpChunk;
      if (j < kMlpChunk * 5 && ck.start + p < rg.npts) {
        const long long o = rg.dst + (long long)v * rg.npts + ck.start + p;
#pragma unroll
        for (int e = 0; e < kMlpMaxStages; ++e)
          if (e < stages) hv[q][e] = hbuf[e * halo_stride + o];
      }
    }
    wave_sync();
    wave_forward_infer(L, W);
    const int pt = ck.start + lane;
    const bool valid = lane < kMlpChunk && pt < rg.npts;
    bool ok = false;
    if (valid) {
      float n2 = 0.f;
#pragma unroll
      for (int v = 0; v < 5; ++v) n2 += W.o[lane * kMlpOut + v] * W.o[lane * kMlpOut + v];
      ok = n2 <= a.tau2;
    }
    const unsigned long long okmask = __ballot(valid && ok);
    n_ok += __popcll(okmask);
    n_fb += __popcll(__ballot(valid && !ok));
    // the 16 x 5 (point, variable) corrections spread over all lanes
#pragma unroll
    for (int q = 0; q < kItems; ++q) {
      const int j = lane + 64 * q;
      const int p = j % kMlpChunk, v = j / kMlpChunk;
      if (j < kMlpChunk * 5 && ((okmask >> p) & 1ull)) {
        const double d = (double)a.r[v] * (double)W.o[p * kMlpOut + v];
        const long long o = rg.dst + (long long)v * rg.npts + ck.start + p;
#pragma unroll
        for (int e = 0; e < kMlpMaxStages; ++e)
          if (e < stages) hbuf[e * halo_stride + o] = (T)((double)hv[q][e] + d);
      }
    }
    wave_sync();   // the next chunk overwrites this wave's scratch
  }
  if (lane == 0) {
    if (n_ok) atomicAdd(&counters[0], n_ok);
    if (n_fb) atomicAdd(&counters[1], n_fb);
  }
}

// ------------------------------------------------------------------ sampler
// Sample i: a face-halo point and a delay drawn by SplitMix64 from (seed, i);
// features as above and the target (U^n - Uhat_AT^(0)) / r_v, U^n from the
// ring's newest level.  X [n][64], Y [n][8] (first 5 used), FP32.
__device__ __forceinline__ unsigned long long mix64(unsigned long long seed, unsigned long long i) {
  unsigned long long z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <typename T>
__global__ void mlp_sample_kernel(MlpFeatArgs<T> a, const HaloRegion* regions, const FaceInfo* faces,
                                  const int* face_regions, int nface, const double* W0 /*[L][C]*/,
                                  unsigned long long seed, int n, float* X, float* Y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned long long h1 = mix64(seed, 2ull * i), h2 = mix64(seed, 2ull * i + 1ull);
  const int rid = face_regions[h1 % (unsigned long long)nface];
  const HaloRegion rg = regions[rid];
  const int pt = (int)((h1 >> 32) % (unsigned long long)rg.npts);
  const int k = (int)(h2 % (unsigned long long)a.L);
  float feat[64];
  face_features(a, rg, faces[rid], pt, k, feat);
  for (int f = 0; f < 64; ++f) X[(long long)i * 64 + f] = feat[f];
  const T* now = a.ring + (long long)a.slot_now * a.slot_stride + rg.src;
  for (int v = 0; v < 5; ++v) {
    double ext = 0.0;
    for (int l = 0; l < kLevels; ++l) {
      int sl = a.slot_now - k - l;
      sl += (sl < 0) ? a.D : 0;
      ext = fma(W0[k * kLevels + l], (double)a.ring[(long long)sl * a.slot_stride + rg.src + (long long)v * rg.npts + pt],
                ext);
    }
    Y[(long long)i * 8 + v] = (float)(((double)now[(long long)v * rg.npts + pt] - ext) * (double)a.inv_r[v]);
  }
  for (int v = 5; v < 8; ++v) Y[(long long)i * 8 + v] = 0.f;
}

// -------------------------------------------------------- forward (plain X)
__global__ void __launch_bounds__(256) mlp_forward_kernel(MlpNet net, const float* X, int n, float* out) {
  __shared__ MlpLds L;
  __shared__ WaveScratch S[4];
  load_net(net, L);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  WaveScratch& W = S[wave];
  const int first = (blockIdx.x * 4 + wave) * 16;
  if (first >= n) return;
  for (int i = lane; i < 16 * kMlpIn; i += 64) {
    const int s = first + i / kMlpIn;
    W.x[i] = f2bf(s < n ? X[(long long)first * kMlpIn + i] : 0.f);
  }
  wave_sync();
  wave_forward(L, W.fwd());
  for (int i = lane; i < 16 * kMlpOut; i += 64)
    if (first + i / kMlpOut < n) out[(long long)first * kMlpOut + i] = W.o[i];
}

// ---------------------------------------------------------- loss + gradient
// Workgroup of 4 waves = 64 samples.  Forward, dO = 2 (O - Y) / (n * 5) on
// the used outputs, backward through the ReLUs, and this workgroup's partial
// parameter gradient (sum over its samples) into part[blockIdx.x][kMlpParams].
// Weight gradients are MFMA products with the samples as the K dimension.
struct alignas(16) TrainLds {
  unsigned short X[64 * kMlpIn];   // BF16 inputs
  float Z1[64 * kMlpH];            // pre-activations, then dZ1 (FP32)
  unsigned short H1[64 * kMlpH];   // BF16 activations
  float Z2[64 * kMlpH];            // pre-activations, then dZ2 (FP32)
  unsigned short H2[64 * kMlpH];
  float O[64 * kMlpOut];           // outputs, then dO (FP32)
  unsigned short dO[64 * kMlpOut]; // BF16 gradients as MFMA operands
  unsigned short dZ2[64 * kMlpH];
  unsigned short dZ1[64 * kMlpH];
  unsigned short pad[4][16 * 32];  // per-wave zero-padded dO (K = 32)
  float loss[64];
};

__global__ void __launch_bounds__(256) mlp_grad_kernel(MlpNet net, const float* X, const float* Y, int n,
                                                        float* part, float* loss_part) {
  __shared__ MlpLds L;
  __shared__ TrainLds T;
  load_net(net, L);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  const int s0 = blockIdx.x * 64;
  for (int i = threadIdx.x; i < 64 * kMlpIn; i += blockDim.x) {
    const int s = s0 + i / kMlpIn;
    T.X[i] = f2bf(s < n ? X[(long long)s0 * kMlpIn + i] : 0.f);
  }
  __syncthreads();
  // forward, 16 samples per wave, straight into the workgroup arrays
  const int w16 = wave * 16;
  wave_forward(L, Fwd{T.X + w16 * kMlpIn, T.Z1 + w16 * kMlpH, T.H1 + w16 * kMlpH, T.Z2 + w16 * kMlpH,
                      T.H2 + w16 * kMlpH, T.O + w16 * kMlpOut});
  const float scale = 2.f / (float)(n * kMlpUse);
  if (lane < 16) {
    const int sl = w16 + lane, s = s0 + sl;
    float l2 = 0.f;
    for (int o = 0; o < kMlpOut; ++o) {
      float d = 0.f;
      if (s < n && o < kMlpUse) {
        d = T.O[sl * kMlpOut + o] - Y[(long long)s * 8 + o];
        l2 += d * d;
      }
      const float gd = d * scale;
      T.O[sl * kMlpOut + o] = gd;          // now dO (FP32)
      T.dO[sl * kMlpOut + o] = f2bf(gd);
    }
    T.loss[sl] = l2;
  }
  wave_sync();
  // dZ2 = (dO W3) * relu'(z2) for the wave's samples; K = 16 padded to 32
  {
    unsigned short* dOpad = T.pad[wave];
    for (int i = lane; i < 16 * 32; i += 64) {
      const int rr = i / 32, cc = i % 32;
      dOpad[i] = cc < kMlpOut ? T.dO[(w16 + rr) * kMlpOut + cc] : (unsigned short)0;
    }
    wave_sync();
    for (int nt = 0; nt < kMlpH / 16; ++nt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      bf16x8 av, bv;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = 8 * g + j;
        av[j] = __builtin_bit_cast(__bf16, dOpad[r * 32 + k]);
        const unsigned short wv = k < kMlpOut ? L.W3[k * kMlpH + nt * 16 + r] : (unsigned short)0;
        bv[j] = __builtin_bit_cast(__bf16, wv);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int sl = w16 + 4 * g + i, u = nt * 16 + r;
        const float d = T.Z2[sl * kMlpH + u] > 0.f ? acc[i] : 0.f;
        T.Z2[sl * kMlpH + u] = d;           // now dZ2 (FP32)
        T.dZ2[sl * kMlpH + u] = f2bf(d);
      }
    }
  }
  wave_sync();
  // dZ1 = (dZ2 W2) * relu'(z1): B[k][n] = W2[k][n]
  for (int nt = 0; nt < kMlpH / 16; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = wave_gemm<kMlpH>(T.dZ2 + w16 * kMlpH, kMlpH, 1, L.W2 + nt * 16, kMlpH, 1, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int sl = w16 + 4 * g + i, u = nt * 16 + r;
      const float d = T.Z1[sl * kMlpH + u] > 0.f ? acc[i] : 0.f;
      T.Z1[sl * kMlpH + u] = d;             // now dZ1 (FP32)
      T.dZ1[sl * kMlpH + u] = f2bf(d);
    }
  }
  __syncthreads();
  // weight gradients (K = the workgroup's 64 samples):
  //   dW1[u][f] = sum_s dZ1[s][u] X[s][f]   (64 x 64, 16 tiles)
  //   dW2[u][v] = sum_s dZ2[s][u] H1[s][v]  (64 x 64, 16 tiles)
  //   dW3[o][v] = sum_s dO[s][o]  H2[s][v]  (16 x 64, 4 tiles)
  float* P = part + (long long)blockIdx.x * kMlpParams;
  for (int t = wave; t < 36; t += 4) {
    const unsigned short *A, *B;
    int sak, sbk, off, ldo, mt, nt;
    if (t < 16) {
      mt = t / 4; nt = t % 4;
      A = T.dZ1 + mt * 16; sak = kMlpH;     // A[m=u][k=s] = dZ1[s][u]
      B = T.X + nt * 16; sbk = kMlpIn;      // B[k=s][n=f] = X[s][f]
      off = kOffW1; ldo = kMlpIn;
    } else if (t < 32) {
      mt = (t - 16) / 4; nt = (t - 16) % 4;
      A = T.dZ2 + mt * 16; sak = kMlpH;
      B = T.H1 + nt * 16; sbk = kMlpH;
      off = kOffW2; ldo = kMlpH;
    } else {
      mt = 0; nt = t - 32;
      A = T.dO; sak = kMlpOut;
      B = T.H2 + nt * 16; sbk = kMlpH;
      off = kOffW3; ldo = kMlpH;
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = wave_gemm<64>(A, 1, sak, B, sbk, 1, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) P[off + (mt * 16 + 4 * g + i) * ldo + nt * 16 + r] = acc[i];
  }
  // bias gradients: column sums over the workgroup's samples, FP32, fixed order
  for (int u = threadIdx.x; u < 2 * kMlpH + kMlpOut; u += blockDim.x) {
    float sacc = 0.f;
    if (u < kMlpH) {
      for (int s = 0; s < 64; ++s) sacc += T.Z1[s * kMlpH + u];
      P[kOffB1 + u] = sacc;
    } else if (u < 2 * kMlpH) {
      for (int s = 0; s < 64; ++s) sacc += T.Z2[s * kMlpH + (u - kMlpH)];
      P[kOffB2 + u - kMlpH] = sacc;
    } else {
      for (int s = 0; s < 64; ++s) sacc += T.O[s * kMlpOut + (u - 2 * kMlpH)];
      P[kOffB3 + u - 2 * kMlpH] = sacc;
    }
  }
  if (threadIdx.x == 0) {
    float l = 0.f;
    for (int s = 0; s < 64; ++s) l += T.loss[s];
    loss_part[blockIdx.x] = l;
  }
}

// Sum the per-workgroup partials in a fixed order (deterministic).
__global__ void mlp_reduce_kernel(const float* part, int nparts, const float* loss_part, int n, float* grad,
                                  float* loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMlpParams) {
    float s = 0.f;
    for (int p = 0; p < nparts; ++p) s += part[(long long)p * kMlpParams + i];
    grad[i] = s;
  }
  if (i == 0) {
    float l = 0.f;
    for (int p = 0; p < nparts; ++p) l += loss_part[p];
    *loss = l / (float)(n * kMlpUse);
  }
}

// Adam step on the FP32 master parameters, then the BF16 working copies.
__global__ void mlp_adam_kernel(float* params, float* m, float* v, const float* grad, float lr, float b1, float b2,
                                float eps, int t, unsigned short* w1, unsigned short* w2, unsigned short* w3) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  const float g = grad[i];
  const float mi = b1 * m[i] + (1.f - b1) * g;
  const float vi = b2 * v[i] + (1.f - b2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.f - powf(b1, (float)t));
  const float vh = vi / (1.f - powf(b2, (float)t));
  const float p = params[i] - lr * mh / (sqrtf(vh) + eps);
  params[i] = p;
  if (i >= kOffW1 && i < kOffW1 + kMlpH * kMlpIn) w1[i - kOffW1] = f2bf(p);
  if (i >= kOffW2 && i < kOffW2 + kMlpH * kMlpH) w2[i - kOffW2] = f2bf(p);
  if (i >= kOffW3 && i < kOffW3 + kMlpOut * kMlpH) w3[i - kOffW3] = f2bf(p);
}

__global__ void mlp_pack_kernel(const float* params, unsigned short* w1, unsigned short* w2, unsigned short* w3) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kMlpParams) return;
  const float p = params[i];
  if (i >= kOffW1 && i < kOffW1 + kMlpH * kMlpIn) w1[i - kOffW1] = f2bf(p);
  if (i >= kOffW2 && i < kOffW2 + kMlpH * kMlpH) w2[i - kOffW2] = f2bf(p);
  if (i >= kOffW3 && i < kOffW3 + kMlpOut * kMlpH) w3[i - kOffW3] = f2bf(p);
}

// ------------------------------------------------------------------ launchers
hipError_t mlp_pack(const MlpNet& net, hipStream_t s) {
  mlp_pack_kernel<<<(kMlpParams + 255) / 256, 256, 0, s>>>(net.params, net.w1, net.w2, net.w3);
  return hipGetLastError();
}

hipError_t mlp_forward(const MlpNet& net, const float* X, int n, float* out, hipStream_t s) {
  mlp_forward_kernel<<<(n + 63) / 64, 256, 0, s>>>(net, X, n, out);
  return hipGetLastError();
}

hipError_t mlp_grad(const MlpNet& net, const float* X, const float* Y, int n, float* part, float* loss_part,
                    float* grad, float* loss, hipStream_t s) {
  const int nparts = (n + 63) / 64;
  mlp_grad_kernel<<<nparts, 256, 0, s>>>(net, X, Y, n, part, loss_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  mlp_reduce_kernel<<<(kMlpParams + 255) / 256, 256, 0, s>>>(part, nparts, loss_part, n, grad, loss);
  return hipGetLastError();
}

hipError_t mlp_adam(const MlpNet& net, float* m, float* v, const float* grad, float lr, int t, hipStream_t s) {
  mlp_adam_kernel<<<(kMlpParams + 255) / 256, 256, 0, s>>>(net.params, m, v, grad, lr, 0.9f, 0.999f, 1e-8f, t,
                                                           net.w1, net.w2, net.w3);
  return hipGetLastError();
}

template <typename T>
hipError_t mlp_sample(const MlpFeatArgs<T>& a, const HaloRegion* regions, const FaceInfo* faces,
                      const int* face_regions, int nface, const double* W0, unsigned long long seed, int n, float* X,
                      float* Y, hipStream_t s) {
  mlp_sample_kernel<T><<<(n + 255) / 256, 256, 0, s>>>(a, regions, faces, face_regions, nface, W0, seed, n, X, Y);
  return hipGetLastError();
}

template <typename T>
hipError_t mlp_halo(const MlpFeatArgs<T>& a, const MlpNet& net, const HaloRegion* regions, const FaceInfo* faces,
                    const HaloWork* chunks, long long nchunks, const int8_t* delays, T* hbuf, long long halo_stride,
                    int stages, unsigned long long* counters, hipStream_t s) {
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const long long nblk = std::min<long long>((nchunks + 3) / 4, (long long)cus * 4);
  if (nblk < 1) return hipSuccess;
  if (stages < 1 || stages > kMlpMaxStages) return hipErrorInvalidValue;
  mlp_halo_kernel<T><<<(unsigned)nblk, 256, 0, s>>>(a, net, regions, faces, chunks, nchunks, delays, hbuf,
                                                    halo_stride, stages, counters);
  return hipGetLastError();
}

#define ATNS_MLP_INST(T)                                                                                       \
  template hipError_t mlp_sample<T>(const MlpFeatArgs<T>&, const HaloRegion*, const FaceInfo*, const int*, int, \
                                    const double*, unsigned long long, int, float*, float*, hipStream_t);     \
  template hipError_t mlp_halo<T>(const MlpFeatArgs<T>&, const MlpNet&, const HaloRegion*, const FaceInfo*,     \
                                  const HaloWork*, long long, const int8_t*, T*, long long, int,               \
                                  unsigned long long*, hipStream_t);
ATNS_MLP_INST(float)
ATNS_MLP_INST(double)

}  // namespace atns
