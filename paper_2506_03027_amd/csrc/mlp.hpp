// Learned halo correction: network sizes, parameter layout and kernel
// arguments shared by the host code and mlp.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "layout.hpp"

namespace atns {

constexpr int kMlpIn = 64, kMlpH = 64, kMlpOut = 16, kMlpUse = 5;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpH * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpH;
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH;
constexpr int kOffB3 = kOffW3 + kMlpOut * kMlpH;
constexpr int kMlpParams = kOffB3 + kMlpOut;   // 9360
constexpr int kMlpChunk = 16;                  // face-halo points per wave
constexpr int kMlpMaxStages = 5;               // RK stages a correction is added to (LSERK4)

struct MlpNet {
  float* params;        // FP32 master parameters (kMlpParams)
  unsigned short* w1;   // BF16 working copies of the weight matrices
  unsigned short* w2;
  unsigned short* w3;
};

// A face halo region: its normal axis and extents (x, y, z).
struct FaceInfo {
  int axis;
  int ext[3];
};

template <typename T>
struct MlpFeatArgs {
  const T* ring;
  long long slot_stride;
  int D;
  int slot_now;
  const long long* nstep;   // when set, slot_now = *nstep % D
  int L;
  float inv_s[5];   // 1 / feature scale per variable
  float inv_r[5];   // 1 / target scale per variable
  float r[5];       // target scale per variable
  float tau2;       // fallback threshold, squared
};

hipError_t mlp_pack(const MlpNet& net, hipStream_t s);
hipError_t mlp_forward(const MlpNet& net, const float* X, int n, float* out, hipStream_t s);
hipError_t mlp_grad(const MlpNet& net, const float* X, const float* Y, int n, float* part, float* loss_part,
                    float* grad, float* loss, hipStream_t s);
hipError_t mlp_adam(const MlpNet& net, float* m, float* v, const float* grad, float lr, int t, hipStream_t s);
template <typename T>
hipError_t mlp_sample(const MlpFeatArgs<T>& a, const HaloRegion* regions, const FaceInfo* faces,
                      const int* face_regions, int nface, const double* W0, unsigned long long seed, int n, float* X,
                      float* Y, hipStream_t s);
template <typename T>
hipError_t mlp_halo(const MlpFeatArgs<T>& a, const MlpNet& net, const HaloRegion* regions, const FaceInfo* faces,
                    const HaloWork* chunks, long long nchunks, const int8_t* delays, T* hbuf, long long halo_stride,
                    int stages, unsigned long long* counters, hipStream_t s);

}  // namespace atns
