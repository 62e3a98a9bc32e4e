// Navier-Stokes stage kernel (placeholder until the viscous kernel lands).
#include "kernels_common.hpp"

namespace atns {

template <typename T>
hipError_t launch_ns_stage(const StageParams<T>&, int, int, hipStream_t) {
  return hipErrorNotSupported;
}
template hipError_t launch_ns_stage<float>(const StageParams<float>&, int, int, hipStream_t);
template hipError_t launch_ns_stage<double>(const StageParams<double>&, int, int, hipStream_t);

}  // namespace atns
