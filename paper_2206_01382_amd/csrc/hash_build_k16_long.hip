// Instantiation of the build-side hash kernels: up to 16 bucket(s) per point, long rotations.
#include "hash_build.hpp"

namespace fpp {
hipError_t launch_hash_build_k16_long(const fpp_index* ix, int t0, int Tc, uint32_t* rb, float* rk,
                                  hipStream_t s) {
  return detail::launch_build_k_long<16>(ix, t0, Tc, rb, rk, s);
}
}  // namespace fpp
