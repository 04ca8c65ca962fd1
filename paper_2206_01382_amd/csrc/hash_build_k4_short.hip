// Instantiation of the build-side hash kernels: up to 4 bucket(s) per point, short rotations.
#include "hash_build.hpp"

namespace fpp {
hipError_t launch_hash_build_k4_short(const fpp_index* ix, int t0, int Tc, uint32_t* rb, float* rk,
                                  hipStream_t s) {
  return detail::launch_build_k_short<4>(ix, t0, Tc, rb, rk, s);
}
}  // namespace fpp
