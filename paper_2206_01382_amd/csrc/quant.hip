// Low-precision scoring stores (an addition to the paper's method).
//   BF16: each element rounded to bfloat16, nearest, ties to even.
//   FP8:  per vector s = fl32(max|x| / 448) (s = 1 for a zero vector); element codes are
//         OCP E4M3 (bias 7, largest finite 448, no infinities) of fl32(x / s), nearest with
//         ties to the even code, magnitudes >= 448 saturating to 448.
// Rows are padded with zeros to a multiple of 16 bytes; an FP8 row may also carry its scale
// (after the codes, in a 16-byte chunk of its own).
#include "fpp_internal.hpp"

namespace fpp {
namespace {

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ uint32_t e4m3_rne_sat(float v) {
  const uint32_t u = __float_as_uint(v);
  const uint32_t sign = (u >> 24) & 0x80u;
  const float a = fabsf(v);
  uint32_t code;
  if (!(a < 448.0f)) {
    code = 0x7eu;
  } else if (a < 0.015625f) {                    // below 2^-6: multiples of 2^-9
    code = (uint32_t)rintf(a * 512.0f);          // exact scaling, nearest-even; 8 is 2^-6
  } else {
    int e = (int)((u >> 23) & 0xffu) - 127;      // a is a normal float32 here
    const float m = ldexpf(a, -e);               // [1, 2), exact
    uint32_t mm = (uint32_t)rintf((m - 1.0f) * 8.0f);
    if (mm == 8u) {
      mm = 0u;
      e += 1;
    }
    code = ((uint32_t)(e + 7) << 3) | mm;
    if (code > 0x7eu) code = 0x7eu;
  }
  return sign | code;
}

__global__ __launch_bounds__(256) void quant_bf16_kernel(const float* __restrict__ X, int64_t n,
                                                         int d, int ldx,
                                                         uint16_t* __restrict__ out, int ld16) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * ld16) return;
  const int64_t r = i / ld16;
  const int c = (int)(i - r * ld16);
  out[i] = c < d ? bf16_rne(X[r * ldx + c]) : (uint16_t)0;
}

// One wavefront per row: the float32 sum of squares, whose rounding (at most d / 64 + 6 steps)
// and that of the square root are covered by the factor 1 + 2^-16, so the value is an upper bound
// of the row's L2 norm; the maximum over rows by an integer atomic max on the (non-negative)
// float bits.
__global__ __launch_bounds__(256) void row_norm_max_kernel(const float* __restrict__ X, int64_t n,
                                                           int d, int ldx, uint32_t* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  const float* x = X + r * ldx;
  float ss = 0.0f;
  for (int c = lane; c < d; c += 64) ss = fmaf(x[c], x[c], ss);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ss += __shfl_xor(ss, o);
  if (lane == 0) atomicMax(out, __float_as_uint(sqrtf(ss) * 1.0000152587890625f));
}

// One wavefront per row. With sc_off >= 0 the scale is also stored inside the row at byte sc_off.
__global__ __launch_bounds__(256) void quant_fp8_kernel(const float* __restrict__ X, int64_t n,
                                                        int d, int ldx, uint8_t* __restrict__ out,
                                                        int ld8, int sc_off, float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  const float* x = X + r * ldx;
  float mx = 0.0f;
  for (int c = lane; c < d; c += 64) mx = fmaxf(mx, fabsf(x[c]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  const float s = mx == 0.0f ? 1.0f : __fdiv_rn(mx, 448.0f);
  for (int c = lane; c < ld8; c += 64)
    if (sc_off < 0 || c < sc_off || c >= sc_off + 4)
      out[r * ld8 + c] = c < d ? (uint8_t)e4m3_rne_sat(__fdiv_rn(x[c], s)) : (uint8_t)0;
  if (lane == 0) {
    scale[r] = s;
    if (sc_off >= 0) *reinterpret_cast<float*>(out + r * ld8 + sc_off) = s;
  }
}

// Centred copy for the build's hashing: xc[i][j] = fl32(x[i][j] - c[j]) for j < d, 0 in the row
// padding (Section 3.4, heuristic 1).
__global__ __launch_bounds__(256) void center_kernel(const float* __restrict__ X, int64_t n, int d,
                                                     int ldx, const float* __restrict__ c,
                                                     float* __restrict__ Xc) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n * ldx) return;
  const int j = (int)(i % ldx);
  Xc[i] = j < d ? X[i] - c[j] : 0.0f;
}

}  // namespace

hipError_t launch_center(const fpp_index* ix, float* Xc, hipStream_t s) {
  const int64_t tot = ix->n * ix->ldx;
  hipLaunchKernelGGL(center_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, ix->X,
                     ix->n, ix->d, ix->ldx, ix->center_vec, Xc);
  return hipGetLastError();
}

hipError_t launch_quantize(const fpp_index* ix, hipStream_t s) {
  if (ix->Xbf16) {
    const int64_t tot = ix->n * ix->ld16;
    hipLaunchKernelGGL(quant_bf16_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                       ix->X, ix->n, ix->d, ix->ldx, ix->Xbf16, ix->ld16);
  }
  if (ix->Xfp8) {
    hipLaunchKernelGGL(quant_fp8_kernel, dim3((unsigned)((ix->n + 3) / 4)), dim3(256), 0, s, ix->X,
                       ix->n, ix->d, ix->ldx, ix->Xfp8, ix->ld8, ix->fp8_sc_off, ix->fp8_scale);
  }
  return hipGetLastError();
}

hipError_t launch_row_norm_max(const fpp_index* ix, uint32_t* out, hipStream_t s) {
  if (ix->n <= 0) return hipSuccess;
  hipLaunchKernelGGL(row_norm_max_kernel, dim3((unsigned)((ix->n + 3) / 4)), dim3(256), 0, s, ix->X,
                     ix->n, ix->d, ix->ldx, out);
  return hipGetLastError();
}

}  // namespace fpp
