// Reduced-precision storage copy on the device: FP8-E4M3 rows with one FP32
// scale per row, the 8-bit storage format searched with FP32 arithmetic (the
// quantization the paper layers under the index, Section 2).
//
// Row r gets s_r = max_i |x_ri| / 448 (1 for an all-zero row), both in FP32,
// and code_ri = E4M3(x_ri / s_r): OCP E4M3 (1 sign, 4 exponent bits with bias
// 7, 3 mantissa bits, no infinities, largest finite 448), rounded to nearest
// even from the FP32 quotient, saturating at +-448, NaN to 0x7F (with sign).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ann.h"
#include "internal.h"

namespace ann {
namespace {

// E4M3 code of an FP32 value, round to nearest even, saturating.
__device__ __forceinline__ uint32_t to_e4m3(float v) {
  const uint32_t bits = __float_as_uint(v);
  const uint32_t sign = (bits >> 24) & 0x80u;
  const uint32_t mag = bits & 0x7FFFFFFFu;
  if (mag > 0x7F800000u) return sign | 0x7Fu;                 // NaN
  const float a = __uint_as_float(mag);
  if (a >= 448.0f) return sign | 0x7Eu;                        // saturate (and +-inf)
  if (a < 0x1p-6f) {                                           // subnormal E4M3: units of 2^-9
    const float q = __builtin_rintf(a * 512.0f);               // exact scaling, then RNE
    return sign | (uint32_t)q;                                 // q = 8 is the smallest normal
  }
  int e = (int)(mag >> 23) - 127;                              // a is a normal FP32 here
  // the 4 leading significand bits (implicit one + 3), rounded to nearest
  // even on the 20 bits below them
  uint32_t m = (0x800000u | (mag & 0x7FFFFFu)) >> 20;
  const uint32_t rest = mag & 0xFFFFFu;
  if (rest > 0x80000u || (rest == 0x80000u && (m & 1u))) ++m;
  if (m == 16u) { m = 8u; ++e; }
  uint32_t code = ((uint32_t)(e + 7) << 3) | (m - 8u);
  if (code > 0x7Eu) code = 0x7Eu;
  return sign | code;
}

// One wavefront per row: the row's largest magnitude (a max, exact in any
// order), the scale, then the codes.
__global__ void __launch_bounds__(256) encode_fp8_rows(const float* X, int64_t n, int d,
                                                       uint8_t* codes, float* scale) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= n) return;
  const float* x = X + (size_t)r * d;
  float mx = 0.0f;
  for (int i = lane; i < d; i += 64) mx = fmaxf(mx, fabsf(x[i]));
  for (int s = 32; s >= 1; s >>= 1) mx = fmaxf(mx, __shfl_xor(mx, s, 64));
  const float sc = mx > 0.0f ? mx / 448.0f : 1.0f;
  if (lane == 0) scale[r] = sc;
  for (int i = lane; i < d; i += 64) codes[(size_t)r * d + i] = (uint8_t)to_e4m3(x[i] / sc);
}

}  // namespace
}  // namespace ann

using namespace ann;

extern "C" int ann_encode_fp8(const float* X, int64_t n, int32_t d, uint8_t* out_codes,
                              float* out_scale, void* stream) {
  if (n < 0 || d < 1) return fail(ANN_EINVAL, "n %lld, d %d", (long long)n, d);
  if (n == 0) return ANN_OK;
  if (!X || !out_codes || !out_scale) return fail(ANN_EINVAL, "NULL pointer");
  hipStream_t st = (hipStream_t)stream;
  const int64_t blocks = (n + 3) / 4;
  if (blocks > 0x7FFFFFFF) return fail(ANN_EINVAL, "n too large");
  hipLaunchKernelGGL(encode_fp8_rows, dim3((unsigned)blocks), dim3(256), 0, st, X, n, d, out_codes,
                     out_scale);
  HIP_OR_RETURN(hipGetLastError(), "encode_fp8_rows launch");
  if (!stream) HIP_OR_RETURN(hipStreamSynchronize(st), "FP8 encoding");
  return ANN_OK;
}
