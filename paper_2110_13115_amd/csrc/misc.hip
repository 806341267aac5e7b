// Small device helpers: finiteness check of the strain, conversion of the
// stored (planar, possibly 16-bit, scaled) basis outputs to natural order.
#include "internal.h"

#include <hip/hip_fp16.h>

namespace rbmf {

namespace {

__global__ void k_check_finite(const float* x, int64_t n, int64_t* flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (__ballot(bad) != 0ull && __lane_id() == 0) atomicOr(reinterpret_cast<unsigned long long*>(flag), 1ull);
}

__device__ __forceinline__ float ld16(const uint16_t* p, int dtype) {
  const uint16_t u = *p;
  if (dtype == 1) return __uint_as_float(((uint32_t)u) << 16);
  return (float)__builtin_bit_cast(_Float16, u);
}

__global__ void k_z_to_natural(const void* z, int dtype, float inv_scale, int64_t N, int K, int N1, int N2,
                               float2* out) {
  const int64_t total = (int64_t)K * N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = i / N, q = i % N;
    const int64_t n = q / N1 + (int64_t)N2 * (q % N1);
    float re, im;
    if (dtype == 0) {
      const float* zf = static_cast<const float*>(z);
      re = zf[(2 * k) * N + q];
      im = zf[(2 * k + 1) * N + q];
    } else {
      const uint16_t* zh = static_cast<const uint16_t*>(z);
      re = ld16(zh + (2 * k) * N + q, dtype);
      im = ld16(zh + (2 * k + 1) * N + q, dtype);
    }
    out[k * N + n] = make_float2(re * inv_scale, im * inv_scale);
  }
}

}  // namespace

hipError_t launch_check_finite(const float* x, int64_t n, int64_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_finite, dim3(256), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}

hipError_t launch_z_to_natural(const void* z, int dtype, float inv_scale, int64_t N, int K, int N1, int N2,
                               float2* out, hipStream_t s) {
  hipLaunchKernelGGL(k_z_to_natural, dim3(4096), dim3(256), 0, s, z, dtype, inv_scale, N, K, N1, N2, out);
  return hipGetLastError();
}

}  // namespace rbmf
