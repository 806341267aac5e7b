// Adjoint of correlation plus reconstruction for the loss
//   L = sum_i g_i |rho_{j_i}[n_i]|^2,  rho_j[n] = sum_k C_jk Z_k[n],
//   Z_k[n] = sum_{f in band} d[f] conj(P_k[f]) e^{+2 pi i f n / N},
//   d[f] = wd[f] sum_m s[m] e^{-2 pi i f m / N}
// (Eq. Beta_eqn with C = conj(c); Eq. basis_SNR for Z).  For a real loss the
// gradient of a complex leaf is dL/dRe + i dL/dIm:
//   dL/dC_jk = 2 sum_{i: j_i = j} g_i rho_i conj(Z_k[n_i])
//   dL/ds[m] = 2 Re sum_f B[f] e^{-2 pi i f m / N},
//   B[f] = wd[f] sum_k conj(P_k[f]) Ahat_k[f],  Ahat_k[f] = sum_n A_k[n] e^{+2 pi i f n / N},
//   A_k[n] = sum_{i: n_i = n} g_i conj(rho_i) C_{j_i k}.
// The scatter of A and the transforms reuse the batched FFT passes.  All
// reductions run in a fixed order (deterministic): triggers are grouped by
// template (for dL/dC) and by sample (for A) on the host.
#include "internal.h"

namespace rbmf {

namespace {

__device__ __forceinline__ int64_t pos_of(int64_t n, int N1, int N2) {
  return (n % N2) * N1 + n / N2;   // n = n2 + N2 n1  ->  q = n2 N1 + n1
}

// rho_i = sum_k C[j_i][k] Z_k[n_i], one wave per trigger.
__global__ void k_rho_at(const float* z, int64_t N, int K, int N1, int N2, const float2* C,
                         const int32_t* tmpl, const int32_t* samp, int64_t n, float2* rho) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n) return;
  const int j = tmpl[i];
  const int64_t q = pos_of(samp[i], N1, N2);
  float re = 0.f, im = 0.f;
  for (int k = lane; k < K; k += 64) {
    const float zr = z[(2 * (int64_t)k) * N + q], zi = z[(2 * (int64_t)k + 1) * N + q];
    const float2 c = C[(int64_t)j * K + k];
    re += c.x * zr - c.y * zi;
    im += c.x * zi + c.y * zr;
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_xor(re, off);
    im += __shfl_xor(im, off);
  }
  if (lane == 0) rho[i] = make_float2(re, im);
}

// dL/dC rows: one workgroup per template segment of the tmpl-sorted order.
__global__ void k_grad_c(const float* z, int64_t N, int K, int N1, int N2, const int32_t* order,
                         const int32_t* seg_off, const int32_t* tmpl, const int32_t* samp, const float2* rho,
                         const float* g, float2* gC) {
  const int s0 = seg_off[blockIdx.x], s1 = seg_off[blockIdx.x + 1];
  const int j = tmpl[order[s0]];
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    float re = 0.f, im = 0.f;
    for (int s = s0; s < s1; ++s) {
      const int i = order[s];
      const int64_t q = pos_of(samp[i], N1, N2);
      const float zr = z[(2 * (int64_t)k) * N + q], zi = z[(2 * (int64_t)k + 1) * N + q];
      const float2 r = rho[i];
      const float w = 2.f * (g ? g[i] : 1.f);
      // rho conj(Z)
      re += w * (r.x * zr + r.y * zi);
      im += w * (r.y * zr - r.x * zi);
    }
    gC[(int64_t)j * K + k] = make_float2(re, im);
  }
}

// A_k[n] for one distinct sample per workgroup (natural order, K x N).
__global__ void k_scatter_a(int K, int64_t N, const int32_t* order, const int32_t* seg_off, const int32_t* tmpl,
                            const int32_t* samp, const float2* rho, const float* g, const float2* C, float2* A) {
  const int s0 = seg_off[blockIdx.x], s1 = seg_off[blockIdx.x + 1];
  const int64_t n = samp[order[s0]];
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    float re = 0.f, im = 0.f;
    for (int s = s0; s < s1; ++s) {
      const int i = order[s];
      const float2 r = rho[i];
      const float2 c = C[(int64_t)tmpl[i] * K + k];
      const float w = g ? g[i] : 1.f;
      // g conj(rho) C
      re += w * (r.x * c.x + r.y * c.y);
      im += w * (r.x * c.y - r.y * c.x);
    }
    A[(int64_t)k * N + n] = make_float2(re, im);
  }
}

// B[f] = wd[f] sum_k conj(P_k[f]) Ahat_k[f] on the band (Ahat natural order).
__global__ void k_bsum(const float2* Ahat, const float2* P, const double* wd, int K, int64_t N, int64_t kb,
                       int64_t nbs, int64_t k_lo, int64_t k_hi, float2* B) {
  for (int64_t f = k_lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f <= k_hi;
       f += (int64_t)gridDim.x * blockDim.x) {
    float re = 0.f, im = 0.f;
    for (int k = 0; k < K; ++k) {
      const float2 p = P[(int64_t)k * nbs + (f - kb)];
      const float2 a = Ahat[(int64_t)k * N + f];
      re += p.x * a.x + p.y * a.y;
      im += p.x * a.y - p.y * a.x;
    }
    const float w = (float)wd[f - kb];
    B[f] = make_float2(re * w, im * w);
  }
}

__global__ void k_real2(const float2* x, int64_t N, float* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = 2.f * x[i].x;
}

}  // namespace

hipError_t launch_rho_at(const float* z, int64_t N, int K, int N1, int N2, const float2* C, const int32_t* tmpl,
                         const int32_t* samp, int64_t n, float2* rho, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int per = 4;   // waves per 256-thread workgroup
  hipLaunchKernelGGL(k_rho_at, dim3((unsigned)((n + per - 1) / per)), dim3(256), 0, s, z, N, K, N1, N2, C, tmpl,
                     samp, n, rho);
  return hipGetLastError();
}

hipError_t launch_grad_c(const float* z, int64_t N, int K, int N1, int N2, const int32_t* order,
                         const int32_t* seg_off, int nseg, const int32_t* tmpl, const int32_t* samp,
                         const float2* rho, const float* g, float2* gC, hipStream_t s) {
  if (nseg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_c, dim3(nseg), dim3(256), 0, s, z, N, K, N1, N2, order, seg_off, tmpl, samp, rho, g,
                     gC);
  return hipGetLastError();
}

hipError_t launch_scatter_a(int K, int64_t N, const int32_t* order, const int32_t* seg_off, int nseg,
                            const int32_t* tmpl, const int32_t* samp, const float2* rho, const float* g,
                            const float2* C, float2* A, hipStream_t s) {
  if (nseg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_a, dim3(nseg), dim3(256), 0, s, K, N, order, seg_off, tmpl, samp, rho, g, C, A);
  return hipGetLastError();
}

hipError_t launch_bsum(const float2* Ahat, const float2* P, const double* wd, int K, int64_t N, int64_t kb,
                       int64_t nbs, int64_t k_lo, int64_t k_hi, float2* B, hipStream_t s) {
  hipLaunchKernelGGL(k_bsum, dim3(2048), dim3(256), 0, s, Ahat, P, wd, K, N, kb, nbs, k_lo, k_hi, B);
  return hipGetLastError();
}

hipError_t launch_real2(const float2* x, int64_t N, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_real2, dim3(1024), dim3(256), 0, s, x, N, out);
  return hipGetLastError();
}

}  // namespace rbmf
