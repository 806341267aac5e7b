// FP64 complex GEMM and helpers for the basis construction (Sec. II.A and
// III.B: covariance / Gram products of the whitened templates, projection of
// the templates on the basis).  Off the timed path; FP64 arithmetic
// throughout, operands may be the stored complex64 templates.
//
// C[m][n] (+)= sum_k opA[m][k] opB[k][n]: 64 x 64 output tiles, 16-deep
// reduction slabs staged in LDS, 4 x 4 complex outputs per thread, split over
// the reduction dimension into deterministic partial sums when the output
// alone cannot fill the GPU.
#include <algorithm>

#include "internal.h"

namespace rbmf {

namespace {

constexpr int TM = 64, TN = 64, TK = 16;

__device__ __forceinline__ double2 zld(const ZOperand& o, int64_t r, int64_t c) {
  const int64_t idx = r * o.rs + c * o.cs;
  double2 v;
  if (o.is_c64) {
    const float2 f = static_cast<const float2*>(o.p)[idx];
    v = make_double2((double)f.x, (double)f.y);
  } else {
    v = static_cast<const double2*>(o.p)[idx];
  }
  if (o.conj) v.y = -v.y;
  return v;
}

__global__ __launch_bounds__(256) void k_zgemm(int64_t M, int64_t Nn, int64_t Kd, ZOperand A, ZOperand B,
                                               double2* C, int64_t ldc, int64_t kchunk, int64_t part_stride,
                                               int accumulate) {
  __shared__ double2 As[TK][TM + 1];
  __shared__ double2 Bs[TK][TN + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t n0 = (int64_t)blockIdx.x * TN;
  const int64_t m0 = (int64_t)blockIdx.y * TM;
  const int64_t k_begin = (int64_t)blockIdx.z * kchunk;
  const int64_t k_end = min(Kd, k_begin + kchunk);
  const bool a_mfast = (A.rs == 1);
  const bool b_nfast = (B.cs == 1) || (B.rs != 1);
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);

  for (int64_t k0 = k_begin; k0 < k_end; k0 += TK) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int idx = tid + 256 * r;
      int mm, kk;
      if (a_mfast) { mm = idx & 63; kk = idx >> 6; } else { kk = idx & 15; mm = idx >> 4; }
      const int64_t gm = m0 + mm, gk = k0 + kk;
      As[kk][mm] = (gm < M && gk < k_end) ? zld(A, gm, gk) : make_double2(0.0, 0.0);
      int nn, kb;
      if (b_nfast) { nn = idx & 63; kb = idx >> 6; } else { kb = idx & 15; nn = idx >> 4; }
      const int64_t gn = n0 + nn, gkb = k0 + kb;
      Bs[kb][nn] = (gn < Nn && gkb < k_end) ? zld(B, gkb, gn) : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < TK; ++kk) {
      double2 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j].x = fma(a[i].x, b[j].x, fma(-a[i].y, b[j].y, acc[i][j].x));
          acc[i][j].y = fma(a[i].x, b[j].y, fma(a[i].y, b[j].x, acc[i][j].y));
        }
    }
    __syncthreads();
  }
  double2* Cp = C + (int64_t)blockIdx.z * part_stride;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t gm = m0 + ty + 16 * i, gn = n0 + tx + 16 * j;
      if (gm < M && gn < Nn) {
        double2* dst = Cp + gm * ldc + gn;
        if (accumulate) {
          const double2 o = *dst;
          *dst = make_double2(o.x + acc[i][j].x, o.y + acc[i][j].y);
        } else {
          *dst = acc[i][j];
        }
      }
    }
}

// C[m][n] (+)= sum_s part[s][m][n] in a fixed order (deterministic).
__global__ void k_zreduce(const double2* part, int S, int64_t M, int64_t Nn, double2* C, int64_t ldc,
                          int accumulate) {
  const int64_t total = M * Nn;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = i / Nn, n = i % Nn;
    double2 s = accumulate ? C[m * ldc + n] : make_double2(0.0, 0.0);
    for (int p = 0; p < S; ++p) {
      const double2 v = part[(int64_t)p * total + i];
      s.x += v.x;
      s.y += v.y;
    }
    C[m * ldc + n] = s;
  }
}

__global__ void k_c128_to_c64(const double2* in, int64_t rows, int64_t cols, int64_t ld_in,
                              const double* row_scale, int conj, float2* out, int64_t ld_out) {
  const int64_t total = rows * cols;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / cols, c = i % cols;
    double2 v = in[r * ld_in + c];
    const double s = row_scale ? row_scale[r] : 1.0;
    out[r * ld_out + c] = make_float2((float)(v.x * s), (float)(conj ? -v.y * s : v.y * s));
  }
}

// Basis rows from BS (nb x K, row stride ld): out[k][off + f] =
// scale[k] conj(BS[f][k]) as complex64, zero for the first `off` stored bins.
__global__ void k_basis_rows(const double2* BS, int64_t nb, int K, int64_t ld, const double* scale,
                             int64_t off, int64_t nbs, float2* out) {
  const int64_t total = (int64_t)K * nbs;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = i / nbs, fs = i % nbs;
    float2 v = make_float2(0.f, 0.f);
    const int64_t f = fs - off;
    if (f >= 0 && f < nb) {
      const double2 b = BS[f * ld + k];
      v = make_float2((float)(b.x * scale[k]), (float)(-b.y * scale[k]));
    }
    out[i] = v;
  }
}

// FP64 squared norms of complex64 rows.
__global__ __launch_bounds__(256) void k_row_norms(const float2* w, int64_t len, int64_t ld, double* out) {
  __shared__ double sh[4];
  const int64_t r = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < len; i += blockDim.x) {
    const float2 v = w[r * ld + i];
    s += (double)v.x * v.x + (double)v.y * v.y;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[r] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Linear interpolation of basis columns from a non-uniform frequency set to
// the uniform band: out[f][k] = scale[k] ((1 - a_f) r_i B[i][k] + a_f r_{i+1}
// B[i+1][k]) with i = idx[f], a_f = frac[f], r = 1/sqrt(cell weight).  One
// thread per (f, k), k fastest: the B rows i and i+1 and the out row f are
// read and written contiguously.
__global__ __launch_bounds__(256) void k_interp_rows(const double2* B, int K, const int32_t* idx, const double* frac,
                                                     const double* r, const double* scale, int64_t nb, double2* out) {
  const int64_t total = nb * (int64_t)K;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = t / K;
    const int k = (int)(t - f * K);
    const int64_t i = idx[f];
    const double a = frac[f];
    const double w0 = (1.0 - a) * r[i] * scale[k], w1 = a * r[i + 1] * scale[k];
    const double2 b0 = B[i * K + k], b1 = B[(i + 1) * K + k];
    out[t] = make_double2(w0 * b0.x + w1 * b1.x, w0 * b0.y + w1 * b1.y);
  }
}

}  // namespace

hipError_t launch_interp_rows(const double2* B, int64_t nt, int K, const int32_t* idx, const double* frac,
                              const double* r, const double* scale, int64_t nb, double2* out, hipStream_t s) {
  if (nt < 2 || K < 1 || nb < 1) return hipErrorInvalidValue;
  const int64_t total = nb * (int64_t)K;
  const int64_t blocks = std::min<int64_t>(8192, (total + 255) / 256);
  hipLaunchKernelGGL(k_interp_rows, dim3((unsigned)blocks), dim3(256), 0, s, B, K, idx, frac, r, scale, nb, out);
  return hipGetLastError();
}

hipError_t launch_zgemm(int64_t M, int64_t Nn, int64_t Kd, ZOperand A, ZOperand B, double2* C, int64_t ldc,
                        int accumulate, double2* workspace, int64_t workspace_elems, hipStream_t s) {
  const int64_t mt = (M + TM - 1) / TM, nt = (Nn + TN - 1) / TN;
  int64_t S = 1;
  const int64_t tiles = mt * nt;
  if (tiles < 1024 && Kd > 512) {
    S = (1024 + tiles - 1) / tiles;
    const int64_t maxS = Kd / 256;
    if (S > maxS) S = maxS;
    if (S < 1) S = 1;
    if (S * M * Nn > workspace_elems) S = workspace_elems / (M * Nn);
    if (S < 2) S = 1;
  }
  int64_t kchunk = (Kd + S - 1) / S;
  kchunk = ((kchunk + TK - 1) / TK) * TK;
  if (S == 1) {
    hipLaunchKernelGGL(k_zgemm, dim3((unsigned)nt, (unsigned)mt, 1), dim3(256), 0, s, M, Nn, Kd, A, B, C, ldc,
                       kchunk, (int64_t)0, accumulate);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_zgemm, dim3((unsigned)nt, (unsigned)mt, (unsigned)S), dim3(256), 0, s, M, Nn, Kd, A, B,
                     workspace, Nn, kchunk, M * Nn, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zreduce, dim3(2048), dim3(256), 0, s, workspace, (int)S, M, Nn, C, ldc, accumulate);
  return hipGetLastError();
}

hipError_t launch_c128_to_c64_rows(const double2* in, int64_t rows, int64_t cols, int64_t ld_in,
                                   const double* row_scale, int conj, float2* out, int64_t ld_out,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_c128_to_c64, dim3(2048), dim3(256), 0, s, in, rows, cols, ld_in, row_scale, conj, out,
                     ld_out);
  return hipGetLastError();
}

hipError_t launch_basis_rows(const double2* BS, int64_t nb, int K, int64_t ld, const double* scale, int64_t off,
                             int64_t nbs, float2* out, hipStream_t s) {
  hipLaunchKernelGGL(k_basis_rows, dim3(4096), dim3(256), 0, s, BS, nb, K, ld, scale, off, nbs, out);
  return hipGetLastError();
}

hipError_t launch_row_norms(const float2* w, int64_t rows, int64_t len, int64_t ld, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_row_norms, dim3((unsigned)rows), dim3(256), 0, s, w, len, ld, out);
  return hipGetLastError();
}

}  // namespace rbmf
