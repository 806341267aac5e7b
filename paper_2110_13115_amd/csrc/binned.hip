// Binned (hierarchical) first stage, Sec. III.C: bin means of the basis
// outputs, the fine reconstruction of every sample of every triggering
// (template, bin), and the selection of the final triggers when the second
// stage is the reconstruction itself.
#include <hip/hip_fp16.h>

#include <algorithm>

#include "internal.h"

namespace rbmf {

namespace {

__device__ __forceinline__ uint16_t bin_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ uint16_t bin_f16_rne(float x) {
  __half h = __float2half_rn(x);
  return *reinterpret_cast<uint16_t*>(&h);
}

// Partial sums [N2/G][N1] -> bin means [N2/w][N1] (bin r'' of slice n1 is
// the natural bin r'' + (N2/w) n1), stored planar in the reconstruction
// dtype: plane 2v = Re, 2v + 1 = Im, plane stride Nb = N / w.
__global__ void k_bin_reduce(BinReduceArgs a) {
  const int64_t Nb = a.N / a.w;
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= Nb) return;
  const int v = a.vec_base + blockIdx.y;
  const int per = a.w / a.G;
  const int64_t r2 = o / a.N1, n1 = o % a.N1;
  const float2* p = a.part + (int64_t)v * (a.N / a.G) + (r2 * per) * a.N1 + n1;
  float sr = 0.f, si = 0.f;
  for (int u = 0; u < per; ++u) {   // fixed order
    const float2 x = p[(int64_t)u * a.N1];
    sr += x.x;
    si += x.y;
  }
  const float inv = 1.f / (float)a.w;   // w is a power of two: exact
  sr *= inv;
  si *= inv;
  if (a.dtype == 0) {
    float* z = static_cast<float*>(a.zavg);
    z[(int64_t)(2 * v) * Nb + o] = sr;
    z[(int64_t)(2 * v + 1) * Nb + o] = si;
    return;
  }
  uint16_t* z = static_cast<uint16_t*>(a.zavg);
  const float xr = sr * a.zscale, xi = si * a.zscale;
  uint16_t* zr = z + (int64_t)(2 * v) * Nb + o;
  uint16_t* zi = zr + Nb;
  if (a.dtype == 3) {
    const uint16_t hr = bin_bf16_rne(xr), hi = bin_bf16_rne(xi);
    zr[0] = hr;
    zi[0] = hi;
    zr[a.zplane] = bin_bf16_rne(xr - __uint_as_float((uint32_t)hr << 16));
    zi[a.zplane] = bin_bf16_rne(xi - __uint_as_float((uint32_t)hi << 16));
  } else if (a.dtype == 1) {
    zr[0] = bin_bf16_rne(xr);
    zi[0] = bin_bf16_rne(xi);
  } else {
    zr[0] = bin_f16_rne(xr);
    zi[0] = bin_f16_rne(xi);
  }
}

__global__ void k_copy_u64(const unsigned long long* src, unsigned long long* dst) {
  if (threadIdx.x == 0) *dst = *src;
}

template <int Z16>
__device__ __forceinline__ float2 fine_z(const void* z, int64_t idx) {
  if constexpr (Z16 == 0) {
    return static_cast<const float2*>(z)[idx];
  } else {
    const uint32_t u = static_cast<const uint32_t*>(z)[idx];
    if constexpr (Z16 == 1) return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
    __half_raw lo, hi;
    lo.x = (unsigned short)(u & 0xffffu);
    hi.x = (unsigned short)(u >> 16);
    return make_float2(__half2float(__half(lo)), __half2float(__half(hi)));
  }
}

constexpr int FINE_WAVES = 4;     // waves per workgroup
constexpr int FINE_STAGE = 128;   // candidate records staged per wave before one counter atomic

// One wave per triggering (template, bin) record: rho_RB at the w samples of
// the bin (Eq. Beta_eqn with C = conj(c), FP32 accumulation), the w lanes of
// sample r each summing every (64/w)-th basis vector, then a butterfly over
// the slices.  Samples with |rho_RB|^2 >= thr_sq are candidates: one count
// atomic per (template, bin), staged per wave in LDS and appended with one
// counter atomic per FINE_STAGE records.
template <int Z16>
__global__ __launch_bounds__(FINE_WAVES * 64) void k_fine_recon(FineArgs a) {
  __shared__ TrigRec stage[FINE_WAVES][FINE_STAGE];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int w = a.w;
  const int r = lane & (w - 1);
  const int slices = 64 / w;
  const int s = lane / w;
  const int64_t end = a.end ? (int64_t)min(*a.end, (unsigned long long)a.bins_cap) : a.end_h;
  const int64_t begin = a.begin ? (int64_t)*a.begin : a.begin_h;
  const int l2 = __builtin_ctz((unsigned)a.N2);
  int nst = 0;   // staged records of this wave (wave-uniform)
  auto flush = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    unsigned lo = 0, hi = 0;
    if (lane == 0) {
      const unsigned long long b = atomicAdd(a.out_count, (unsigned long long)nst);
      lo = (unsigned)b;
      hi = (unsigned)(b >> 32);
    }
    const unsigned long long base = ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)hi) << 32) |
                                    (unsigned)__builtin_amdgcn_readfirstlane((int)lo);
    for (int t = lane; t < nst; t += 64)
      if ((int64_t)(base + t) < a.out_cap) a.out[base + t] = stage[wave][t];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    nst = 0;
  };
  for (int64_t i = begin + (int64_t)blockIdx.x * FINE_WAVES + wave; i < end;
       i += (int64_t)gridDim.x * FINE_WAVES) {
    const TrigRec b = a.bins[i];
    const int j = b.tmpl - a.t0;
    const int64_t n = (int64_t)b.sample * w + r;
    const int row = (int)(n & (a.N2 - 1));
    const int64_t n1 = n >> l2;
    const int64_t q = (int64_t)(row & ~(a.F - 1)) * a.N1 + n1 * a.F + (row & (a.F - 1));
    const float2* c = a.C + (int64_t)j * a.K;
    float re = 0.f, im = 0.f;
    for (int k = s; k < a.K; k += slices) {
      const float2 zk = fine_z<Z16>(a.z, (int64_t)k * a.N + q);
      const float2 ck = c[k];
      re += ck.x * zk.x - ck.y * zk.y;
      im += ck.x * zk.y + ck.y * zk.x;
    }
    for (int off = w; off < 64; off <<= 1) {
      re += __shfl_xor(re, off);
      im += __shfl_xor(im, off);
    }
    const bool hit = lane < w && re * re + im * im >= a.thr_sq;
    const unsigned long long mask = __ballot(hit);
    if (mask == 0ull) continue;
    const int cnt = __popcll(mask);
    if (lane == 0) atomicAdd(&a.tmpl_count[b.tmpl], cnt);
    if (nst + cnt > FINE_STAGE) flush();
    if (hit) {
      TrigRec t;
      t.tmpl = b.tmpl;
      t.sample = (int32_t)n;
      t.re = re;
      t.im = im;
      stage[wave][nst + __popcll(mask & ((1ull << lane) - 1ull))] = t;
    }
    nst += cnt;
  }
  if (nst > 0) flush();
}

// Second stage = the reconstruction: candidates whose |rho|^2 (values times
// the template's inverse storage scale, if any) reaches thr2_sq are final;
// the per-template maximum runs over every candidate.
__global__ void k_select_final(const TrigRec* in, const unsigned long long* n_in, int64_t cap_in,
                               const float* inv_scale, float thr2_sq, TrigRec* out, int64_t out_cap,
                               unsigned long long* out_count, int32_t* tmpl_count,
                               unsigned long long* tmpl_max) {
  const int64_t n = (int64_t)min(*n_in, (unsigned long long)cap_in);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    TrigRec t = in[i];
    if (inv_scale) {
      const float sc = inv_scale[t.tmpl];
      t.re *= sc;
      t.im *= sc;
    }
    const float p = t.re * t.re + t.im * t.im;
    if (tmpl_max)
      atomicMax(&tmpl_max[t.tmpl],
                ((unsigned long long)__float_as_uint(p) << 32) | (unsigned long long)(0xffffffffu - (uint32_t)t.sample));
    if (p >= thr2_sq) {
      atomicAdd(&tmpl_count[t.tmpl], 1);
      const unsigned long long idx = atomicAdd(out_count, 1ull);
      if ((int64_t)idx < out_cap) out[idx] = t;
    }
  }
}

}  // namespace

hipError_t launch_bin_reduce(const BinReduceArgs& a, hipStream_t s) {
  if (a.nvec <= 0) return hipSuccess;
  const int64_t Nb = a.N / a.w;
  dim3 grid((unsigned)((Nb + 255) / 256), (unsigned)a.nvec);
  hipLaunchKernelGGL(k_bin_reduce, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_copy_u64(const unsigned long long* src, unsigned long long* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_u64, dim3(1), dim3(64), 0, s, src, dst);
  return hipGetLastError();
}

hipError_t launch_fine_recon(const FineArgs& a, int grid, hipStream_t s) {
  const dim3 g(grid > 0 ? grid : 1), b(FINE_WAVES * 64);
  if (a.w < 1 || a.w > 64 || (a.w & (a.w - 1)) != 0) return hipErrorInvalidValue;
  if (a.z16 == 1) hipLaunchKernelGGL(k_fine_recon<1>, g, b, 0, s, a);
  else if (a.z16 == 2) hipLaunchKernelGGL(k_fine_recon<2>, g, b, 0, s, a);
  else hipLaunchKernelGGL(k_fine_recon<0>, g, b, 0, s, a);
  return hipGetLastError();
}

hipError_t launch_select_final(const TrigRec* in, const unsigned long long* n_in, int64_t cap_in,
                               const float* inv_scale, float thr2_sq, TrigRec* out, int64_t out_cap,
                               unsigned long long* out_count, int32_t* tmpl_count,
                               unsigned long long* tmpl_max, int64_t n_bound, hipStream_t s) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(4096, (n_bound + 255) / 256));
  hipLaunchKernelGGL(k_select_final, dim3((unsigned)blocks), dim3(256), 0, s, in, n_in, cap_in, inv_scale,
                     thr2_sq, out, out_cap, out_count, tmpl_count, tmpl_max);
  return hipGetLastError();
}

}  // namespace rbmf
