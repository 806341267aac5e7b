// Sparse exact second stage: for every template j selected by the first stage,
// the exact complex SNR (Eq. IFFT, discretised as in the template method)
//   rho_j[n] = sum_{f in support_j} d[f] conj(w_j[f]) e^{+2 pi i f n / N}
// evaluated only at the samples n where the first stage crossed (direct
// frequency sums instead of a full inverse FFT).  Every final trigger
// (|rho| >= thr2 >= thr1) is a first-stage crossing as long as the first-stage
// reconstruction error stays below thr2 - thr1, so the final trigger set equals
// the template method's.
//
// With workgroup offsets (host-known list), workgroup b takes one group of up
// to SP_M crossings of one template, so a template with many crossings (near
// a loud signal) spreads over as many workgroups as it has groups and no
// workgroup is launched for a group that does not exist.  Without them
// (device-side counts), workgroup (x, y) takes template list[x] and its
// crossing groups y, y + G, y + 2G, ... (G = gridDim.y).  A workgroup streams
// w_j once per group.  A thread owns the bins t, t + 256, ...,
// t + 7 * 256 of each 2048-bin tile (so every load of a wave is contiguous).
// Per crossing n, the eight products x_r = d conj(w) of a thread's bins are
// first summed against a table of the exact offset phases
// e^{2 pi i r 256 n / N}, r < 8 (built once per group in LDS from the
// two-level twiddle table, the same for every thread), and the sum is then
// multiplied by the phase of the thread's first bin of the tile, also taken
// exactly from the table (e = f n mod N): four FMAs per bin and crossing, no
// phase recurrence.
#include "internal.h"

namespace rbmf {

namespace {

constexpr int SP_T = 256;      // threads
constexpr int SP_R = 8;        // consecutive bins per thread and tile
constexpr int SP_M = 8;        // crossings per pass

// Every product and sum of this file is written as an explicit fmaf / mul
// with contraction off, so that each crossing's SNR has the same bits in
// every instantiation of sparse_group (the grouping of crossings depends on
// the order in which the first stage appended them).
#pragma clang fp contract(off)

__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}

// One group of M (>= m) crossings of template j: slots m..M-1 repeat the last
// crossing and are discarded, so the sums are straight-line code across the
// M crossings (the caller instantiates M = m).
template <int M>
__device__ __forceinline__ void sparse_group(const SparseArgs& a, const float2* tlo, const float2* thi,
                                             float2 (*red)[SP_T / 64], float2 (*sp)[SP_R], int j, int c0, int m,
                                             int lo, int hi, const float2* __restrict__ d,
                                             const float2* __restrict__ wj, unsigned long long& best) {
  const int mask = (1 << a.s_lo) - 1;
  const int N = (int)a.N;                       // N <= 2^30
  auto tw = [&](int e) { return cmulf(thi[e >> a.s_lo], tlo[e & mask]); };   // e in [0, N)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int off = a.offsets[j];
  int ns[M], e[M], inc[M];
  float2 acc[M];
  const int f00 = lo + threadIdx.x;
#pragma unroll
  for (int i = 0; i < M; ++i) ns[i] = a.recs[off + c0 + min(i, m - 1)].sample;
  // the phases of the bin offsets r SP_T within a thread's eight bins,
  // e^{2 pi i r SP_T n / N}, one table per crossing in LDS (the same for
  // every thread), exact from the twiddle table
  __syncthreads();   // (the previous group's readers are done)
  if ((int)threadIdx.x < M * SP_R) {
    const int i = threadIdx.x / SP_R, r = threadIdx.x % SP_R;
    sp[i][r] = tw((int)(((int64_t)(r * SP_T) * ns[i]) % N));
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < M; ++i) {
    acc[i] = make_float2(0.f, 0.f);
    e[i] = (int)(((int64_t)f00 * ns[i]) % N);                   // exponent of this thread's first bin
    inc[i] = (int)(((int64_t)(SP_T * SP_R) * ns[i]) % N);       // advance per tile
  }
  // Bins past hi are read at hi (in bounds) and masked to zero; the next
  // tile's operands are loaded while this tile's sums run.
  float2 dn[SP_R], wn[SP_R];
  auto fetch = [&](int f0) {
#pragma unroll
    for (int r = 0; r < SP_R; ++r) {
      const int f = min(f0 + r * SP_T, hi);
      dn[r] = d[f];
      wn[r] = wj[f];
    }
  };
  fetch(f00);
  for (int f0 = f00; f0 <= hi; f0 += SP_T * SP_R) {
    float2 x[SP_R];
#pragma unroll
    for (int r = 0; r < SP_R; ++r) {
      const float2 dv = dn[r], wv = wn[r];
      const float mk = (f0 + r * SP_T <= hi) ? 1.f : 0.f;
      x[r] = make_float2(mk * fmaf(dv.x, wv.x, dv.y * wv.y), mk * fmaf(dv.y, wv.x, -(dv.x * wv.y)));   // d conj(w)
    }
    fetch(f0 + SP_T * SP_R);
#pragma unroll
    for (int i = 0; i < M; ++i) {
      // y = sum_r x_r e^{2 pi i r SP_T n / N}, then acc += y e^{2 pi i f0 n / N}
      float2 y = make_float2(0.f, 0.f);
#pragma unroll
      for (int r = 0; r < SP_R; ++r) {
        const float2 sv = sp[i][r];
        y.x = fmaf(-x[r].y, sv.y, fmaf(x[r].x, sv.x, y.x));
        y.y = fmaf(x[r].y, sv.x, fmaf(x[r].x, sv.y, y.y));
      }
      const float2 w = tw(e[i]);
      acc[i].x = fmaf(-y.y, w.y, fmaf(y.x, w.x, acc[i].x));
      acc[i].y = fmaf(y.y, w.x, fmaf(y.x, w.y, acc[i].y));
      e[i] += inc[i];
      if (e[i] >= N) e[i] -= N;
    }
  }
  // workgroup reduction of the accumulators
#pragma unroll
  for (int i = 0; i < M; ++i) {
    float re = acc[i].x, im = acc[i].y;
    for (int o = 32; o > 0; o >>= 1) {
      re += __shfl_xor(re, o);
      im += __shfl_xor(im, o);
    }
    if (lane == 0) red[i][wave] = make_float2(re, im);
  }
  __syncthreads();
  if ((int)threadIdx.x < m) {
    const int i = threadIdx.x;
    float re = 0.f, im = 0.f;
    for (int w = 0; w < SP_T / 64; ++w) {
      re += red[i][w].x;
      im += red[i][w].y;
    }
    const float p = fmaf(re, re, im * im);
    const int n = a.recs[off + c0 + i].sample;
    const unsigned long long key =
        ((unsigned long long)__float_as_uint(p) << 32) | (unsigned long long)(0xffffffffu - (uint32_t)n);
    best = key > best ? key : best;
    if (p >= a.thr2) {
      const unsigned long long idx = atomicAdd(a.out_count, 1ull);
      atomicAdd(&a.tmpl_count[j], 1);
      if ((int64_t)idx < a.out_cap) {
        TrigRec t;
        t.tmpl = j;
        t.sample = n;
        t.re = re;
        t.im = im;
        a.out[idx] = t;
      }
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(SP_T) void k_sparse_exact(SparseArgs a) {
  __shared__ float2 tlo[2048];
  __shared__ float2 thi[1024];
  __shared__ float2 red[SP_M][SP_T / 64];
  __shared__ float2 sp[SP_M][SP_R];
  if (a.d_count != nullptr && (int)blockIdx.x >= *a.d_count) return;
  if (a.n1_dev != nullptr && *a.n1_dev > a.n1_cap) return;
  int j, cnt, cfirst, cstep;
  if (a.goff != nullptr) {
    // one group per workgroup: list entry i with goff[i] <= b < goff[i + 1]
    const int b = (int)blockIdx.x;
    if (b >= a.goff[a.nlist]) return;   // (the grid is an upper bound)
    int lo = 0, hi = a.nlist - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.goff[mid] <= b) lo = mid;
      else hi = mid - 1;
    }
    j = a.list[lo];
    cnt = a.counts[j];
    cfirst = (b - a.goff[lo]) * SP_M;
    cstep = cnt;                        // a single group
  } else {
    j = a.list[blockIdx.x];
    cnt = a.counts[j];
    if ((int)blockIdx.y * SP_M >= cnt) return;   // no group of this template for this workgroup
    cfirst = blockIdx.y * SP_M;
    cstep = gridDim.y * SP_M;
  }
  const int nlo = 1 << a.s_lo, nhi = (int)(a.N >> a.s_lo);
  // table copies: every load of a thread (clamped in bounds) issued before its LDS stores
  {
    constexpr int PL = 2048 / SP_T, PH = 1024 / SP_T;
    float2 vl[PL], vh[PH];
#pragma unroll
    for (int i = 0; i < PL; ++i) vl[i] = a.tlo[min((int)threadIdx.x + i * SP_T, nlo - 1)];
#pragma unroll
    for (int i = 0; i < PH; ++i) vh[i] = a.thi[min((int)threadIdx.x + i * SP_T, nhi - 1)];
#pragma unroll
    for (int i = 0; i < PL; ++i)
      if ((int)threadIdx.x + i * SP_T < nlo) tlo[threadIdx.x + i * SP_T] = vl[i];
#pragma unroll
    for (int i = 0; i < PH; ++i)
      if ((int)threadIdx.x + i * SP_T < nhi) thi[threadIdx.x + i * SP_T] = vh[i];
  }
  __syncthreads();
  const int lo = a.sup_lo[j], hi = a.sup_hi[j];
  const float2* __restrict__ wj = a.tmpl + (int64_t)j * a.nbs - a.kb;   // indexed by absolute bin
  const float2* __restrict__ d = a.d - a.kb;
  unsigned long long best = 0ull;
  for (int c0 = cfirst; c0 < cnt; c0 += cstep) {
    const int m = min(SP_M, cnt - c0);            // uniform over the workgroup
    switch (m) {   // straight-line sums over exactly m crossings
      case 1: sparse_group<1>(a, tlo, thi, red, sp, j, c0, m, lo, hi, d, wj, best); break;
      case 2: sparse_group<2>(a, tlo, thi, red, sp, j, c0, m, lo, hi, d, wj, best); break;
      case 3: sparse_group<3>(a, tlo, thi, red, sp, j, c0, m, lo, hi, d, wj, best); break;
      case 4: sparse_group<4>(a, tlo, thi, red, sp, j, c0, m, lo, hi, d, wj, best); break;
      case 5: sparse_group<5>(a, tlo, thi, red, sp, j, c0, m, lo, hi, d, wj, best); break;
      case 6: sparse_group<6>(a, tlo, thi, red, sp, j, c0, m, lo, hi, d, wj, best); break;
      case 7: sparse_group<7>(a, tlo, thi, red, sp, j, c0, m, lo, hi, d, wj, best); break;
      default: sparse_group<8>(a, tlo, thi, red, sp, j, c0, m, lo, hi, d, wj, best); break;
    }
  }
  if (a.tmpl_max != nullptr && threadIdx.x < SP_M && best != 0ull) atomicMax(&a.tmpl_max[j], best);
}

}  // namespace

hipError_t launch_sparse_exact(const SparseArgs& a, int grid, int groups, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  groups = a.goff != nullptr ? 1 : (groups < 1 ? 1 : (groups > 64 ? 64 : groups));
  hipLaunchKernelGGL(k_sparse_exact, dim3(grid, groups), dim3(SP_T), 0, s, a);
  return hipGetLastError();
}

int sparse_crossings_per_group() { return SP_M; }

}  // namespace rbmf
