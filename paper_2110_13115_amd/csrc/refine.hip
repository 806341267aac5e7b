// Refinement of a trigger's coefficient vector between bank points.
//
// For a trigger (template j, sample n) of a sub-bank basis, the first-stage
// SNR is rho = sum_k C_jk Z_k[n] (Eq. Beta_eqn with C = conj(c)).  Any unit
// vector C in the span of C_j and the coefficient rows of j's nearest bank
// neighbours (largest |<c_j, c_l>|) describes a template between those bank
// points (Sec. II.A: the basis represents every template of the bank's
// span).  Projected gradient ascent of |rho|^2 over that set:
//   g = d|rho|^2 / dC = 2 rho conj(Z[:, n])   (the reconstruction adjoint)
//   C <- C + g / (2 |rho|^2),  C <- P C,  C <- C / |C|
// with P the orthogonal projector onto the span.  With an orthonormal basis
// Q of the span (C = Q^T a), every step is exact in the coordinates a:
// rho = sum_t a_t b_t with b_t = sum_k Q_tk Z_k[n], P g = 2 rho conj(b),
// |C| = |a|.  The span, the coordinates and the steps are FP64.
#include "internal.h"

namespace rbmf {

namespace {

constexpr int RT = 256;           // threads per workgroup
constexpr int KPT = 8;            // coefficients per thread: K <= RT * KPT

__device__ __forceinline__ double2 dmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 dcmul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Sum over the workgroup (every thread receives it); red holds RT / 64 entries.
__device__ double2 block_sum(double2 v, double2* red) {
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off);
    v.y += __shfl_xor(v.y, off);
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();                         // red may still be read by a previous call
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double2 s = red[0];
  for (int i = 1; i < RT / 64; ++i) {
    s.x += red[i].x;
    s.y += red[i].y;
  }
  return s;
}

// |<c_j, c_l>| = |sum_k conj(C_jk) C_lk| for every template l of the basis and
// the trigger rows of a tile of TT triggers: one wave per template at a time,
// lanes over k; the tile's rows in LDS.
__global__ __launch_bounds__(RT) void k_overlaps(const float2* __restrict__ C, int T, int K,
                                                 const int32_t* __restrict__ rows, int n, int TT,
                                                 double* __restrict__ ov) {
  extern __shared__ float2 crow[];         // TT x K
  const int i0 = blockIdx.y * TT;
  const int tt = min(TT, n - i0);
  for (int e = threadIdx.x; e < tt * K; e += RT) crow[e] = C[(int64_t)rows[i0 + e / K] * K + e % K];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l_end = min(T, (int)(blockIdx.x + 1) * 64);
  for (int l = blockIdx.x * 64 + wave; l < l_end; l += RT / 64) {
    const float2* cl = C + (int64_t)l * K;
    for (int t = 0; t < tt; ++t) {
      double re = 0.0, im = 0.0;
      for (int k = lane; k < K; k += 64) {
        const float2 a = crow[t * K + k], b = cl[k];
        re += (double)a.x * b.x + (double)a.y * b.y;
        im += (double)a.x * b.y - (double)a.y * b.x;
      }
      for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_xor(re, off);
        im += __shfl_xor(im, off);
      }
      if (lane == 0) ov[(int64_t)(i0 + t) * T + l] = sqrt(re * re + im * im);
    }
  }
}

struct RefineArgs {
  const float* z;            // FP32 planar Z [2K][N], four-step positions
  int64_t N;
  int N1, N2;
  int K, T, t0;              // rank, templates of the basis, global index of its first template
  const float2* C;           // T x K, C = conj(c)
  const int32_t* rows;       // local template of each trigger
  const int32_t* samp;       // sample of each trigger
  const double* ov;          // n x T overlaps (k_overlaps)
  int m;                     // neighbours
  int iters;
  double2* Q;                // scratch: n x (m + 1) x K
  float2* c_out;             // n x K refined coefficient rows
  int32_t* nbr_out;          // n x m global template indices, or NULL
  float* p_out;              // n x 2: |rho|^2 of the trigger's own row, after refinement, or NULL
};

// One workgroup per trigger.
__global__ __launch_bounds__(RT) void k_refine(RefineArgs a) {
  __shared__ double2 red[RT / 64];
  __shared__ int taken[33];
  __shared__ double2 coord[33], bq[33];
  __shared__ int rank_s;
  __shared__ double best_v[RT / 64];
  __shared__ int best_i[RT / 64];
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  const int K = a.K, T = a.T, m = a.m, r_max = m + 1;
  const int j = a.rows[i];
  const int64_t n = a.samp[i];
  const int64_t q = (n % a.N2) * a.N1 + n / a.N2;     // n = n2 + N2 n1  ->  q = n2 N1 + n1
  double2 z[KPT];
#pragma unroll
  for (int u = 0; u < KPT; ++u) {
    const int k = tid + u * RT;
    z[u] = k < K ? make_double2(a.z[(2 * (int64_t)k) * a.N + q], a.z[(2 * (int64_t)k + 1) * a.N + q])
                 : make_double2(0.0, 0.0);
  }
  // ---- neighbours: m rounds of a workgroup argmax (larger overlap, then lower index)
  if (tid == 0) taken[0] = j;
  __syncthreads();
  const double* ovr = a.ov + (int64_t)i * T;
  for (int s = 0; s < m; ++s) {
    double bv = -1.0;
    int bi = 0x7fffffff;
    for (int l = tid; l < T; l += RT) {
      bool skip = false;
      for (int t = 0; t <= s; ++t) skip |= taken[t] == l;
      const double v = ovr[l];
      if (!skip && (v > bv || (v == bv && l < bi))) {
        bv = v;
        bi = l;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov2 = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      if (ov2 > bv || (ov2 == bv && oi < bi)) {
        bv = ov2;
        bi = oi;
      }
    }
    if ((tid & 63) == 0) {
      best_v[tid >> 6] = bv;
      best_i[tid >> 6] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      for (int w = 1; w < RT / 64; ++w)
        if (best_v[w] > bv || (best_v[w] == bv && best_i[w] < bi)) {
          bv = best_v[w];
          bi = best_i[w];
        }
      if (bi < 0 || bi >= T) bi = j;   // no candidate (non-finite overlaps): repeat j, dropped as dependent
      taken[s + 1] = bi;
      if (a.nbr_out) a.nbr_out[(int64_t)i * m + s] = a.t0 + bi;
    }
    __syncthreads();
  }
  // ---- orthonormal basis of the span: modified Gram-Schmidt, two passes,
  // dependent vectors dropped
  double2* Qi = a.Q + (int64_t)i * r_max * K;
  if (tid == 0) rank_s = 0;
  __syncthreads();
  double2 cj[KPT];
  for (int s = 0; s < r_max; ++s) {
    const float2* src = a.C + (int64_t)taken[s] * K;
    double2 x[KPT];
    double nrm0 = 0.0;
#pragma unroll
    for (int u = 0; u < KPT; ++u) {
      const int k = tid + u * RT;
      const float2 c = k < K ? src[k] : make_float2(0.f, 0.f);
      x[u] = make_double2(c.x, c.y);
      nrm0 += x[u].x * x[u].x + x[u].y * x[u].y;
      if (s == 0) cj[u] = x[u];
    }
    nrm0 = block_sum(make_double2(nrm0, 0.0), red).x;
    const int r = rank_s;
    for (int pass = 0; pass < 2; ++pass)
      for (int t = 0; t < r; ++t) {
        double2 part = make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < KPT; ++u) {
          const int k = tid + u * RT;
          if (k < K) {
            const double2 qv = Qi[(int64_t)t * K + k], p = dcmul(qv, x[u]);
            part.x += p.x;
            part.y += p.y;
          }
        }
        const double2 cf = block_sum(part, red);
#pragma unroll
        for (int u = 0; u < KPT; ++u) {
          const int k = tid + u * RT;
          if (k < K) {
            const double2 p = dmul(cf, Qi[(int64_t)t * K + k]);
            x[u].x -= p.x;
            x[u].y -= p.y;
          }
        }
      }
    double nrm = 0.0;
#pragma unroll
    for (int u = 0; u < KPT; ++u) nrm += x[u].x * x[u].x + x[u].y * x[u].y;
    nrm = block_sum(make_double2(nrm, 0.0), red).x;
    if (nrm > 1e-20 * nrm0 && nrm > 0.0) {
      const double inv = 1.0 / sqrt(nrm);
#pragma unroll
      for (int u = 0; u < KPT; ++u) {
        const int k = tid + u * RT;
        if (k < K) Qi[(int64_t)r * K + k] = make_double2(x[u].x * inv, x[u].y * inv);
      }
      __syncthreads();     // Q row r visible to the workgroup before it is read back
      if (tid == 0) rank_s = r + 1;
    }
    __syncthreads();
  }
  const int r = rank_s;
  // ---- span coordinates: b_t = sum_k Q_tk Z_k, a_t = sum_k conj(Q_tk) C_jk, rho0 = sum_k C_jk Z_k
  double2 part = make_double2(0.0, 0.0);
#pragma unroll
  for (int u = 0; u < KPT; ++u) {
    const double2 p = dmul(cj[u], z[u]);
    part.x += p.x;
    part.y += p.y;
  }
  const double2 rho0 = block_sum(part, red);
  for (int t = 0; t < r; ++t) {
    double2 pb = make_double2(0.0, 0.0), pa = make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < KPT; ++u) {
      const int k = tid + u * RT;
      if (k < K) {
        const double2 qv = Qi[(int64_t)t * K + k];
        const double2 x1 = dmul(qv, z[u]), x2 = dcmul(qv, cj[u]);
        pb.x += x1.x;
        pb.y += x1.y;
        pa.x += x2.x;
        pa.y += x2.y;
      }
    }
    const double2 sb = block_sum(pb, red);
    const double2 sa = block_sum(pa, red);
    if (tid == 0) {
      bq[t] = sb;
      coord[t] = sa;
    }
  }
  __syncthreads();
  // ---- the ascent, in the coordinates (one thread: r <= 33 terms per step)
  if (tid == 0) {
    for (int it = 0; it < a.iters; ++it) {
      double2 rho = make_double2(0.0, 0.0);
      for (int t = 0; t < r; ++t) {
        const double2 p = dmul(coord[t], bq[t]);
        rho.x += p.x;
        rho.y += p.y;
      }
      const double p2 = rho.x * rho.x + rho.y * rho.y;
      if (!(p2 > 0.0)) break;
      // a <- a + (P g) / (2 |rho|^2) with P g = 2 rho conj(b)
      double nrm = 0.0;
      for (int t = 0; t < r; ++t) {
        const double2 g = dmul(rho, make_double2(bq[t].x, -bq[t].y));
        coord[t].x += g.x / p2;
        coord[t].y += g.y / p2;
        nrm += coord[t].x * coord[t].x + coord[t].y * coord[t].y;
      }
      const double inv = 1.0 / sqrt(nrm);
      for (int t = 0; t < r; ++t) {
        coord[t].x *= inv;
        coord[t].y *= inv;
      }
    }
    double2 rho = make_double2(0.0, 0.0);
    for (int t = 0; t < r; ++t) {
      const double2 p = dmul(coord[t], bq[t]);
      rho.x += p.x;
      rho.y += p.y;
    }
    if (a.p_out) {
      a.p_out[2 * (int64_t)i] = (float)(rho0.x * rho0.x + rho0.y * rho0.y);
      a.p_out[2 * (int64_t)i + 1] = (float)(rho.x * rho.x + rho.y * rho.y);
    }
  }
  __syncthreads();
  // ---- C = sum_t a_t Q_t
#pragma unroll
  for (int u = 0; u < KPT; ++u) {
    const int k = tid + u * RT;
    if (k < K) {
      double2 c = make_double2(0.0, 0.0);
      for (int t = 0; t < r; ++t) {
        const double2 p = dmul(coord[t], Qi[(int64_t)t * K + k]);
        c.x += p.x;
        c.y += p.y;
      }
      a.c_out[(int64_t)i * K + k] = make_float2((float)c.x, (float)c.y);
    }
  }
}

}  // namespace

int refine_max_rank() { return RT * KPT; }

hipError_t launch_refine(const float* z, int64_t N, int N1, int N2, int K, int T, int t0, const float2* C,
                         const int32_t* rows, const int32_t* samp, int n, int m, int iters, double* ov,
                         double2* Q, float2* c_out, int32_t* nbr_out, float* p_out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int TT = std::max(1, std::min(8, 8192 / K));     // trigger rows per overlap workgroup (<= 64 KB LDS)
  hipLaunchKernelGGL(k_overlaps, dim3((unsigned)((T + 63) / 64), (unsigned)((n + TT - 1) / TT)), dim3(RT),
                     (size_t)TT * K * sizeof(float2), s, C, T, K, rows, n, TT, ov);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  RefineArgs a;
  a.z = z;
  a.N = N;
  a.N1 = N1;
  a.N2 = N2;
  a.K = K;
  a.T = T;
  a.t0 = t0;
  a.C = C;
  a.rows = rows;
  a.samp = samp;
  a.ov = ov;
  a.m = m;
  a.iters = iters;
  a.Q = Q;
  a.c_out = c_out;
  a.nbr_out = nbr_out;
  a.p_out = p_out;
  hipLaunchKernelGGL(k_refine, dim3((unsigned)n), dim3(RT), 0, s, a);
  return hipGetLastError();
}

}  // namespace rbmf
