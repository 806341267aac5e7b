// Batched LDS-staged radix FFT passes for gfx950.
//
// An N-point transform is split N = N1 * N2 (four-step).  Pass 1 runs
// N2-point FFTs down adjacent columns (16 for FP32, 8 for FP64, so every
// global access is a 128-byte row segment), multiplies by the inter-pass
// twiddle and writes the [N2][N1] intermediate.  Pass 2 runs N1-point FFTs along rows.
// The result stays in the four-step (transposed) order: position
// q = n2 * N1 + n1 holds index n = n2 + N2 * n1; consumers that need natural
// order map q -> n themselves.
//
// Inside a workgroup each FFT is a self-sorting mixed-radix Stockham
// factorisation (radix 8/16 butterflies in registers, LDS exchanges between
// stages).  The first stage reads global memory directly and the last stage
// writes global memory directly, so an FFT of length L with s stages costs
// s - 1 LDS round trips.
//
// Fused prologues (pass 1):  IN_CORR  X[f] = d[f] conj(src_v[f]) on the
//   vector's support (Sec. III.C: filter the whitened data with every basis
//   vector / template); negative frequencies are zero, so only the first half
//   of every column is read.  IN_FOLD: the same product folded onto
//   M = N / w bins with the geometric-sum weights of Sec. III.D (Eq.
//   avg_fft2), X~[f'] = (1/w) sum_l X[l M + f'] G[l M + f'], whose M-point
//   inverse transform is the bin mean of the template's SNR series.
//   IN_REAL: the real strain.  IN_DENSE: complex.
// The batched passes run in FP32.  The one forward transform of the strain
// runs in FP64: raw strain carries out-of-band (low-frequency) power many
// orders of magnitude above the band, and FP32 rounding relative to the total
// energy would swamp the whitened in-band bins.
// Fused epilogues (pass 2): planar FP32 / 16-bit Z for the reconstruction
//   GEMM, threshold + trigger append + per-template max (template method,
//   Eq. IFFT and the trigger definition of Sec. II), whitened band spectrum
//   of the strain, natural-order dumps.
#include "internal.h"

#include <hip/hip_fp16.h>

namespace rbmf {

namespace {

constexpr int NT = 256;      // threads per workgroup
constexpr int ROW_ELEMS = 4096;  // elements per pass-2 workgroup

// Complex helpers generic over float2 / double2.
template <class V> struct Re;
template <> struct Re<float2> { using T = float; };
template <> struct Re<double2> { using T = double; };
template <class V>
__device__ __forceinline__ V mk(typename Re<V>::T x, typename Re<V>::T y) {
  V v;
  v.x = x;
  v.y = y;
  return v;
}
template <class V>
__device__ __forceinline__ V cadd(V a, V b) { return mk<V>(a.x + b.x, a.y + b.y); }
template <class V>
__device__ __forceinline__ V csub(V a, V b) { return mk<V>(a.x - b.x, a.y - b.y); }
template <class V>
__device__ __forceinline__ V cmul(V a, V b) { return mk<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// a * conj(b)
template <class V>
__device__ __forceinline__ V cmulc(V a, V b) { return mk<V>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }
template <int S, class V>
__device__ __forceinline__ V signed_tw(V w) { return S > 0 ? w : mk<V>(w.x, -w.y); }

// x * e^{S 2 pi i k / R} for 0 <= k < R/2, R <= 16 (k is a compile-time
// constant after unrolling, so the switch folds away).
template <int R, int S, class V>
__device__ __forceinline__ V rot(V x, int k) {
  using T = typename Re<V>::T;
  const int k16 = k * (16 / R);
  if (k16 == 0) return x;
  if (k16 == 4) return S > 0 ? mk<V>(-x.y, x.x) : mk<V>(x.y, -x.x);
  const T C1 = (T)0.92387953251128674, S1 = (T)0.38268343236508978, H2 = (T)0.70710678118654752;
  T c = 1, s = 0;
  switch (k16) {
    case 1: c = C1; s = S1; break;
    case 2: c = H2; s = H2; break;
    case 3: c = S1; s = C1; break;
    case 5: c = -S1; s = C1; break;
    case 6: c = -H2; s = H2; break;
    case 7: c = -C1; s = S1; break;
    default: break;
  }
  if (S < 0) s = -s;
  return mk<V>(x.x * c - x.y * s, x.x * s + x.y * c);
}

// In-register DFT of size R (radix-2 decimation in time, recursively).
template <int R, int S>
struct Dft {
  template <class V>
  static __device__ __forceinline__ void run(V* v) {
    constexpr int H = R / 2;
    V e[H], o[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    Dft<H, S>::run(e);
    Dft<H, S>::run(o);
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const V t = rot<R, S>(o[k], k);
      v[k] = cadd(e[k], t);
      v[k + H] = csub(e[k], t);
    }
  }
};
template <int S>
struct Dft<1, S> {
  template <class V>
  static __device__ __forceinline__ void run(V*) {}
};

// Powers w^r, r = 0..R-1 (R <= 16), from the table entries w^1, w^2, w^4, w^8
// and at most three products each (a few ulp), instead of R-1 table gathers.
// base(p) must return the table entry for exponent multiplier p in {1,2,4,8}.
template <int R, class V, class Base>
__device__ __forceinline__ void powers(V* w, Base&& base) {
  w[0] = mk<V>(1, 0);
  if (R > 1) w[1] = base(1);
  if (R > 2) w[2] = base(2);
  if (R > 4) w[4] = base(4);
  if (R > 8) w[8] = base(8);
#pragma unroll
  for (int r = 3; r < R; ++r) {
    if (r == 4 || r == 8) continue;
    const int hb = (r >= 8) ? 8 : (r >= 4 ? 4 : 2);   // highest power of two <= r
    w[r] = cmul(w[hb], w[r - hb]);
  }
}

// Stage twiddles: input r of a butterfly with k = j mod Ns gets
// e^{S 2 pi i r k / (Ns R)} = pyr[Ns R + r k].  The table entries for
// r = 1, 2, 4, 8 (the bases of `powers`) are gathered first (stage_tw_load),
// ahead of the LDS traffic and barriers, and applied later (stage_tw_apply).
template <int R> struct NBase { static constexpr int value = R > 8 ? 4 : (R > 4 ? 3 : (R > 2 ? 2 : 1)); };
template <int R, int Ns, int S, class V>
__device__ __forceinline__ void stage_tw_load(V (&b)[NBase<R>::value], int k, const V* __restrict__ pyr) {
  if (Ns == 1) return;
#pragma unroll
  for (int q = 0; q < NBase<R>::value; ++q) b[q] = signed_tw<S>(pyr[Ns * R + (1 << q) * k]);
}
template <int R, int Ns, class V>
__device__ __forceinline__ void stage_tw_apply(V* v, const V (&b)[NBase<R>::value]) {
  if (Ns == 1) return;
  V w[R];
  powers<R>(w, [&](int p) { return b[p == 1 ? 0 : (p == 2 ? 1 : (p == 4 ? 2 : 3))]; });
#pragma unroll
  for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r]);
}

// ------------------------------------------------------------------ layouts
// Column layout (pass 1): C FFTs, element (c, pos) at pos * C + c.
template <int L, int C>
struct ColLayout {
  static constexpr int NF = C;
  static constexpr int SIZE = L * C;
  template <int R>
  static __device__ __forceinline__ void split(int b, int& f, int& j) {
    f = b % C;
    j = b / C;
  }
  static __device__ __forceinline__ int addr(int f, int pos) { return pos * C + f; }
};
// columns per pass-1 workgroup: one 128-byte row segment
template <class V> struct Cols { static constexpr int value = 128 / sizeof(V); };
// ... of the stored intermediate: 32 columns of FP16 pairs for IN_CORR_H
// (while the L x 32 complex64 LDS tile fits), else one segment of V
template <class V, int L, int IN>
struct Cols1 {
  static constexpr int value = (IN == IN_CORR_H && L <= 256) ? 32 : Cols<V>::value;
};
// Row layout (pass 2): F FFTs, element (f, pos) at f * (L + L/8) + pos + pos/8
// (one pad slot every 8 elements keeps the radix-8/16 scatter conflict-free).
template <int L>
struct RowLayout {
  static constexpr int NF = (ROW_ELEMS / L) > 0 ? (ROW_ELEMS / L) : 1;
  static constexpr int LP = L + L / 8;
  static constexpr int SIZE = NF * LP;
  template <int R>
  static __device__ __forceinline__ void split(int b, int& f, int& j) {
    f = b / (L / R);
    j = b % (L / R);
  }
  static __device__ __forceinline__ int addr(int f, int pos) { return f * LP + pos + (pos >> 3); }
};

// One LDS-to-LDS Stockham stage (radix R, Ns already-combined length).
template <class Lay, int L, int R, int Ns, int S, class V>
__device__ __forceinline__ void lds_stage(V* lds, const V* __restrict__ pyr, int tid) {
  constexpr int NB = Lay::NF * L / R;
  constexpr int PER = (NB + NT - 1) / NT;
  V v[PER][R];
  V tb[PER][NBase<R>::value];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = tid + i * NT;
    if (NB % NT == 0 || b < NB) {   // (the test folds away when NT divides NB)
      int f, j;
      Lay::template split<R>(b, f, j);
      stage_tw_load<R, Ns, S>(tb[i], j % Ns, pyr);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = lds[Lay::addr(f, j + r * (L / R))];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = tid + i * NT;
    if (NB % NT == 0 || b < NB) {   // (the test folds away when NT divides NB)
      int f, j;
      Lay::template split<R>(b, f, j);
      const int k = j % Ns;
      stage_tw_apply<R, Ns>(v[i], tb[i]);
      Dft<R, S>::run(v[i]);
      const int idxD = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int m = 0; m < R; ++m) lds[Lay::addr(f, idxD + m * Ns)] = v[i][m];
    }
  }
  __syncthreads();
}

// Reads the R inputs of the final stage's butterflies and applies the stage
// twiddles and DFT; the caller stores.  Output m of butterfly j is position
// j + m * (L / R); the last argument of store is the output's index among the
// calling thread's outputs (i * R + m, a compile-time constant once unrolled).
template <class Lay, int L, int R, int S, class V, class Store>
__device__ __forceinline__ void final_stage(const V* lds, const V* __restrict__ pyr, int tid,
                                            Store&& store) {
  constexpr int Ns = L / R;
  constexpr int NB = Lay::NF * L / R;
  constexpr int PER = (NB + NT - 1) / NT;
  V tb[PER][NBase<R>::value];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = tid + i * NT;
    if (NB % NT == 0 || b < NB) {
      int f, j;
      Lay::template split<R>(b, f, j);
      stage_tw_load<R, Ns, S>(tb[i], j, pyr);
    }
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = tid + i * NT;
    if (NB % NT == 0 || b < NB) {   // (the test folds away when NT divides NB)
      int f, j;
      Lay::template split<R>(b, f, j);
      V v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = lds[Lay::addr(f, j + r * (L / R))];
      stage_tw_apply<R, Ns>(v, tb[i]);
      Dft<R, S>::run(v);
#pragma unroll
      for (int m = 0; m < R; ++m) store(f, j + m * Ns, v[m], i * R + m);
    }
  }
}

__device__ __forceinline__ int resolve_vec(const PassArgs& a, int bv, bool& skip) {
  skip = false;
  if (a.d_count != nullptr && a.vec_base + bv >= *a.d_count) {
    skip = true;
    return 0;
  }
  return a.vec_list ? a.vec_list[a.vec_base + bv] : a.vec_base + bv;
}

// Pointers of the FP32 (batched) or FP64 (strain spectrum) variant.
template <class V> struct PassPtr;
template <> struct PassPtr<float2> {
  static __device__ __forceinline__ const float2* pyr(const PassArgs& a) { return a.tw.pyr; }
  static __device__ __forceinline__ const float2* tlo(const PassArgs& a) { return a.tw.tlo; }
  static __device__ __forceinline__ const float2* thi(const PassArgs& a) { return a.tw.thi; }
  static __device__ __forceinline__ float2* work(const PassArgs& a) { return a.work; }
};
template <> struct PassPtr<double2> {
  static __device__ __forceinline__ const double2* pyr(const PassArgs& a) { return a.tw64.pyr; }
  static __device__ __forceinline__ const double2* tlo(const PassArgs& a) { return a.tw64.tlo; }
  static __device__ __forceinline__ const double2* thi(const PassArgs& a) { return a.tw64.thi; }
  static __device__ __forceinline__ double2* work(const PassArgs& a) { return a.work64; }
};

// FP16 (Re, Im) pair in one word (Re in the low half), rounded to nearest even.
__device__ __forceinline__ uint32_t pack_f16x2(float re, float im) {
  const __half hr = __float2half_rn(re), hi = __float2half_rn(im);
  return (uint32_t)__builtin_bit_cast(uint16_t, hr) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
}
__device__ __forceinline__ float2 unpack_f16x2(uint32_t w) {
  return make_float2(__half2float(__builtin_bit_cast(__half, (uint16_t)(w & 0xffffu))),
                     __half2float(__builtin_bit_cast(__half, (uint16_t)(w >> 16))));
}

// ------------------------------------------------------------------ pass 1
template <class V, int L, int R1, int R2, int R3, int IN, int S>
__global__ __launch_bounds__(NT) void k_pass1(PassArgs a) {
  using T = typename Re<V>::T;
  constexpr int C = Cols1<V, L, IN>::value;
  using Lay = ColLayout<L, C>;
  __shared__ V lds[Lay::SIZE];
  const int tid = threadIdx.x;
  bool skip;
  const int v = resolve_vec(a, blockIdx.y, skip);
  if (skip) return;
  const int bv = blockIdx.y;
  const int N1 = a.g.N1;
  const int f1_0 = blockIdx.x * C;
  const V* __restrict__ pyr = PassPtr<V>::pyr(a);

  constexpr bool CORR = (IN == IN_CORR || IN == IN_CORR_H);
  int lo = a.band_lo, hi = a.band_hi;
  if ((CORR || IN == IN_FOLD) && a.sup_lo != nullptr) {
    lo = a.sup_lo[v];
    hi = a.sup_hi[v];
  }
  // ---- stage 1: global -> registers -> LDS (Ns = 1, no twiddles)
  {
    constexpr int NB = C * L / R1;
    constexpr int PER = (NB + NT - 1) / NT;
    constexpr bool HALF = CORR;   // one-sided input: rows >= L/2 are zero
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int b = tid + i * NT;
      if (NB % NT == 0 || b < NB) {   // (the test folds away when NT divides NB)
        const int c = b % C, j = b / C;
        const int f1 = f1_0 + c;
        V x[R1];
#pragma unroll
        for (int r = 0; r < R1; ++r) {
          x[r] = mk<V>(0, 0);
          if (HALF && r >= R1 / 2) continue;
          const int f2 = j + r * (L / R1);
          const int64_t f = (int64_t)f1 + (int64_t)N1 * f2;
          if (CORR) {
            // read at the bin clamped into the support [lo, hi] (always in
            // bounds, no branch around the loads) and mask bins outside it
            const int64_t fc = f < lo ? lo : (f > hi ? hi : f);
            const float2 dv = a.d[fc - a.kb];
            const float2 pv = a.src[(int64_t)v * a.nbs + (fc - a.kb)];
            const float m = (f == fc) ? 1.f : 0.f;
            x[r] = mk<V>(m * (dv.x * pv.x + dv.y * pv.y), m * (dv.y * pv.x - dv.x * pv.y));
          } else if (IN == IN_FOLD) {
            // f < M; the one-sided spectrum is zero from N/2 = (w/2) M on
            float xr = 0.f, xi = 0.f;
            for (int l = 0; l < a.fold_half; ++l) {
              const int64_t F = f + (int64_t)l * a.g.N;
              const int64_t fc = F < lo ? lo : (F > hi ? hi : F);
              const float2 dv = a.d[fc - a.kb];
              const float2 pv = a.src[(int64_t)v * a.nbs + (fc - a.kb)];
              const float2 gv = a.gfold[F];
              const float m = (F == fc) ? 1.f : 0.f;
              const float cr = m * (dv.x * pv.x + dv.y * pv.y), ci = m * (dv.y * pv.x - dv.x * pv.y);
              xr += cr * gv.x - ci * gv.y;
              xi += cr * gv.y + ci * gv.x;
            }
            x[r] = mk<V>((T)(xr * a.fold_inv), (T)(xi * a.fold_inv));
          } else if (IN == IN_REAL) {
            x[r] = mk<V>((T)a.real_in[f], 0);
          } else {
            const float2 in = a.src[(int64_t)v * a.g.N + f];
            x[r] = mk<V>(in.x, in.y);
          }
        }
        Dft<R1, S>::run(x);
#pragma unroll
        for (int m = 0; m < R1; ++m) lds[Lay::addr(c, j * R1 + m)] = x[m];
      }
    }
  }
  __syncthreads();
  if (R3 > 1) lds_stage<Lay, L, R2, R1, S>(lds, pyr, tid);
  constexpr int RL = (R3 > 1) ? R3 : R2;
  // ---- final stage: LDS -> inter-pass twiddle -> global [n2][N1]
  const int s_lo = a.g.s_lo;
  const int mask = (1 << s_lo) - 1;
  const V* __restrict__ thi = PassPtr<V>::thi(a);
  const V* __restrict__ tlo = PassPtr<V>::tlo(a);
  V* __restrict__ outv = PassPtr<V>::work(a) + (int64_t)bv * a.g.N;
  // IN_CORR_H: FP16 (Re, Im) pairs, element for element at the same index
  uint32_t* __restrict__ outh = reinterpret_cast<uint32_t*>(a.work) + (int64_t)bv * a.g.N;
  const float hs = (IN == IN_CORR_H) ? a.hscale[0] : 1.f;
  {
    // outputs n2 = j + m Ns of column f1 get w^{f1 n2} = w^{f1 j} (w^{f1 Ns})^m
    constexpr int Ns = L / RL;
    constexpr int NB = Lay::NF * L / RL;
    constexpr int PER = (NB + NT - 1) / NT;
    // table gathers of PC butterflies are issued together, then the butterflies run
    constexpr int PC = PER < 4 ? PER : 4;
    static_assert(PER % PC == 0, "butterflies per thread");
#pragma unroll
    for (int i0 = 0; i0 < PER; i0 += PC) {
      V tb[PC][NBase<RL>::value], bh[PC], bl[PC], sh[PC], sl[PC];
#pragma unroll
      for (int u = 0; u < PC; ++u) {
        const int b = tid + (i0 + u) * NT;
        if (NB % NT == 0 || b < NB) {
          int c, j;
          Lay::template split<RL>(b, c, j);
          stage_tw_load<RL, Ns, S>(tb[u], j, pyr);
          const int64_t e1 = (int64_t)(f1_0 + c) * j, e2 = (int64_t)(f1_0 + c) * Ns;
          bh[u] = thi[e1 >> s_lo];
          bl[u] = tlo[e1 & mask];
          sh[u] = thi[e2 >> s_lo];
          sl[u] = tlo[e2 & mask];
        }
      }
#pragma unroll
      for (int u = 0; u < PC; ++u) {
      const int b = tid + (i0 + u) * NT;
      if (NB % NT == 0 || b < NB) {   // (the test folds away when NT divides NB)
        int c, j;
        Lay::template split<RL>(b, c, j);
        V v[RL];
#pragma unroll
        for (int r = 0; r < RL; ++r) v[r] = lds[Lay::addr(c, j + r * Ns)];
        stage_tw_apply<RL, Ns>(v, tb[u]);
        Dft<RL, S>::run(v);
        const int f1 = f1_0 + c;
        const V base = signed_tw<S>(cmul(bh[u], bl[u]));
        const V step = signed_tw<S>(cmul(sh[u], sl[u]));
        V sp[RL];
        powers<RL>(sp, [&](int p) {
          V s = step;
          for (int q = 1; q < p; q <<= 1) s = cmul(s, s);
          return s;
        });
#pragma unroll
        for (int m = 0; m < RL; ++m) {
          const V y = cmul(v[m], cmul(base, sp[m]));
          if constexpr (IN == IN_CORR_H)
            outh[(int64_t)(j + m * Ns) * N1 + f1] = pack_f16x2((float)y.x * hs, (float)y.y * hs);
          else
            outv[(int64_t)(j + m * Ns) * N1 + f1] = y;
        }
      }
      }
    }
  }
}

// ------------------------------------------------------------------ pass 2
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ uint16_t f32_to_f16_rne(float x) {
  __half h = __float2half_rn(x);
  return *reinterpret_cast<uint16_t*>(&h);
}

template <class V, int L, int R1, int R2, int R3, int OUT, int S>
__global__ __launch_bounds__(NT) void k_pass2(PassArgs a) {
  using Lay = RowLayout<L>;
  constexpr int F = Lay::NF;
  __shared__ V lds[Lay::SIZE];
  const int tid = threadIdx.x;
  bool skip;
  const int v = resolve_vec(a, blockIdx.y, skip);
  if (skip) return;
  const int bv = blockIdx.y;
  const int N2 = a.g.N2;
  const int row0 = blockIdx.x * F;
  const V* __restrict__ pyr = PassPtr<V>::pyr(a);
  const V* __restrict__ inv = PassPtr<V>::work(a) + (int64_t)bv * a.g.N;
  // ---- stage 1: global rows -> LDS
  {
    constexpr int NB = F * L / R1;
    constexpr int PER = (NB + NT - 1) / NT;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int b = tid + i * NT;
      if (NB % NT == 0 || b < NB) {   // (the test folds away when NT divides NB)
        int f, j;
        Lay::template split<R1>(b, f, j);
        V x[R1];
        if constexpr (OUT == OUT_Z16_H || OUT == OUT_ZBIN_H) {
          const uint32_t* rowh =
              reinterpret_cast<const uint32_t*>(a.work) + (int64_t)bv * a.g.N + (int64_t)(row0 + f) * L;
#pragma unroll
          for (int r = 0; r < R1; ++r) x[r] = unpack_f16x2(rowh[j + r * (L / R1)]);
        } else {
          const V* rowp = inv + (int64_t)(row0 + f) * L;
#pragma unroll
          for (int r = 0; r < R1; ++r) x[r] = rowp[j + r * (L / R1)];
        }
        Dft<R1, S>::run(x);
#pragma unroll
        for (int m = 0; m < R1; ++m) lds[Lay::addr(f, j * R1 + m)] = x[m];
      }
    }
  }
  __syncthreads();
  if (R3 > 1) lds_stage<Lay, L, R2, R1, S>(lds, pyr, tid);
  constexpr int RL = (R3 > 1) ? R3 : R2;
  const int64_t N = a.g.N;

  if constexpr (OUT == OUT_Z32) {
    float* __restrict__ zr = a.zout + (int64_t)(2 * v) * N;
    float* __restrict__ zi = zr + N;
    final_stage<Lay, L, RL, S>(lds, pyr, tid, [&](int f, int n1, V val, int) {
      const int64_t q = (int64_t)(row0 + f) * L + n1;
      zr[q] = val.x;
      zi[q] = val.y;
    });
  } else if constexpr (OUT == OUT_Z16 || OUT == OUT_Z16_H) {
    uint16_t* __restrict__ zr = reinterpret_cast<uint16_t*>(a.zout) + (int64_t)(2 * v) * N;
    uint16_t* __restrict__ zi = zr + N;
    const float sc = OUT == OUT_Z16_H ? a.zscale * a.hscale[1] : a.zscale;   // (a power of two: exact)
    if (a.zdtype == 3) {   // hi = bf16(x), lo = bf16(x - hi) in a second plane
      uint16_t* __restrict__ lr = zr + a.zplane;
      uint16_t* __restrict__ li = zi + a.zplane;
      final_stage<Lay, L, RL, S>(lds, pyr, tid, [&](int f, int n1, V val, int) {
        const int64_t q = (int64_t)(row0 + f) * L + n1;
        const float xr = val.x * sc, xi = val.y * sc;
        const uint16_t hr = f32_to_bf16_rne(xr), hi = f32_to_bf16_rne(xi);
        zr[q] = hr;
        zi[q] = hi;
        lr[q] = f32_to_bf16_rne(xr - __uint_as_float((uint32_t)hr << 16));
        li[q] = f32_to_bf16_rne(xi - __uint_as_float((uint32_t)hi << 16));
      });
    } else {
      const bool bf = (a.zdtype == 1);
      final_stage<Lay, L, RL, S>(lds, pyr, tid, [&](int f, int n1, V val, int) {
        const int64_t q = (int64_t)(row0 + f) * L + n1;
        const float xr = val.x * sc, xi = val.y * sc;
        zr[q] = bf ? f32_to_bf16_rne(xr) : f32_to_f16_rne(xr);
        zi[q] = bf ? f32_to_bf16_rne(xi) : f32_to_f16_rne(xi);
      });
    }
  } else if constexpr (OUT == OUT_THRESH) {
    const float thr2 = a.thr2;
    const int lane = __lane_id();
    // running maximum in registers (ties to the lowest sample), tracked only
    // when the caller asked for per-template peaks (tmpl_max != NULL).
    // Crossings of a wave are staged in LDS and appended with one counter
    // atomic per 64 records: near a loud signal every sample of a template
    // crosses, and per-lane atomics on the one counter would serialise.
    // (Every lane of the workgroup runs every store of the final stage, so
    // the ballots see whole waves.)
    __shared__ TrigRec stage_buf[NT / 64][64];
    TrigRec* const stg = stage_buf[tid >> 6];
    int ns = 0;
    auto flush = [&]() {
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      unsigned lo = 0, hi = 0;
      if (lane == 0) {
        const unsigned long long b = atomicAdd(a.trig_count, (unsigned long long)ns);
        lo = (unsigned)b;
        hi = (unsigned)(b >> 32);
      }
      const unsigned long long base = ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)hi) << 32) |
                                      (unsigned)__builtin_amdgcn_readfirstlane((int)lo);
      for (int t = lane; t < ns; t += 64)
        if ((int64_t)(base + t) < a.trig_cap) a.trig[base + t] = stg[t];
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      ns = 0;
    };
    const bool track = a.tmpl_max != nullptr;
    float bp = -1.f;
    int bn = 0x7fffffff;
    final_stage<Lay, L, RL, S>(lds, pyr, tid, [&](int f, int n1, V val, int) {
      const int n = (row0 + f) + N2 * n1;
      const float p = val.x * val.x + val.y * val.y;
      if (track && (p > bp || (p == bp && n < bn))) {
        bp = p;
        bn = n;
      }
      const bool hit = p >= thr2;
      const unsigned long long mask = __ballot(hit);
      if (mask != 0ull) {                                   // (wave-uniform)
        const int cnt = __popcll(mask);
        if (lane == 0) atomicAdd(&a.tmpl_count[v], cnt);
        if (ns + cnt > 64) flush();
        if (hit) {
          TrigRec t;
          t.tmpl = v;
          t.sample = n;
          t.re = val.x;
          t.im = val.y;
          stg[ns + __popcll(mask & ((1ull << lane) - 1ull))] = t;
        }
        ns += cnt;
      }
    });
    if (ns > 0) flush();
    if (track) {
      unsigned long long best =
          bp < 0.f ? 0ull
                   : ((unsigned long long)__float_as_uint(bp) << 32) | (unsigned long long)(0xffffffffu - (uint32_t)bn);
      // wave-reduce the running maximum, one atomic per wave
      for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(best, off);
        best = o > best ? o : best;
      }
      if (lane == 0 && best != 0ull) atomicMax(&a.tmpl_max[v], best);
    }
  } else if constexpr (OUT == OUT_NATURAL) {
    float2* __restrict__ o = a.cout + (int64_t)v * N;
    final_stage<Lay, L, RL, S>(lds, pyr, tid, [&](int f, int n1, V val, int) {
      const int64_t n = (int64_t)(row0 + f) + (int64_t)N2 * n1;
      o[n] = make_float2(val.x, val.y);
    });
  } else if constexpr (OUT == OUT_ZBIN || OUT == OUT_ZBIN_H) {
    // Binned first stage.  The block holds F consecutive rows (samples
    // row0 .. row0 + F - 1 of every n1 slice).  After the final stage the
    // outputs go back to LDS as X[e], e = n1 F + f (one pad slot every 32
    // elements keeps both the row-wise stores and the e-wise loads free of
    // bank conflicts) and leave as
    //  (a) complex64 Z with each slice's F samples adjacent,
    //      q = row0 L + n1 F + f, so that the fine reconstruction of a bin
    //      reads whole runs;
    //  (b) sums over G = min(F, w) consecutive samples in a fixed order
    //      (f ascending): the bin means themselves when G = w (planar, in the
    //      reconstruction dtype, [N2 / w][L] per plane), else partial sums
    //      ([N2 / G][L] complex64) that k_bin_reduce completes.
    constexpr int F = Lay::NF;
    constexpr int NBF = F * L / RL;
    constexpr int PERF = (NBF + NT - 1) / NT;
    V keep[PERF * RL];
    if constexpr (OUT == OUT_ZBIN_H) {   // remove the FP16 intermediate's scale (a power of two: exact)
      const float is = a.hscale[1];
      final_stage<Lay, L, RL, S>(lds, pyr, tid, [&](int, int, V val, int idx) { keep[idx] = mk<V>(val.x * is, val.y * is); });
    } else {
      final_stage<Lay, L, RL, S>(lds, pyr, tid, [&](int, int, V val, int idx) { keep[idx] = val; });
    }
    __syncthreads();
    auto xa = [](int e) { return e + (e >> 5); };
#pragma unroll
    for (int i = 0; i < PERF; ++i) {
      const int b = tid + i * NT;
      if (NBF % NT == 0 || b < NBF) {
        int f, j;
        Lay::template split<RL>(b, f, j);
#pragma unroll
        for (int m = 0; m < RL; ++m) lds[xa((j + m * (L / RL)) * F + f)] = keep[i * RL + m];
      }
    }
    __syncthreads();
    if (a.zfine16 == 0) {
      float2* __restrict__ zf = static_cast<float2*>(a.zfine) + (int64_t)v * N + (int64_t)row0 * L;
      for (int e = tid; e < F * L; e += NT) zf[e] = lds[xa(e)];
    } else {   // 16-bit (Re, Im) pairs: bf16 (1) or f16 (2)
      uint32_t* __restrict__ zf = static_cast<uint32_t*>(a.zfine) + (int64_t)v * N + (int64_t)row0 * L;
      const bool bf = a.zfine16 == 1;
      for (int e = tid; e < F * L; e += NT) {
        const V x = lds[xa(e)];
        const uint32_t lo = bf ? f32_to_bf16_rne(x.x) : f32_to_f16_rne(x.x);
        const uint32_t hi = bf ? f32_to_bf16_rne(x.y) : f32_to_f16_rne(x.y);
        zf[e] = lo | (hi << 16);
      }
    }
    const int G = a.bin_g;            // power of two dividing F
    const int ng = F / G;
    const int64_t r0 = row0 / G;
    if (G == a.bin_w) {
      const int64_t Nb = N / G;
      const float sc = a.zscale / (float)G;   // G is a power of two: exact
      for (int o = tid; o < ng * L; o += NT) {
        const int n1 = o % L, gi = o / L;
        float sr = 0.f, si = 0.f;
        for (int f = 0; f < G; ++f) {
          const V x = lds[xa(n1 * F + gi * G + f)];
          sr += x.x;
          si += x.y;
        }
        const int64_t ob = (r0 + gi) * L + n1;
        const float xr = sr * sc, xi = si * sc;
        if (a.zdtype == 0) {
          a.zout[(int64_t)(2 * v) * Nb + ob] = xr;
          a.zout[(int64_t)(2 * v + 1) * Nb + ob] = xi;
        } else {
          uint16_t* zr = reinterpret_cast<uint16_t*>(a.zout) + (int64_t)(2 * v) * Nb + ob;
          uint16_t* zi = zr + Nb;
          if (a.zdtype == 3) {
            const uint16_t hr = f32_to_bf16_rne(xr), hi = f32_to_bf16_rne(xi);
            zr[0] = hr;
            zi[0] = hi;
            zr[a.zplane] = f32_to_bf16_rne(xr - __uint_as_float((uint32_t)hr << 16));
            zi[a.zplane] = f32_to_bf16_rne(xi - __uint_as_float((uint32_t)hi << 16));
          } else if (a.zdtype == 1) {
            zr[0] = f32_to_bf16_rne(xr);
            zi[0] = f32_to_bf16_rne(xi);
          } else {
            zr[0] = f32_to_f16_rne(xr);
            zi[0] = f32_to_f16_rne(xi);
          }
        }
      }
    } else {
      float2* __restrict__ part = a.zpart + (int64_t)v * (N / G) + r0 * L;
      for (int o = tid; o < ng * L; o += NT) {
        const int n1 = o % L, gi = o / L;
        float sr = 0.f, si = 0.f;
        for (int f = 0; f < G; ++f) {
          const V x = lds[xa(n1 * F + gi * G + f)];
          sr += x.x;
          si += x.y;
        }
        part[(int64_t)gi * L + n1] = make_float2(sr, si);
      }
    }
  } else if constexpr (OUT == OUT_TRANSPOSED) {
    float2* __restrict__ o = a.cout + (int64_t)v * N;
    final_stage<Lay, L, RL, S>(lds, pyr, tid, [&](int f, int n1, V val, int) {
      o[(int64_t)(row0 + f) * L + n1] = make_float2(val.x, val.y);
    });
  } else {   // OUT_SPECTRUM: whitening in the pass's own precision, then FP32
    final_stage<Lay, L, RL, S>(lds, pyr, tid, [&](int f, int n1, V val, int) {
      const int64_t k = (int64_t)(row0 + f) + (int64_t)N2 * n1;
      if (k >= a.k_lo && k <= a.k_hi) {
        const double w = a.wd64[k - a.kb];
        a.cout[k - a.kb] = make_float2((float)(val.x * w), (float)(val.y * w));
      }
    });
  }
}

// ------------------------------------------------------------------ FP16 intermediate scale
// Partial maxima of |d| (one per workgroup, kHalfScaleParts workgroups).
__global__ __launch_bounds__(256) void k_absmax_part(const float2* d, int64_t n, float* part) {
  float m = 0.f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float2 x = d[i];
    m = fmaxf(m, x.x * x.x + x.y * x.y);
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  __shared__ float wm[4];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmaxf(fmaxf(wm[0], wm[1]), fmaxf(wm[2], wm[3]));
}

// {s, 1 / s} from the partial maxima of |d|^2 (one wave).
__global__ void k_half_scale(const float* part, int n2, float* hs) {
  float m = 0.f;
  for (int i = threadIdx.x; i < kHalfScaleParts; i += 64) m = fmaxf(m, part[i]);
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if (threadIdx.x == 0) {
    const float bound = 2.f * sqrtf((float)n2) * sqrtf(m);   // >= every pass-1 output's magnitude
    int e = 0;
    if (bound > 0.f) e = (int)floorf(log2f(32768.f / bound));
    e = e < -120 ? -120 : (e > 120 ? 120 : e);
    hs[0] = ldexpf(1.f, e);
    hs[1] = ldexpf(1.f, -e);
  }
}

// ------------------------------------------------------------------ dispatch
template <int L>
struct Radices;
template <> struct Radices<64> { static constexpr int r1 = 8, r2 = 8, r3 = 1; };
template <> struct Radices<128> { static constexpr int r1 = 16, r2 = 8, r3 = 1; };
template <> struct Radices<256> { static constexpr int r1 = 16, r2 = 16, r3 = 1; };
template <> struct Radices<512> { static constexpr int r1 = 8, r2 = 8, r3 = 8; };
template <> struct Radices<1024> { static constexpr int r1 = 16, r2 = 8, r3 = 8; };
template <> struct Radices<2048> { static constexpr int r1 = 16, r2 = 16, r3 = 8; };

template <class V, int L, int IN, int S>
hipError_t go1(const PassArgs& a, hipStream_t st) {
  using Rd = Radices<L>;
  dim3 grid(a.g.N1 / Cols1<V, L, IN>::value, a.nvec);
  hipLaunchKernelGGL((k_pass1<V, L, Rd::r1, Rd::r2, Rd::r3, IN, S>), grid, dim3(NT), 0, st, a);
  return hipGetLastError();
}
template <class V, int L, int OUT, int S>
hipError_t go2(const PassArgs& a, hipStream_t st) {
  using Rd = Radices<L>;
  dim3 grid(a.g.N2 / RowLayout<L>::NF, a.nvec);
  hipLaunchKernelGGL((k_pass2<V, L, Rd::r1, Rd::r2, Rd::r3, OUT, S>), grid, dim3(NT), 0, st, a);
  return hipGetLastError();
}

template <class V, int IN, int S>
hipError_t disp1(const PassArgs& a, hipStream_t st) {
  switch (a.g.N2) {   // N2 <= 1024 for N <= 2^21
    case 64: return go1<V, 64, IN, S>(a, st);
    case 128: return go1<V, 128, IN, S>(a, st);
    case 256: return go1<V, 256, IN, S>(a, st);
    case 512: return go1<V, 512, IN, S>(a, st);
    case 1024: return go1<V, 1024, IN, S>(a, st);
    default: return hipErrorInvalidValue;
  }
}
template <class V, int OUT, int S>
hipError_t disp2(const PassArgs& a, hipStream_t st) {
  switch (a.g.N1) {
    case 64: return go2<V, 64, OUT, S>(a, st);
    case 128: return go2<V, 128, OUT, S>(a, st);
    case 256: return go2<V, 256, OUT, S>(a, st);
    case 512: return go2<V, 512, OUT, S>(a, st);
    case 1024: return go2<V, 1024, OUT, S>(a, st);
    case 2048: return go2<V, 2048, OUT, S>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

FftGeom make_geom(int64_t N, int n2log) {
  FftGeom g;
  g.N = N;
  int m = 0;
  while ((int64_t(1) << m) < N) ++m;
  g.log2N = m;
  if (n2log < 0) n2log = m / 2;
  g.N2 = 1 << n2log;
  g.N1 = 1 << (m - n2log);
  g.s_lo = (m + 1) / 2;
  return g;
}

bool geom_supported(const FftGeom& g) {
  return g.N2 >= 64 && g.N2 <= 1024 && g.N1 >= 64 && g.N1 <= 2048 && g.N1 * (int64_t)g.N2 == g.N;
}

hipError_t launch_half_scale(const float2* d, int64_t n, int n2, float* part, float* hs, hipStream_t st) {
  if (n <= 0 || n2 <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_absmax_part, dim3(kHalfScaleParts), dim3(256), 0, st, d, n, part);
  hipLaunchKernelGGL(k_half_scale, dim3(1), dim3(64), 0, st, part, n2, hs);
  return hipGetLastError();
}

hipError_t launch_pass1(const PassArgs& a, InKind in, hipStream_t st) {
  if (a.nvec <= 0) return hipSuccess;
  if (in == IN_CORR) return a.sign > 0 ? disp1<float2, IN_CORR, 1>(a, st) : disp1<float2, IN_CORR, -1>(a, st);
  if (in == IN_CORR_H) return a.sign > 0 && a.hscale ? disp1<float2, IN_CORR_H, 1>(a, st) : hipErrorInvalidValue;
  if (in == IN_FOLD) return a.sign > 0 ? disp1<float2, IN_FOLD, 1>(a, st) : hipErrorInvalidValue;
  if (in == IN_REAL) return disp1<double2, IN_REAL, -1>(a, st);     // strain spectrum: FP64
  return a.sign > 0 ? disp1<float2, IN_DENSE, 1>(a, st) : disp1<float2, IN_DENSE, -1>(a, st);
}

hipError_t launch_pass2(const PassArgs& a, OutKind out, hipStream_t st) {
  if (a.nvec <= 0) return hipSuccess;
  switch (out) {
    case OUT_Z32: return disp2<float2, OUT_Z32, 1>(a, st);
    case OUT_Z16: return disp2<float2, OUT_Z16, 1>(a, st);
    case OUT_Z16_H: return a.hscale ? disp2<float2, OUT_Z16_H, 1>(a, st) : hipErrorInvalidValue;
    case OUT_THRESH: return disp2<float2, OUT_THRESH, 1>(a, st);
    case OUT_NATURAL:
      return a.sign > 0 ? disp2<float2, OUT_NATURAL, 1>(a, st) : disp2<float2, OUT_NATURAL, -1>(a, st);
    case OUT_ZBIN: return disp2<float2, OUT_ZBIN, 1>(a, st);
    case OUT_ZBIN_H: return a.hscale ? disp2<float2, OUT_ZBIN_H, 1>(a, st) : hipErrorInvalidValue;
    case OUT_TRANSPOSED:
      return a.sign > 0 ? disp2<float2, OUT_TRANSPOSED, 1>(a, st) : disp2<float2, OUT_TRANSPOSED, -1>(a, st);
    case OUT_SPECTRUM: return disp2<double2, OUT_SPECTRUM, -1>(a, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace rbmf
