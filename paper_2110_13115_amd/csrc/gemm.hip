// Reconstruction GEMM rho = C * Z on MFMA with a fused first-stage threshold
// (Sec. II.A Eq. Beta_eqn: rho_j = sum_k c*_{jk} beta_k; Sec. III.C: first
// stage over the whole bank).  rho is never written to memory.
//
// The complex product is realified: output row 2j is Re rho_j, row 2j+1 is
// Im rho_j, reduction index 2k / 2k+1 runs over Re / Im of beta_k, with
//   A[2j  ][2k] =  Re C_jk   A[2j  ][2k+1] = -Im C_jk
//   A[2j+1][2k] =  Im C_jk   A[2j+1][2k+1] =  Re C_jk
// so that Re rho and Im rho of one (template, sample) land in the same lane
// of the 32x32 MFMA accumulator (rows 4g..4g+3 of a lane are consecutive).
//
// FP32 path: v_mfma_f32_32x32x2_f32, one complex k per instruction.
// 16-bit path: v_mfma_f32_32x32x16_{bf16,f16}, eight complex k per
// instruction, FP32 accumulation.
#include "internal.h"

namespace rbmf {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int WAVES = 4;
constexpr int WT_ROWB = 2;       // 32-row MFMA blocks per wave (= 32 templates)
constexpr int WT_COLB = 2;       // 32-column MFMA blocks per wave (= 64 samples)
constexpr int TILE_T = WAVES * WT_ROWB * 16;   // templates per workgroup (128)
constexpr int TILE_N = WT_COLB * 32;           // samples per workgroup (64)
constexpr size_t kLdsMax = 160 * 1024;         // gfx950 LDS per workgroup

// Crossing records of one wave staged in LDS: a tile whose samples meet many
// crossings (an injection seen by every template of the bank) would otherwise
// wait on one returning counter atomic per step; staged, it takes one per
// kStage records.
constexpr int kStage = 64;
constexpr size_t kStageBytes = (size_t)WAVES * kStage * sizeof(TrigRec);
struct WaveStage {
  TrigRec* buf;   // this wave's kStage LDS slots
  int n;          // records staged (wave-uniform)
};

__device__ __forceinline__ void stage_flush(const GemmArgs& a, WaveStage& s, int lane) {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  unsigned lo = 0, hi = 0;
  if (lane == 0) {
    const unsigned long long b = atomicAdd(a.trig_count, (unsigned long long)s.n);
    lo = (unsigned)b;
    hi = (unsigned)(b >> 32);
  }
  const unsigned long long base = ((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)hi) << 32) |
                                  (unsigned)__builtin_amdgcn_readfirstlane((int)lo);
  for (int t = lane; t < s.n; t += 64)
    if ((int64_t)(base + t) < a.trig_cap) a.trig[base + t] = s.buf[t];
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  s.n = 0;
}

// Appends the crossings of one accumulator step (lanes 0-31 hold one template
// row, lanes 32-63 another, each lane one sample): one count atomic per row
// and the records at the ballot's prefix count in the wave's stage.
__device__ __forceinline__ void stage_append(const GemmArgs& a, WaveStage& stg, int lane, bool hit, int j, int n,
                                             float re, float im) {
  const unsigned long long mask = __ballot(hit);
  if (mask == 0ull) return;                                  // (wave-uniform)
  const unsigned half = (unsigned)(mask >> (lane & 32));
  if ((lane & 31) == 0 && half != 0u) atomicAdd(&a.tmpl_count[j], __popc(half));
  const int cnt = __popcll(mask);
  if (stg.n + cnt > kStage) stage_flush(a, stg, lane);
  if (hit) {
    TrigRec t;
    t.tmpl = a.tmpl_base + j;
    t.sample = n;
    t.re = re;
    t.im = im;
    stg.buf[stg.n + __popcll(mask & ((1ull << lane) - 1ull))] = t;
  }
  stg.n += cnt;
}

// Threshold epilogue of the FP32 realified kernels: each output element tests
// its own |rho|^2 against its row's threshold; the crossings of a step are
// appended through the wave's LDS stage (one counter atomic per 64 records:
// a tile under a loud injection, where every template crosses, would
// otherwise serialise on one returning atomic per crossing).
template <int RB, int CB>
__device__ __forceinline__ void epilogue_lane(const GemmArgs& a, const f32x16 (&acc)[RB][CB], int rb0,
                                              int64_t q0, WaveStage& stg) {
  const int lane = __lane_id();
  const int l1 = __builtin_ctz((unsigned)a.N1);            // N1 is a power of two
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    // a lane's outputs of one row block cover 8 templates and CB samples:
    // their thresholds are fetched once per block
    float th[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int j = (rb0 + rb) * 16 + 4 * (h >> 1) + 2 * (lane >> 5) + (h & 1);
      th[h] = j < a.T ? a.thr2_row[j] : __builtin_inff();
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int q = (int)q0 + CB * (lane & 31) + cb;        // q < N < 2^31 (column CB l + cb)
      const int n = (q >> l1) + a.N2 * (q & (a.N1 - 1));
#pragma unroll
      for (int i = 0; i < 16; i += 2) {
        const int m = 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);   // even: Re row
        const int j = (rb0 + rb) * 16 + (m >> 1);
        const float re = acc[rb][cb][i], im = acc[rb][cb][i + 1];
        const float p = re * re + im * im;
        if (a.rho_out != nullptr && j < a.T) {
          const float s = a.row_inv ? a.row_inv[j] : 1.f;
          a.rho_out[(int64_t)j * a.N + n] = make_float2(re * s, im * s);
        }
        stage_append(a, stg, lane, j < a.T && p >= th[i >> 1], j, n, re, im);
      }
    }
  }
}

// Wave-level threshold epilogue (16-bit kernels, whose short k-loops make the
// epilogue a large part of a tile): one threshold load and one ballot per
// template-row step after a maximum over the columns; crossings are staged
// per wave (stage_flush appends them).
// The thresholds of a lane's template rows (h = i / 2 of accumulator element i).
template <int RB>
__device__ __forceinline__ void epi_thresholds(const GemmArgs& a, int rb0, float (&th)[RB][8]) {
  const int lane = __lane_id();
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int j = (rb0 + rb) * 16 + 4 * (h >> 1) + 2 * (lane >> 5) + (h & 1);
      th[rb][h] = a.thr2_row[j];   // padded rows: C = 0, so |rho|^2 = 0 never reaches it
    }
}

template <int RB, int CB>
__device__ __forceinline__ void epilogue(const GemmArgs& a, const f32x16 (&acc)[RB][CB], int rb0,
                                         int64_t q0, WaveStage& stg, const float (&th)[RB][8]) {
  const int lane = __lane_id();
  const int l1 = __builtin_ctz((unsigned)a.N1);            // N1 is a power of two
  if (a.rho_out != nullptr) {   // debug dump (thresholds are infinite then: nothing is appended)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const int q = (int)q0 + cb * 32 + (lane & 31);      // q < N < 2^31
        const int n = (q >> l1) + a.N2 * (q & (a.N1 - 1));
#pragma unroll
        for (int i = 0; i < 16; i += 2) {
          const int m = 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);   // even: Re row
          const int j = (rb0 + rb) * 16 + (m >> 1);
          if (j < a.T) {
            const float s = a.row_inv ? a.row_inv[j] : 1.f;
            a.rho_out[(int64_t)j * a.N + n] = make_float2(acc[rb][cb][i] * s, acc[rb][cb][i + 1] * s);
          }
        }
      }
    return;
  }
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
    for (int i = 0; i < 16; i += 2) {
      // one template row per half-wave at this step; its threshold (padded
      // rows have C = 0, so |rho|^2 = 0 never reaches a positive threshold)
      const int m = 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
      const int j = (rb0 + rb) * 16 + (m >> 1);
      const float thr = th[rb][i >> 1];
      float pmax = 0.f;
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const float re = acc[rb][cb][i], im = acc[rb][cb][i + 1];
        pmax = fmaxf(pmax, re * re + im * im);
      }
      if (__ballot(pmax >= thr) == 0ull) continue;   // the common case: no crossing in the step
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        const float re = acc[rb][cb][i], im = acc[rb][cb][i + 1];
        // one count atomic per template row (lanes 0-31 and 32-63 each hold
        // one row of this step); the records go to the wave's stage at the
        // prefix count of the ballot
        const bool hit = j < a.T && re * re + im * im >= thr;
        const unsigned long long mask = __ballot(hit);
        if (mask == 0ull) continue;
        const int cnt = __popcll(mask);
        const unsigned half = (unsigned)(mask >> (lane & 32));
        if ((lane & 31) == 0 && half != 0u) atomicAdd(&a.tmpl_count[j], __popc(half));
        if (stg.n + cnt > kStage) stage_flush(a, stg, lane);
        if (hit) {
          const int q = (int)q0 + cb * 32 + (lane & 31);
          TrigRec t;
          t.tmpl = a.tmpl_base + j;
          t.sample = (q >> l1) + a.N2 * (q & (a.N1 - 1));
          t.re = re;
          t.im = im;
          stg.buf[stg.n + __popcll(mask & ((1ull << lane) - 1ull))] = t;
        }
        stg.n += cnt;
      }
    }
  }
}

// Compact 16-bit form (k_recon_16_lds with CX): acc[0][cb] / acc[1][cb] hold
// Re / Im rho of 32 templates from j0 x 32 samples; element i of a lane is
// template j0 + 8 (i / 4) + 4 (lane / 32) + i % 4, whose squared threshold
// goes to th[i / 8][i % 8].
__device__ __forceinline__ void epi_thresholds_c(const GemmArgs& a, int j0, float (&th)[2][8]) {
  const int lane = __lane_id();
#pragma unroll
  for (int i = 0; i < 16; ++i) th[i >> 3][i & 7] = a.thr2_row[j0 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3)];
}

template <int CB>
__device__ __forceinline__ void epilogue_c(const GemmArgs& a, const f32x16 (&acc)[2][CB], int j0, int64_t q0,
                                           WaveStage& stg, const float (&th)[2][8]) {
  const int lane = __lane_id();
  const int l1 = __builtin_ctz((unsigned)a.N1);            // N1 is a power of two
  if (a.rho_out != nullptr) {   // debug dump (thresholds are infinite then: nothing is appended)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int q = (int)q0 + cb * 32 + (lane & 31);        // q < N < 2^31
      const int n = (q >> l1) + a.N2 * (q & (a.N1 - 1));
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int j = j0 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        if (j < a.T) {
          const float s = a.row_inv ? a.row_inv[j] : 1.f;
          a.rho_out[(int64_t)j * a.N + n] = make_float2(acc[0][cb][i] * s, acc[1][cb][i] * s);
        }
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    // one template per half-wave at this step (padded templates have C = 0)
    const int j = j0 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
    const float thr = th[i >> 3][i & 7];
    float pmax = 0.f;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const float re = acc[0][cb][i], im = acc[1][cb][i];
      pmax = fmaxf(pmax, re * re + im * im);
    }
    if (__ballot(pmax >= thr) == 0ull) continue;   // the common case: no crossing in the step
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const float re = acc[0][cb][i], im = acc[1][cb][i];
      const int q = (int)q0 + cb * 32 + (lane & 31);
      stage_append(a, stg, lane, j < a.T && re * re + im * im >= thr, j, (q >> l1) + a.N2 * (q & (a.N1 - 1)), re,
                   im);
    }
  }
}

// The Im-output operand of the compact form from its Re-output operand: each
// 32-bit word (Re C, -Im C) (low, high half) becomes (Im C, Re C), a rotate by
// 16 bits and a flip of the new low half's sign bit (exact for BF16 and FP16
// alike, and for both planes of the split form: the lo plane of -x is -lo).
__device__ __forceinline__ u16x8 im_operand(u16x8 v) {
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  u32x4 w = __builtin_bit_cast(u32x4, v);
#pragma unroll
  for (int e = 0; e < 4; ++e) w[e] = ((w[e] >> 16) | (w[e] << 16)) ^ 0x8000u;
  return __builtin_bit_cast(u16x8, w);
}

// One 16-bit MFMA step; DT 1 = bf16, 2 = f16.
template <int DT>
__device__ __forceinline__ f32x16 mfma16(u16x8 a, u16x8 b, f32x16 c) {
  if constexpr (DT == 2)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                  0, 0);
  else
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// Accumulates one k-step: DT 1 / 2 one product; DT 3 (bf16 hi + lo split of
// both operands) the three leading partial products, smallest first.
template <int DT>
__device__ __forceinline__ f32x16 kstep(u16x8 ah, u16x8 al, u16x8 bh, u16x8 bl, f32x16 c) {
  if constexpr (DT == 3) {
    c = mfma16<1>(al, bh, c);
    c = mfma16<1>(ah, bl, c);
    return mfma16<1>(ah, bh, c);
  } else {
    return mfma16<DT>(ah, bh, c);
  }
}

// Maps a linear workgroup id to (template tile, sample tile) so that the
// template tiles sharing one sample tile run on the same XCD (workgroups are
// dispatched round-robin over the 8 XCDs): Z is then fetched into each L2 once.
__device__ __forceinline__ bool xcd_tile(int ntt, int64_t nwg, int& tt, int64_t& st) {
  // (nwg = template tiles x sample tiles)
  const int64_t per = (nwg + 7) / 8;
  const int64_t bid = blockIdx.x;
  const int64_t L = (bid % 8) * per + bid / 8;
  if (L >= nwg) return false;
  tt = (int)(L % ntt);
  st = L / ntt;
  return true;
}

// RB x CB: 16-template row blocks x 32-sample column blocks per wave.
// Operands of G k-steps (a group, G even) are loaded into one of three
// register buffers two groups before their MFMAs run; the last K mod G
// k-steps run one at a time.  All operand loads are 8 or 16 bytes wide: lane l
// holds, in block cb, the column CB (l % 32) + cb of the wave's 32 CB samples,
// so one load gives its B values of all CB blocks, and the packed A holds a
// lane's values of both row blocks and two k-steps in one float4.  (With one
// 4-byte load per block and k-step, the vector memory path, not the MFMAs,
// bounds the loop.)
// Main loop and epilogue of one wave's RB x CB tile (templates from row
// block rb0, samples from q0); RB = 1 uses the first row block of the packed
// pair only.
template <int CB>
struct BVec;
template <>
struct BVec<4> {
  typedef float4 T;
  static __device__ __forceinline__ float at(const float4& v, int c) {
    return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w;
  }
};
template <>
struct BVec<2> {
  typedef float2 T;
  static __device__ __forceinline__ float at(const float2& v, int c) { return c == 0 ? v.x : v.y; }
};

template <int RB, int CB, int G>
__device__ __forceinline__ void recon_f32_tile(const GemmArgs& a, int rb0, int64_t q0, WaveStage& stg) {
  static_assert(G % 2 == 0, "groups hold whole k-pairs");
  static_assert(RB == 1 || RB == 2 || RB == 4, "one, two or four 16-template blocks");
  constexpr int NT = RB == 4 ? 2 : 1;                      // packed 32-template tiles per wave
  typedef typename BVec<CB>::T bvec;
  const int lane = threadIdx.x & 63;
  const int K = a.K;
  const int64_t N = a.N;
  const int KP = (K + 1) / 2;                              // packed k-pairs
  const int64_t tstr = (int64_t)KP * 64;                   // float4 per packed tile
  const float4* __restrict__ ap = static_cast<const float4*>(a.cpk) + (int64_t)(rb0 / 2) * tstr + lane;
  const float* zrow = static_cast<const float*>(a.z) + (int64_t)(lane >> 5) * N + q0 + CB * (lane & 31);
  const bvec* __restrict__ bp = reinterpret_cast<const bvec*>(zrow);
  const int64_t rstep = (2 * N) / CB;                      // one k-step (two reduction rows), in bvec

  f32x16 acc[RB][CB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = (f32x16){};

  const float4* pa = ap;
  const bvec* pb = bp;
  float4 fa[3][G / 2][NT];
  bvec fb[3][G];
  auto load = [&](int s) {   // loads the group at the pointers, then advances them
#pragma unroll
    for (int h = 0; h < G / 2; ++h)
#pragma unroll
      for (int t = 0; t < NT; ++t) fa[s][h][t] = pa[t * tstr + h * 64];
#pragma unroll
    for (int g = 0; g < G; ++g) fb[s][g] = pb[g * rstep];
    pa += (G / 2) * 64;
    pb += G * rstep;
  };
  // A value of row block rb at k-step g of a group (entries: block 2t + (e & 1), k-step e >> 1)
  auto aval = [&](const float4 (&f)[NT], int g, int rb) {
    const float4 v = f[rb >> 1];
    return (g & 1) ? ((rb & 1) ? v.w : v.z) : ((rb & 1) ? v.y : v.x);
  };
  auto mma = [&](int s) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const float av = aval(fa[s][g / 2], g, rb);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, BVec<CB>::at(fb[s][g], cb), acc[rb][cb], 0, 0, 0);
      }
    }
  };
  const int ng = K / G;                 // full groups; the last K mod G k-steps run singly
  const int Kmain = ng * G;
  int gi = 0;
  // Steady state: groups gi and gi + 1 are in buffers 0 and 1, and the three
  // loads of an iteration (groups gi + 2 .. gi + 4) all exist.  Neither the
  // body nor the path into it has a conditional load: on a path with fewer
  // loads in flight the compiler's wait counts would cover that path too and
  // stall on loads issued just before.  The scheduling barriers keep each
  // load batch ahead of the MFMAs that follow.
  if (ng >= 5) {
    load(0);
    __builtin_amdgcn_sched_barrier(0);   // issued in the loop's order
    load(1);
    __builtin_amdgcn_sched_barrier(0);
    do {
      load(2);
      __builtin_amdgcn_sched_barrier(0);
      mma(0);
      __builtin_amdgcn_sched_barrier(0);
      load(0);
      __builtin_amdgcn_sched_barrier(0);
      mma(1);
      __builtin_amdgcn_sched_barrier(0);
      load(1);
      __builtin_amdgcn_sched_barrier(0);
      mma(2);
      __builtin_amdgcn_sched_barrier(0);
      gi += 3;
    } while (gi + 4 < ng);
  } else {
    if (ng > 0) load(0);
    if (ng > 1) load(1);
  }
  // at most four groups remain (gi .. gi + 3), the first two already loaded
  if (gi + 2 < ng) load(2);
  if (gi < ng) mma(0);
  if (gi + 3 < ng) load(0);
  if (gi + 1 < ng) mma(1);
  if (gi + 2 < ng) mma(2);
  if (gi + 3 < ng) mma(0);
  for (int k = Kmain; k < K; ++k) {
    float4 f[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) f[t] = ap[t * tstr + (int64_t)(k >> 1) * 64];
    const bvec bv = bp[(int64_t)k * rstep];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const float av = aval(f, k, rb);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, BVec<CB>::at(bv, cb), acc[rb][cb], 0, 0, 0);
    }
  }
  epilogue_lane<RB, CB>(a, acc, rb0, q0, stg);
}

// One workgroup = one row tile of 32 templates (two 16-template blocks); its
// four waves take adjacent column tiles of CB 32-sample blocks (so every wave
// of a workgroup has the same share of padding rows, and a sub-bank whose
// template count is not a multiple of 128 leaves no wave idle beside busy
// ones).
template <int CB, int G>
__global__ __launch_bounds__(256, 2) void k_recon_f32(GemmArgs a) {   // at least 2 waves per SIMD
  constexpr int TN = CB * 32;           // samples per wave; G: k-steps per pipeline group
  // row tiles with at least one real template only: workgroups of all-padding
  // tiles, even though they exit at once, measured 15-19 % slower launches
  const int ntt = (a.T + 31) / 32;
  const int64_t ncol = (a.N + WAVES * TN - 1) / (WAVES * TN);
  const int64_t nwg = (int64_t)ntt * ncol;
  int tt;
  int64_t st;
  if (!xcd_tile(ntt, nwg, tt, st)) return;
  const int wave = threadIdx.x >> 6;
  const int rb0 = tt * 2;                                  // first 16-template row block
  if (rb0 * 16 >= a.T) return;                             // all of this tile's rows are padding
  const int64_t q0 = (st * WAVES + wave) * TN;
  if (q0 >= a.N) return;                                   // (N is a multiple of TN)
  __shared__ TrigRec stage_mem[WAVES][kStage];
  WaveStage stg{stage_mem[wave], 0};
  // a wave whose second row block is all padding runs the one-block tile
  if ((rb0 + 1) * 16 >= a.T)
    recon_f32_tile<1, CB, G>(a, rb0, q0, stg);
  else
    recon_f32_tile<2, CB, G>(a, rb0, q0, stg);
  if (stg.n > 0) stage_flush(a, stg, threadIdx.x & 63);
}

// 64 templates (four 16-template blocks) x 32 CB samples per wave, one wave
// per SIMD (256 accumulator registers): half the B loads per MFMA of the
// 32-template tiles, measured 142 against 110 TFLOP/s in the main loop.  A
// row tile with fewer templates runs as a two- or one-block tile (the
// launcher gives this kernel whole 64-template tiles only).
template <int CB, int G>
__global__ __launch_bounds__(256, 1) void k_recon_f32_w64(GemmArgs a) {
  constexpr int TN = CB * 32;
  const int ntt = (a.T + 63) / 64;
  const int64_t ncol = (a.N + WAVES * TN - 1) / (WAVES * TN);
  const int64_t nwg = (int64_t)ntt * ncol;
  int tt;
  int64_t st;
  if (!xcd_tile(ntt, nwg, tt, st)) return;
  const int wave = threadIdx.x >> 6;
  const int rb0 = tt * 4;
  const int64_t q0 = (st * WAVES + wave) * TN;
  if (q0 >= a.N) return;                                   // (N is a multiple of TN)
  const int rows = a.T - rb0 * 16;                         // templates in this tile (>= 1)
  __shared__ TrigRec stage_mem[WAVES][kStage];
  WaveStage stg{stage_mem[wave], 0};
  if (rows > 32)
    recon_f32_tile<4, CB, G>(a, rb0, q0, stg);
  else if (rows > 16)
    recon_f32_tile<2, CB, G>(a, rb0, q0, stg);
  else
    recon_f32_tile<1, CB, G>(a, rb0, q0, stg);
  if (stg.n > 0) stage_flush(a, stg, threadIdx.x & 63);
}

// FP32 by Gauss's three real products instead of the realified four:
//   P1 = Cr Zr, P2 = Ci Zi, P3 = (Cr + Ci)(Zr + Zi);  Re rho = P1 - P2,
//   Im rho = P3 - P1 - P2
// (three MFMAs where the realified form needs four; the cancellation in Im
// costs about one more rounding of sum |C||Z|, far below the FP32 tolerance).
// One instruction reduces over a k-pair: lanes 0-31 hold k = 2 kp, lanes
// 32-63 k = 2 kp + 1, rows are templates.  A wave takes 32 templates x 128
// samples (three accumulator sets of four 32 x 32 blocks); the workgroup's
// four waves take adjacent sample tiles.  Pipeline as in recon_f32_tile, one
// k-pair per group.
__global__ __launch_bounds__(256, 2) void k_recon_f32_3m(GemmArgs a) {
  constexpr int CB = 4, TN = 128;
  const int ntt = (a.T + 31) / 32;
  const int64_t ncol = (a.N + WAVES * TN - 1) / (WAVES * TN);
  int tt;
  int64_t st;
  if (!xcd_tile(ntt, (int64_t)ntt * ncol, tt, st)) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t q0 = (st * WAVES + wave) * TN;
  if (q0 >= a.N) return;
  const int K = a.K;
  const int64_t N = a.N;
  const int KP = (K + 1) / 2;
  // Wave-uniform bases (scalar registers, advanced per k-pair) and 32-bit
  // per-lane byte offsets: the loads take the scalar-base form and the
  // k-loop holds no per-lane 64-bit addresses, which leaves the registers for
  // a fourth operand buffer.  A: float4 lane of the packed pair; Z: rows
  // 2k (Re) and 2k + 1 (Im) of k = 2 kp + lane / 32 (offsets < 2^32 bytes
  // for N <= 2^26).
  const char* pa = reinterpret_cast<const char*>(static_cast<const float4*>(a.cpk3) + (int64_t)tt * KP * 64);
  const char* pz = reinterpret_cast<const char*>(static_cast<const float*>(a.z) + q0);
  const uint32_t aoff = 16u * (uint32_t)lane;
  const uint32_t zro = 4u * ((uint32_t)(2 * (lane >> 5)) * (uint32_t)N + (uint32_t)(CB * (lane & 31)));
  const uint32_t zio = zro + 4u * (uint32_t)N;
  f32x16 p1[CB], p2[CB], p3[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) p1[c] = p2[c] = p3[c] = (f32x16){};
  constexpr int D = 3;                   // k-pairs in flight (a ring of D + 1 buffers)
  float4 fa[D + 1], fr[D + 1], fi[D + 1];
  auto load = [&](int s) {
    fa[s] = *reinterpret_cast<const float4*>(pa + aoff);
    fr[s] = *reinterpret_cast<const float4*>(pz + zro);
    fi[s] = *reinterpret_cast<const float4*>(pz + zio);
    pa += 64 * 16;
    pz += 4 * N * 4;
  };
  auto mma3 = [&](const float4& av, const float4& br4, const float4& bi4) {
    const float br[4] = {br4.x, br4.y, br4.z, br4.w};
    const float bi[4] = {bi4.x, bi4.y, bi4.z, bi4.w};
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      p1[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, br[c], p1[c], 0, 0, 0);
      p2[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, bi[c], p2[c], 0, 0, 0);
      p3[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, br[c] + bi[c], p3[c], 0, 0, 0);
    }
  };
  auto mma = [&](int s) { mma3(fa[s], fr[s], fi[s]); };
  const int ng = K / 2;                 // whole k-pairs; an odd K's last k runs after them
  int gi = 0;
  if (ng >= 2 * D + 1) {
    // steady state: k-pairs gi .. gi + D - 1 sit in buffers 0 .. D - 1;
    // sub-step s loads k-pair gi + s + D into buffer (s + D) mod (D + 1)
#pragma unroll
    for (int s = 0; s < D; ++s) {
      load(s);
      __builtin_amdgcn_sched_barrier(0);
    }
    do {
#pragma unroll
      for (int s = 0; s <= D; ++s) {
        load((s + D) % (D + 1));
        __builtin_amdgcn_sched_barrier(0);
        mma(s);
        __builtin_amdgcn_sched_barrier(0);
      }
      gi += D + 1;
    } while (gi + 2 * D + 1 <= ng);
  } else {
#pragma unroll
    for (int s = 0; s < D; ++s)
      if (s < ng) load(s);
  }
  // at most 2 D k-pairs remain, the first D loaded; pair gi + t is in buffer t mod (D + 1)
#pragma unroll
  for (int t = 0; t < 2 * D; ++t) {
    if (t < D && gi + t + D < ng) load((t + D) % (D + 1));
    if (gi + t < ng) mma(t % (D + 1));
  }
  if (K & 1) {
    // k = K - 1 in lanes 0-31; lanes 32-63 (k = K, zero coefficients) read
    // the same rows, which exist.  The bases have advanced past the ng
    // k-pairs (pa to the last packed pair, pz to row 2 (K - 1)).
    const uint32_t zt = 4u * (uint32_t)(CB * (lane & 31));
    mma3(*reinterpret_cast<const float4*>(pa + aoff), *reinterpret_cast<const float4*>(pz + zt),
         *reinterpret_cast<const float4*>(pz + zt + 4 * N));
  }
  // epilogue: element i of a block is template row 8 (i / 4) + 4 (lane / 32) + i % 4;
  // crossings go through the wave's LDS stage
  __shared__ TrigRec stage_mem[WAVES][kStage];
  // (the lane id again, from mbcnt: a value derived from it before the k-loop
  // would be kept across the loop, which has no register to spare)
  const int el = __lane_id();
  WaveStage stg{stage_mem[wave], 0};
  const int l1 = __builtin_ctz((unsigned)a.N1);
  // Re rho into p1, Im rho into p3 first: P2's registers are free before the
  // thresholds are fetched
#pragma unroll
  for (int c = 0; c < CB; ++c)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const float re = p1[c][i] - p2[c][i];
      p3[c][i] = p3[c][i] - p1[c][i] - p2[c][i];
      p1[c][i] = re;
    }
  float th[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int j = tt * 32 + 8 * (i >> 2) + 4 * (el >> 5) + (i & 3);
    th[i] = j < a.T ? a.thr2_row[j] : __builtin_inff();
  }
  if (a.rho_out != nullptr) {   // debug dump of the reconstructed series
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int q = (int)q0 + CB * (el & 31) + c;
      const int n = (q >> l1) + a.N2 * (q & (a.N1 - 1));
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int j = tt * 32 + 8 * (i >> 2) + 4 * (el >> 5) + (i & 3);
        if (j < a.T) {
          const float sc = a.row_inv ? a.row_inv[j] : 1.f;
          a.rho_out[(int64_t)j * a.N + n] = make_float2(p1[c][i] * sc, p3[c][i] * sc);
        }
      }
    }
  }
  // one ballot per template-row step over the maximum of its CB columns (the
  // common case: no crossing in the step), then the crossings of the step
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int j = tt * 32 + 8 * (i >> 2) + 4 * (el >> 5) + (i & 3);
    float pw[CB], pmax = 0.f;   // (each |rho|^2 computed once: the test and the append agree)
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      pw[c] = p1[c][i] * p1[c][i] + p3[c][i] * p3[c][i];
      pmax = fmaxf(pmax, pw[c]);
    }
    if (__ballot(j < a.T && pmax >= th[i]) == 0ull) continue;
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int q = (int)q0 + CB * (el & 31) + c;
      const int n = (q >> l1) + a.N2 * (q & (a.N1 - 1));
      stage_append(a, stg, el, j < a.T && pw[c] >= th[i], j, n, p1[c][i], p3[c][i]);
    }
  }
  if (stg.n > 0) stage_flush(a, stg, el);
}

// 16-bit operands: one instruction reduces over 16 realified entries = 8
// complex k.  A lane l holds entries [8 (l/32), 8 (l/32) + 8) of row l%32
// (4 complex k, Re/Im interleaved); B lane l holds the same 8 reduction rows
// of column l%32.  C is pre-packed so each lane loads 16 contiguous bytes; Z is planar
// (row 2k = Re, 2k+1 = Im) and gathered into the interleaved order here.
template <int DT>
__global__ __launch_bounds__(256) void k_recon_16(GemmArgs a) {
  constexpr int NP = DT == 3 ? 2 : 1;   // operand planes (hi, lo)
  const int ntt = a.Tp / TILE_T;
  const int64_t nwg = (int64_t)ntt * (a.N / TILE_N);
  int tt;
  int64_t st;
  if (!xcd_tile(ntt, nwg, tt, st)) return;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int rb0 = tt * (TILE_T / 16) + wave * WT_ROWB;
  if (rb0 * 16 >= a.T) return;                             // all of this wave's rows are padding
  const int64_t q0 = st * TILE_N;
  const u16x8* __restrict__ cpk = static_cast<const u16x8*>(a.cpk);
  const uint16_t* __restrict__ z = static_cast<const uint16_t*>(a.z);
  const int KB = a.Kp / 8;        // k-steps of 8 complex values (16 reduction rows)
  const int64_t N = a.N;
  const int64_t cplane = (int64_t)(a.Tp / 16) * KB * 64;   // u16x8 per C plane
  const int64_t zplane = (int64_t)2 * a.Kp * N;            // u16 per Z plane
  f32x16 acc[WT_ROWB][WT_COLB];
#pragma unroll
  for (int rb = 0; rb < WT_ROWB; ++rb)
#pragma unroll
    for (int cb = 0; cb < WT_COLB; ++cb) acc[rb][cb] = (f32x16){};
#pragma unroll 2
  for (int kb = 0; kb < KB; ++kb) {
    u16x8 av[NP][WT_ROWB], bv[NP][WT_COLB];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int rb = 0; rb < WT_ROWB; ++rb) av[p][rb] = cpk[p * cplane + ((int64_t)(rb0 + rb) * KB + kb) * 64 + lane];
#pragma unroll
      for (int cb = 0; cb < WT_COLB; ++cb) {
        const int64_t col = q0 + cb * 32 + (lane & 31);
        const int64_t row = 16 * kb + 8 * (lane >> 5);   // planar rows 2k+t of complex k = 8kb + 4h + ..
        u16x8 b;
#pragma unroll
        for (int e = 0; e < 8; ++e) b[e] = z[p * zplane + (row + e) * N + col];
        bv[p][cb] = b;
      }
    }
#pragma unroll
    for (int rb = 0; rb < WT_ROWB; ++rb)
#pragma unroll
      for (int cb = 0; cb < WT_COLB; ++cb)
        acc[rb][cb] = kstep<DT>(av[0][rb], av[NP - 1][rb], bv[0][cb], bv[NP - 1][cb], acc[rb][cb]);
  }
  __shared__ TrigRec stage_mem[WAVES][kStage];
  WaveStage stg{stage_mem[wave], 0};
  float th[WT_ROWB][8];
  epi_thresholds<WT_ROWB>(a, rb0, th);
  epilogue<WT_ROWB, WT_COLB>(a, acc, rb0, q0, stg, th);
  if (stg.n > 0) stage_flush(a, stg, lane);
}

// LDS layout of the staged Z tile: one row per sample holding the 32-bit
// (Re, Im) words of every plane and k (word p Kp + k), rows padded to a
// multiple of 64 words plus 4, so the 16-byte fragment reads of sixteen
// consecutive samples cover 64 distinct banks.  Word w of sample s is stored
// at w ^ zs_swizzle(s), a swizzle constant over each 16 samples (the
// fragment reads keep their banks) that separates the sixteen staging
// threads writing one k for samples 8 apart: their row offsets alternate
// between two bank halves and the swizzle spreads each half over eight bank
// quads (measured: a third of the kernel's cycles were LDS bank-conflict
// stalls without it).  A fragment's four words (w a multiple of 4) stay
// together.
__host__ __device__ __forceinline__ int zs_row_u16(int np, int kp) { return 2 * (((np * kp + 63) & ~63) + 4); }
__device__ __forceinline__ int zs_swizzle(int s) { return ((s >> 4) & 7) << 2; }

// 16-bit operands, Z tile staged in LDS.  One workgroup owns 32 CB samples and
// loops over every 128-template tile of the (sub-)bank: the planar Z tile
// (2Kp rows x 64 samples) is read from HBM once with 16-byte loads and stored
// transposed (sample-major, reduction index contiguous, rows padded by 16 B)
// so each lane's B fragment is a single 16-byte LDS read; the packed C tiles
// come from L2.
//
// CX (compact coefficients): an A fragment holds 32 templates instead of 16
// realified pairs, lane l carrying template l % 32 and the words
// (Re C_jk, -Im C_jk) of its four complex k (the k_pack_16c layout).  That
// fragment gives Re rho directly; the operand for Im rho, words
// (Im C_jk, Re C_jk), is formed in registers (im_operand), so each wave
// loads one coefficient fragment per k-step for its 32 templates where the
// realified form loads two.  The accumulators then pair up as acc[0][cb] =
// Re rho and acc[1][cb] = Im rho of the same 32 templates x 32 samples.
template <int DT, int CB, bool CX>
__global__ __launch_bounds__(256, 2) void k_recon_16_lds(GemmArgs a) {
  constexpr int TNS = CB * 32;          // samples per workgroup
  constexpr int NP = DT == 3 ? 2 : 1;   // operand planes (hi, lo)
  extern __shared__ uint16_t zs[];
  __shared__ TrigRec stage_mem[WAVES][kStage];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  WaveStage stg{stage_mem[wave], 0};
  const int64_t q0 = (int64_t)blockIdx.x * TNS;
  const int Kp = a.Kp, KB = Kp / 8, R2 = 2 * Kp;
  const int RS = zs_row_u16(NP, Kp);   // LDS row stride (u16) of one sample: planes side by side
  const int64_t N = a.N;
  const int64_t zplane = (int64_t)R2 * N;
  const uint16_t* __restrict__ z = static_cast<const uint16_t*>(a.z);
  {
    // One item = (plane p, complex k, 8 samples): rows 2k (Re) and 2k+1 (Im) are
    // loaded with 16-byte reads and stored as (Re, Im) 32-bit LDS words at
    // sample * RS + p * R2 + 2k; CH items per thread are in flight at once.
    uint32_t* zs32 = reinterpret_cast<uint32_t*>(zs);
    const int RS2 = RS / 2;
    const int items = NP * Kp * (TNS / 8);
    constexpr int CH = 4;
    for (int base = threadIdx.x; base < items; base += 256 * CH) {
      u16x8 vr[CH], vi[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int idx = base + c * 256;
        if (idx < items) {
          const int pk = idx / (TNS / 8), c8 = (idx % (TNS / 8)) * 8;   // pk = p * Kp + k
          const int p = pk / Kp, k = pk % Kp;
          const uint16_t* src = z + p * zplane + (int64_t)(2 * k) * N + q0 + c8;
          vr[c] = *reinterpret_cast<const u16x8*>(src);
          vi[c] = *reinterpret_cast<const u16x8*>(src + N);
        }
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int idx = base + c * 256;
        if (idx < items) {
          const int pk = idx / (TNS / 8), c8 = (idx % (TNS / 8)) * 8;
#pragma unroll
          for (int e = 0; e < 8; ++e)
            zs32[(c8 + e) * RS2 + (pk ^ zs_swizzle(c8))] = (uint32_t)vr[c][e] | ((uint32_t)vi[c][e] << 16);
        }
      }
    }
  }
  __syncthreads();
  // RU templates per A fragment, RBN fragments per wave and k-step
  constexpr int RU = CX ? 32 : 16, RBN = CX ? 1 : WT_ROWB;
  const u16x8* __restrict__ cpk = static_cast<const u16x8*>(CX ? a.cpkc : a.cpk);
  const int ntt = a.Tp / TILE_T;
  const int64_t cplane = (int64_t)ntt * (TILE_T / RU) * KB * 64;
  // A fragments of G k-steps (a group) go into a ring of D + 1 register
  // buffers D groups before their MFMAs; B fragments come from LDS just
  // before use.  The first D groups of the next template tile are loaded
  // before the current tile's epilogue (after its threshold loads), so a
  // short k-loop (small rank) does not start every tile with a full load
  // latency.  A long k-loop runs a branch-free steady state, with the same D
  // groups in flight on every path into it (otherwise the compiler's wait
  // counts would stall on the loads just issued).
  // (register budget at two waves per SIMD; the compact form's A ring is half as large)
  constexpr int G = (CB == 4 || NP == 2) ? 1 : 2;
  constexpr int D = 3;                              // groups in flight
  const int ng = KB / G;
  // Sample row s = 32 cb + (lane & 31) has swizzle 8 cb + 4 h, h = (lane & 31) / 16
  // (disjoint bits), and the fragment's first word is 8 (p Kp / 8 + kb) + 4 (lane / 32):
  // the swizzled word is 8 ((p Kp / 8 + kb) ^ cb) + 4 ((lane / 32) ^ h), so the lane's part
  // goes into its base pointer and only an XOR with the unrolled cb remains per read.
  const uint16_t* zl = zs + (lane & 31) * RS + 8 * ((lane >> 5) ^ ((lane & 31) >> 4));
  const int K8 = Kp >> 3;
  auto tile_rb0 = [&](int t) { return t * (TILE_T / RU) + wave * RBN; };   // in units of RU templates
  u16x8 fa[D + 1][G][NP][RBN];
  const u16x8* pa = nullptr;
  auto load = [&](int s) {   // the group at pa, then advance pa
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int rb = 0; rb < RBN; ++rb) fa[s][g][p][rb] = pa[p * cplane + ((int64_t)rb * KB + g) * 64];
    pa += G * 64;
  };
  // the first D groups of a tile (pa at its start): all of them on the steady
  // path (ng >= 2 D + 1), the ones that exist otherwise
  auto first_groups = [&](bool steady) {
    if (steady) {
#pragma unroll
      for (int s = 0; s < D; ++s) {
        load(s);
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
#pragma unroll
      for (int s = 0; s < D; ++s)
        if (s < ng) load(s);
    }
  };
  f32x16 acc[WT_ROWB][CB];
  auto read_b = [&](int kb, u16x8 (&bv)[NP][CB]) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
        bv[p][cb] = *reinterpret_cast<const u16x8*>(zl + cb * 32 * RS + 16 * ((p * K8 + kb) ^ cb));
  };
  auto step = [&](const u16x8 (&av)[NP][RBN], int kb) {
    u16x8 bv[NP][CB];
    read_b(kb, bv);
    if constexpr (CX) {
      u16x8 ai[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) ai[p] = im_operand(av[p][0]);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) {
        acc[0][cb] = kstep<DT>(av[0][0], av[NP - 1][0], bv[0][cb], bv[NP - 1][cb], acc[0][cb]);
        acc[1][cb] = kstep<DT>(ai[0], ai[NP - 1], bv[0][cb], bv[NP - 1][cb], acc[1][cb]);
      }
    } else {
#pragma unroll
      for (int rb = 0; rb < WT_ROWB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
          acc[rb][cb] = kstep<DT>(av[0][rb], av[NP - 1][rb], bv[0][cb], bv[NP - 1][cb], acc[rb][cb]);
    }
  };
  auto mma = [&](int s, int grp) {
#pragma unroll
    for (int g = 0; g < G; ++g) step(fa[s][g], grp * G + g);
  };
  // one template tile: the groups (the first D already loaded), the last
  // KB mod G k-step, then the next tile's first groups and the epilogue
  auto tile = [&](int tt, bool steady) {
    const int rb0 = tile_rb0(tt);
    const u16x8* __restrict__ ap = cpk + (int64_t)rb0 * KB * 64 + lane;
#pragma unroll
    for (int rb = 0; rb < WT_ROWB; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = (f32x16){};
    int gi = 0;
    if (steady) {
      // groups gi .. gi + D - 1 sit in buffers 0 .. D - 1; sub-step s loads
      // group gi + s + D into buffer (s + D) mod (D + 1) and runs group gi + s
      do {
#pragma unroll
        for (int s = 0; s <= D; ++s) {
          load((s + D) % (D + 1));
          __builtin_amdgcn_sched_barrier(0);
          mma(s, gi + s);
          __builtin_amdgcn_sched_barrier(0);
        }
        gi += D + 1;
      } while (gi + 2 * D + 1 <= ng);
    }
    // at most 2 D groups remain (gi .. gi + 2 D - 1), the first D already
    // loaded; group gi + t is in buffer t mod (D + 1)
#pragma unroll
    for (int t = 0; t < 2 * D; ++t) {
      if (t < D && gi + t + D < ng) load((t + D) % (D + 1));
      if (gi + t < ng) mma(t % (D + 1), gi + t);
    }
    if (KB % G) {
      u16x8 av[NP][RBN];
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int rb = 0; rb < RBN; ++rb) av[p][rb] = ap[p * cplane + ((int64_t)rb * KB + KB - 1) * 64];
      step(av, KB - 1);
    }
    float th[WT_ROWB][8];
    if constexpr (CX)
      epi_thresholds_c(a, rb0 * 32, th);
    else
      epi_thresholds<WT_ROWB>(a, rb0, th);
    const bool more = tt + 1 < ntt && tile_rb0(tt + 1) * RU < a.T;
    if (more) {
      pa = cpk + (int64_t)tile_rb0(tt + 1) * KB * 64 + lane;
      first_groups(steady);
    }
    if constexpr (CX)
      epilogue_c<CB>(a, acc, rb0 * 32, q0, stg, th);
    else
      epilogue<WT_ROWB, CB>(a, acc, rb0, q0, stg, th);
    return more;
  };
  if (tile_rb0(0) * RU < a.T) {
    pa = cpk + (int64_t)tile_rb0(0) * KB * 64 + lane;
    if (ng >= 2 * D + 1) {
      first_groups(true);
      for (int tt = 0; tile(tt, true); ++tt) {
      }
    } else {
      first_groups(false);
      for (int tt = 0; tile(tt, false); ++tt) {
      }
    }
  }
  if (stg.n > 0) stage_flush(a, stg, lane);
}

// ------------------------------------------------------------------ packing
__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint16_t to16(float x, int dtype) {
  if (dtype == 1 || dtype == 3) return bf16_rne(x);
  _Float16 h = (_Float16)x;
  return __builtin_bit_cast(uint16_t, h);
}

// Realified A entry for lane-row r (0..31) within a 16-template block and
// reduction index t (0 = Re beta_k, 1 = Im beta_k).
__device__ __forceinline__ float a_entry(const float2* C, int T, int K, int rb, int r, int k,
                                         int t, const float* row_scale) {
  const int j = rb * 16 + (r >> 1);
  if (j >= T || k >= K) return 0.f;
  float2 c = C[(int64_t)j * K + k];
  if (row_scale) {
    c.x *= row_scale[j];
    c.y *= row_scale[j];
  }
  const int part = r & 1;
  if (part == 0) return t == 0 ? c.x : -c.y;
  return t == 0 ? c.y : c.x;
}

// FP32 A, packed [32-template tile][k-pair][lane][4]: entries (block 0, k),
// (block 1, k), (block 0, k + 1), (block 1, k + 1) for k = 2 * pair; a k = K
// entry (K odd) is zero.
__global__ void k_pack_f32(const float2* C, int T, int Tp, int K, float* out) {
  const int KP = (K + 1) / 2;
  const int64_t total = (int64_t)(Tp / 32) * KP * 64 * 4;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(i & 3);
    const int l = (int)((i >> 2) & 63);
    const int64_t tk = i >> 8;
    const int kp = (int)(tk % KP);
    const int tile = (int)(tk / KP);
    out[i] = a_entry(C, T, K, 2 * tile + (e & 1), l & 31, 2 * kp + (e >> 1), l >> 5, nullptr);
  }
}

// C for k_recon_f32_3m: [32-template tile][k-pair][lane] float4 (Cr, Ci, Cr + Ci, 0)
// of template l % 32 of the tile and k = 2 pair + l / 32 (zero past T or K).
__global__ void k_pack_f32_3m(const float2* C, int T, int Tp, int K, float4* out) {
  const int KP = (K + 1) / 2;
  const int64_t total = (int64_t)(Tp / 32) * KP * 64;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(i & 63);
    const int64_t tk = i >> 6;
    const int kp = (int)(tk % KP);
    const int tile = (int)(tk / KP);
    const int j = tile * 32 + (l & 31), k = 2 * kp + (l >> 5);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (j < T && k < K) {
      const float2 c = C[(int64_t)j * K + k];
      v = make_float4(c.x, c.y, c.x + c.y, 0.f);
    }
    out[i] = v;
  }
}

__global__ void k_pack_16(const float2* C, int T, int Tp, int K, int Kp, int dtype,
                          const float* row_scale, uint16_t* out) {
  const int KB = Kp / 8;
  const int64_t total = (int64_t)(Tp / 16) * KB * 64 * 8;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(i & 7);
    const int l = (int)((i >> 3) & 63);
    const int64_t rkb = i >> 9;
    const int kb = (int)(rkb % KB);
    const int rb = (int)(rkb / KB);
    const int red = 8 * (l >> 5) + e;          // reduction index within the 16-step
    const int k = kb * 8 + (red >> 1);
    const float x = a_entry(C, T, K, rb, l & 31, k, red & 1, row_scale);
    const uint16_t h = to16(x, dtype);
    out[i] = h;
    if (dtype == 3) out[total + i] = bf16_rne(x - __uint_as_float((uint32_t)h << 16));   // lo plane
  }
}

// C for the compact 16-bit form: [32-template block][k-step][lane][8] per
// plane, lane l holding template 32 block + l % 32 and, for e = 0..7, entry
// Re C (e even) or -Im C (e odd) of complex k = 8 kb + 4 (l / 32) + e / 2
// (row-scaled for FP16; zero past T or K); the split form's lo plane follows.
__global__ void k_pack_16c(const float2* C, int T, int Tp, int K, int Kp, int dtype, const float* row_scale,
                           uint16_t* out) {
  const int KB = Kp / 8;
  const int64_t total = (int64_t)(Tp / 32) * KB * 64 * 8;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(i & 7);
    const int l = (int)((i >> 3) & 63);
    const int64_t bkb = i >> 9;
    const int kb = (int)(bkb % KB);
    const int blk = (int)(bkb / KB);
    const int j = blk * 32 + (l & 31), k = kb * 8 + 4 * (l >> 5) + (e >> 1);
    float x = 0.f;
    if (j < T && k < K) {
      float2 c = C[(int64_t)j * K + k];
      if (row_scale) {
        c.x *= row_scale[j];
        c.y *= row_scale[j];
      }
      x = (e & 1) ? -c.y : c.x;
    }
    const uint16_t h = to16(x, dtype);
    out[i] = h;
    if (dtype == 3) out[total + i] = bf16_rne(x - __uint_as_float((uint32_t)h << 16));   // lo plane
  }
}

}  // namespace

int recon_variants(int dtype) { return dtype == 0 ? 7 : 5; }

double recon_mfma_flop(const GemmArgs& a) {
  const double N = (double)a.N;
  auto up = [](int x, int m) { return (double)((x + m - 1) / m * m); };
  if (a.dtype == 0 && a.variant == 6)   // three real products per k-pair over 32-template tiles
    return 6.0 * up(a.T, 32) * up(a.K, 2) * N;
  if (a.dtype == 0)                     // realified, 16-template blocks (a block of padding only is skipped)
    return 8.0 * up(a.T, 16) * a.K * N;
  // 16-bit: waves of 32 templates (skipped when all padding), k-steps of 8
  // complex values; the split-BF16 form issues three products per step
  return 8.0 * up(a.T, 32) * a.Kp * N * (a.dtype == 3 ? 3.0 : 1.0);
}

hipError_t launch_recon_gemm(const GemmArgs& a, hipStream_t st) {
  if (a.Tp % TILE_T != 0 || a.N % 128 != 0) return hipErrorInvalidValue;
  if (a.dtype == 0 && a.variant == 6) {   // three real products per k-pair (Gauss)
    if (a.cpk3 == nullptr) return hipErrorInvalidValue;
    const int64_t nwg = (int64_t)((a.T + 31) / 32) * ((a.N + WAVES * 128 - 1) / (WAVES * 128));
    const int64_t launch = ((nwg + 7) / 8) * 8;
    hipLaunchKernelGGL(k_recon_f32_3m, dim3((unsigned)launch), dim3(256), 0, st, a);
    return hipGetLastError();
  }
  if (a.dtype == 0 && a.variant >= 4) {   // 64 templates x 128 samples per wave: variant 4 = G 2, 5 = G 4
    // The whole 64-template tiles run here; the T mod 64 templates left
    // would run as a one- or two-block tile at one wave per SIMD, whose few
    // MFMAs per load cannot cover the load latency (measured: as long as a
    // full tile), so they run as the 32-template kernel's tiles, a second
    // launch on the same template-shifted arguments.
    const int full = (a.T / 64) * 64;
    if (full > 0) {
      GemmArgs a1 = a;
      a1.T = full;
      const int64_t nwg = (int64_t)(full / 64) * ((a.N + WAVES * 128 - 1) / (WAVES * 128));
      const int64_t launch = ((nwg + 7) / 8) * 8;
      if (a.variant == 4)
        hipLaunchKernelGGL((k_recon_f32_w64<4, 2>), dim3((unsigned)launch), dim3(256), 0, st, a1);
      else
        hipLaunchKernelGGL((k_recon_f32_w64<4, 4>), dim3((unsigned)launch), dim3(256), 0, st, a1);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (a.T > full) {
      GemmArgs a2 = a;                   // templates [full, T): every per-template array shifted
      a2.T = a.T - full;
      a2.cpk = static_cast<const float4*>(a.cpk) + (int64_t)(full / 32) * ((a.K + 1) / 2) * 64;
      a2.thr2_row = a.thr2_row + full;
      a2.tmpl_base = a.tmpl_base + full;
      a2.tmpl_count = a.tmpl_count + full;
      if (a.rho_out) a2.rho_out = a.rho_out + (int64_t)full * a.N;
      if (a.row_inv) a2.row_inv = a.row_inv + full;
      const int64_t nwg = (int64_t)((a2.T + 31) / 32) * ((a.N + WAVES * 128 - 1) / (WAVES * 128));
      const int64_t launch = ((nwg + 7) / 8) * 8;
      hipLaunchKernelGGL((k_recon_f32<4, 2>), dim3((unsigned)launch), dim3(256), 0, st, a2);
    }
    return hipGetLastError();
  }
  if (a.dtype == 0) {   // per-wave tiles: 32 templates x 32 CB samples, G k-steps per pipeline group:
                        // variant 0 = CB 4 / G 2, 1 = 4 / 4, 2 = 2 / 2, 3 = 2 / 4
    const int cbw = a.variant < 2 ? 4 : 2;
    const int TN = cbw * 32;
    const int64_t nwg = (int64_t)((a.T + 31) / 32) * ((a.N + WAVES * TN - 1) / (WAVES * TN));
    const int64_t launch = ((nwg + 7) / 8) * 8;
    if (a.variant == 0)
      hipLaunchKernelGGL((k_recon_f32<4, 2>), dim3((unsigned)launch), dim3(256), 0, st, a);
    else if (a.variant == 1)
      hipLaunchKernelGGL((k_recon_f32<4, 4>), dim3((unsigned)launch), dim3(256), 0, st, a);
    else if (a.variant == 2)
      hipLaunchKernelGGL((k_recon_f32<2, 2>), dim3((unsigned)launch), dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL((k_recon_f32<2, 4>), dim3((unsigned)launch), dim3(256), 0, st, a);
    return hipGetLastError();
  }
  // 16-bit: variant 0 / 2 stage a 64 / 128-sample Z tile in LDS (when it fits),
  // variant 1 loads fragments directly; variants 3 / 4 are 0 / 2 with compact
  // coefficients (a.cpkc)
  const int np = a.dtype == 3 ? 2 : 1;
  const bool cx = a.variant >= 3;
  if (cx && a.cpkc == nullptr) return hipErrorInvalidValue;
  int tns = (a.variant == 2 && a.dtype != 3) ? 128 : 64;   // (the split-BF16 operands do not fit 128)
  // (the compact split-BF16 kernel at 128 samples would spill)
  if (a.variant == 4 && a.dtype != 3 && (size_t)128 * zs_row_u16(np, a.Kp) * 2 + kStageBytes <= kLdsMax) tns = 128;
  const size_t lds = (size_t)tns * zs_row_u16(np, a.Kp) * 2;   // dynamic part (the staging is static)
  if (a.variant != 1 && lds + kStageBytes <= kLdsMax) {
    // the dynamic-LDS limit is raised once per device (calls on several
    // devices, from several threads, each see their own device's flag)
    static std::mutex attr_mu;
    static uint64_t attr_set = 0;   // bit d: done on device d
    int dev = 0;
    {
      const hipError_t e = hipGetDevice(&dev);
      if (e != hipSuccess) return e;
    }
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    {
      std::lock_guard<std::mutex> lock(attr_mu);
      if (!(attr_set >> dev & 1u)) {
        const void* fns[] = {reinterpret_cast<const void*>(&k_recon_16_lds<1, 2, false>),
                             reinterpret_cast<const void*>(&k_recon_16_lds<2, 2, false>),
                             reinterpret_cast<const void*>(&k_recon_16_lds<3, 2, false>),
                             reinterpret_cast<const void*>(&k_recon_16_lds<1, 4, false>),
                             reinterpret_cast<const void*>(&k_recon_16_lds<2, 4, false>),
                             reinterpret_cast<const void*>(&k_recon_16_lds<1, 2, true>),
                             reinterpret_cast<const void*>(&k_recon_16_lds<2, 2, true>),
                             reinterpret_cast<const void*>(&k_recon_16_lds<3, 2, true>),
                             reinterpret_cast<const void*>(&k_recon_16_lds<1, 4, true>),
                             reinterpret_cast<const void*>(&k_recon_16_lds<2, 4, true>)};
        for (const void* f : fns) {
          const hipError_t e =
              hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLdsMax - kStageBytes));
          if (e != hipSuccess) return e;
        }
        attr_set |= uint64_t(1) << dev;
      }
    }
    const unsigned grid = (unsigned)(a.N / tns);
#define RB_LAUNCH16(DT, CB, CX_) hipLaunchKernelGGL((k_recon_16_lds<DT, CB, CX_>), dim3(grid), dim3(256), lds, st, a)
    if (cx) {
      if (tns == 128) {
        if (a.dtype == 1)
          RB_LAUNCH16(1, 4, true);
        else
          RB_LAUNCH16(2, 4, true);
      } else {
        if (a.dtype == 1)
          RB_LAUNCH16(1, 2, true);
        else if (a.dtype == 2)
          RB_LAUNCH16(2, 2, true);
        else
          RB_LAUNCH16(3, 2, true);
      }
    } else if (tns == 128) {
      if (a.dtype == 1)
        RB_LAUNCH16(1, 4, false);
      else
        RB_LAUNCH16(2, 4, false);
    } else {
      if (a.dtype == 1)
        RB_LAUNCH16(1, 2, false);
      else if (a.dtype == 2)
        RB_LAUNCH16(2, 2, false);
      else
        RB_LAUNCH16(3, 2, false);
    }
#undef RB_LAUNCH16
    return hipGetLastError();
  }
  const int64_t nwg = (int64_t)(a.Tp / TILE_T) * (a.N / TILE_N);
  const int64_t launch = ((nwg + 7) / 8) * 8;
  if (a.dtype == 1)
    hipLaunchKernelGGL(k_recon_16<1>, dim3((unsigned)launch), dim3(256), 0, st, a);
  else if (a.dtype == 2)
    hipLaunchKernelGGL(k_recon_16<2>, dim3((unsigned)launch), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_recon_16<3>, dim3((unsigned)launch), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_pack_c(const float2* C, int T, int Tp, int K, int Kp, int dtype,
                         const float* row_scale, void* cpk, hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_pack_f32, dim3(1024), dim3(256), 0, st, C, T, Tp, K, static_cast<float*>(cpk));
  else
    hipLaunchKernelGGL(k_pack_16, dim3(1024), dim3(256), 0, st, C, T, Tp, K, Kp, dtype, row_scale,
                       static_cast<uint16_t*>(cpk));
  return hipGetLastError();
}

hipError_t launch_pack_c16c(const float2* C, int T, int Tp, int K, int Kp, int dtype, const float* row_scale,
                            void* cpkc, hipStream_t st) {
  if (dtype < 1 || dtype > 3 || Tp % 32 != 0 || Kp % 8 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pack_16c, dim3(1024), dim3(256), 0, st, C, T, Tp, K, Kp, dtype, row_scale,
                     static_cast<uint16_t*>(cpkc));
  return hipGetLastError();
}

hipError_t launch_pack_c3(const float2* C, int T, int Tp, int K, void* cpk3, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_f32_3m, dim3(1024), dim3(256), 0, st, C, T, Tp, K, static_cast<float4*>(cpk3));
  return hipGetLastError();
}

int gemm_tile_templates() { return TILE_T; }

}  // namespace rbmf
