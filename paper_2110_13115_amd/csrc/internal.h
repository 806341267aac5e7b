// Internal interfaces between the C-ABI host layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>

namespace rbmf {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
#define RB_HIP(call)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      ::rbmf::set_error(std::string(#call " failed: ") + hipGetErrorString(e_));        \
      return RB_ERR_DEVICE;                                                             \
    }                                                                                   \
  } while (0)

// ---------------------------------------------------------------- FFT plan
// N = N1 * N2.  Pass 1: N2-point FFTs down the N1 columns of the [N2][N1]
// array (input index f = f1 + N1 f2), twiddle w_N^{f1 n2}, stored at
// n2 * N1 + f1.  Pass 2: N1-point FFTs along each row; the output at position
// q = n2 * N1 + n1 is time (or frequency) index n = n2 + N2 n1.
struct FftGeom {
  int64_t N;
  int log2N;
  int N1, N2;      // row length, column length
  int s_lo;        // split of the inter-pass twiddle exponent: lo table 2^s_lo entries
};

struct FftTables {   // device pointers, FP32 values from FP64 host math
  const float2* pyr;   // pyr[L + i] = e^{+2 pi i i / L}, L = 2..2048
  const float2* tlo;   // e^{+2 pi i e / N}, e < 2^s_lo
  const float2* thi;   // e^{+2 pi i (e << s_lo) / N}, e < N >> s_lo
};

struct FftTables64 {
  const double2* pyr;
  const double2* tlo;
  const double2* thi;
};

// n2log < 0: the balanced split N2 = 2^floor(log2 N / 2).
FftGeom make_geom(int64_t N, int n2log = -1);
bool geom_supported(const FftGeom& g);

// Pass-1 input variants.
// IN_CORR_H: IN_CORR with the intermediate stored as FP16 (Re, Im) pairs times
// the power of two hscale[0] (for bases whose Z is stored in 16 bits).
enum InKind { IN_CORR = 0, IN_REAL = 1, IN_DENSE = 2, IN_FOLD = 3, IN_CORR_H = 4 };
// Pass-2 output variants.
enum OutKind {
  OUT_Z32 = 0,       // planar FP32 Z: row 2v = Re, row 2v+1 = Im, row stride N
  OUT_Z16 = 1,       // planar 16-bit Z (bf16, f16, or bf16 hi + lo planes), same layout, values * zscale
  OUT_THRESH = 2,    // |x|^2 >= thr2: append trigger, per-vector count and max
  OUT_NATURAL = 3,   // complex64 natural order out[v][n]
  OUT_SPECTRUM = 4,  // forward transform of the strain: d[k - kb] = wd[k] X[k], band only
  OUT_TRANSPOSED = 5, // complex64 in the pass order out[v][q] (adjoint)
  OUT_ZBIN = 6,      // binned first stage: Z in zfine (complex64 or 16-bit pairs) with each pass-2 block's F
                     // rows adjacent per n1 (q = row0 N1 + n1 F + f, F = pass2_rows(N1)),
                     // plus sums over bin_g = min(F, bin_w) consecutive samples: the bin
                     // means in zout (planar, zdtype, plane stride N / bin_w) when
                     // bin_g == bin_w, else partial sums in zpart ([N2 / bin_g][N1]
                     // complex64 per vector)
  OUT_Z16_H = 7,     // OUT_Z16 from the FP16 intermediate of IN_CORR_H (its scale removed)
  OUT_ZBIN_H = 8     // OUT_ZBIN from the FP16 intermediate of IN_CORR_H (its scale removed)
};

struct TrigRec {     // device trigger record before sorting
  int32_t tmpl;
  int32_t sample;
  float re;
  float im;
};

struct PassArgs {
  FftGeom g;
  FftTables tw;
  FftTables64 tw64;          // FP64 tables (strain spectrum)
  double2* work64;           // FP64 intermediate (strain spectrum)
  const double* wd64;        // OUT_SPECTRUM: dt * sqrt(4 df / Sn[k]) from kb, FP64
  int sign;                  // +1 inverse (e^{+}), -1 forward
  int nvec;                  // vectors in this launch
  int vec_base;              // first vector (or first list entry)
  const int32_t* vec_list;   // optional gather list (device)
  const int32_t* d_count;    // optional device count: entries >= *d_count are skipped
  // pass-1 inputs
  const float2* d;           // IN_CORR: whitened data, band-packed from kb
  const float2* src;         // IN_CORR: vectors (stride nbs) / IN_DENSE: vectors (stride N)
  const float* real_in;      // IN_REAL
  int64_t kb;                // first stored bin
  int64_t nbs;               // stored bins per vector
  const int32_t* sup_lo;     // IN_CORR: per-vector first non-zero bin (absolute)
  const int32_t* sup_hi;     // IN_CORR: per-vector last non-zero bin
  int32_t band_lo, band_hi;  // IN_CORR when sup_* are NULL
  const float2* gfold;       // IN_FOLD: G[F] = sum_{r<w} e^{+2 pi i F r / (w g.N)}, F < (w/2) g.N
  int fold_half;             // IN_FOLD: w / 2 (folded bins per output below N/2)
  float fold_inv;            // IN_FOLD: 1 / w
  // intermediate [nvec][N] complex64 (FP16 pairs for IN_CORR_H / OUT_Z16_H)
  float2* work;
  const float* hscale;       // IN_CORR_H / OUT_Z16_H: device {s, 1 / s}
  // pass-2 outputs
  float* zout;               // OUT_Z32 / OUT_Z16 (as raw bytes for 16-bit)
  int zdtype;                // 0 f32, 1 bf16, 2 f16, 3 bf16 hi plane + bf16 lo plane
  float zscale;
  int64_t zplane;            // dtype 3: offset (16-bit elements) of the lo plane
  float thr2;                // OUT_THRESH: squared threshold
  TrigRec* trig;             // OUT_THRESH
  int64_t trig_cap;
  unsigned long long* trig_count;
  int32_t* tmpl_count;       // per template crossing counts
  unsigned long long* tmpl_max;  // per template packed (|x|^2 bits << 32 | ~n)
  void* zfine;               // OUT_ZBIN: Z for the fine reconstruction, N per vector:
  int zfine16;               //   complex64 (0) or 16-bit (Re, Im) pairs, bf16 (1) / f16 (2)
  float2* zpart;             // OUT_ZBIN: partial bin sums, N / bin_g per vector
  int bin_g;                 // OUT_ZBIN: samples per partial sum, min(F, bin_w)
  int bin_w;                 // OUT_ZBIN: samples per bin
  float2* cout;              // OUT_NATURAL / OUT_SPECTRUM / OUT_TRANSPOSED
  int32_t k_lo;              // OUT_SPECTRUM band
  int32_t k_hi;
};

// {s, 1 / s} of the FP16 intermediate for whitened data d (n bins): s is the
// largest power of two with 2 sqrt(N2) max|d| s <= 2^15, so every pass-1
// output of a unit-norm vector stays below 2^15 (Cauchy-Schwarz over the
// column's N2 terms, with a factor 2 for rounding of the norm).  part holds
// kHalfScaleParts floats of scratch.  Graph-capturable (two launches, no
// memset).
constexpr int kHalfScaleParts = 256;
hipError_t launch_half_scale(const float2* d, int64_t n, int n2, float* part, float* hs, hipStream_t stream);

// Launch pass 1 / pass 2 on `stream`.  Return hipSuccess or the launch error.
hipError_t launch_pass1(const PassArgs& a, InKind in, hipStream_t stream);
hipError_t launch_pass2(const PassArgs& a, OutKind out, hipStream_t stream);

// ---------------------------------------------------------------- GEMM
struct GemmArgs {
  int64_t N;
  int T, Tp;                 // templates, padded to the row tile
  int K, Kp;                 // basis rank, padded
  int dtype;                 // 0 f32, 1 bf16, 2 f16
  const void* cpk;           // packed realified coefficients
  const void* cpk3;          // FP32: C packed for the three-product kernel (Cr, Ci, Cr + Ci), or NULL
  const void* cpkc;          // 16-bit: C packed for the compact-coefficient variants, or NULL
  const void* z;             // planar Z [2Kp][N]
  const float* thr2_row;     // per-template squared threshold (16-bit scales folded in)
  int N1, N2;                // position q -> n = q / N1 + N2 * (q % N1)
  TrigRec* trig;
  int64_t trig_cap;
  unsigned long long* trig_count;
  int tmpl_base;             // global index of local template 0 (sub-bank bases)
  int32_t* tmpl_count;       // per local template (already offset by tmpl_base)
  float2* rho_out;           // debug: natural order T x N, or NULL
  const float* row_inv;      // per-template 1/scale applied to rho_out (16-bit), or NULL
  int variant;               // kernel variant (autotuned): see launch_recon_gemm
};
int recon_variants(int dtype);
hipError_t launch_recon_gemm(const GemmArgs& a, hipStream_t stream);
// Floating-point operations launch_recon_gemm(a) issues on the matrix cores,
// padding rows and reduction steps included.
double recon_mfma_flop(const GemmArgs& a);
// FP32 C for the three-product kernel: [Tp/32][ceil(K/2)][64] float4.
hipError_t launch_pack_c3(const float2* C, int T, int Tp, int K, void* cpk3, hipStream_t stream);
// 16-bit C for the compact-coefficient variants: [Tp/32][Kp/8][64][8] u16 per
// plane (two planes for the split form).
hipError_t launch_pack_c16c(const float2* C, int T, int Tp, int K, int Kp, int dtype, const float* row_scale,
                            void* cpkc, hipStream_t stream);
// Packs C (T x K complex, FP32 interleaved, device) into the kernel's layout.
hipError_t launch_pack_c(const float2* C, int T, int Tp, int K, int Kp, int dtype,
                         const float* row_scale, void* cpk, hipStream_t stream);

// ---------------------------------------------------------------- triggers
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
// list -> heavy (counts >= thresh) / light lists; n_out[2] (zeroed) receives their lengths
hipError_t launch_split_list(const int32_t* list, int64_t n, const int32_t* counts, int thresh, int32_t* heavy,
                             int32_t* light, int32_t* n_out, hipStream_t s);
// summary (device, 3 x int64): total, number of listed templates, max count
hipError_t launch_scan_counts(const int32_t* counts, int T, int32_t* offsets, int32_t* fill,
                              int32_t* list, int64_t* summary, hipStream_t s);
// n_dev / summary_dev: optional device-side counts (graph-capturable form);
// n / nlist are then upper bounds used to size the launch.
hipError_t launch_scatter_triggers(const TrigRec* in, int64_t n, const int64_t* n_dev,
                                   const int32_t* offsets, int32_t* fill, TrigRec* out,
                                   hipStream_t s);
hipError_t launch_segment_sort(TrigRec* recs, TrigRec* tmp, const int32_t* offsets,
                               const int32_t* counts, const int32_t* list, int nlist, void* out,
                               const int64_t* summary_dev, int64_t out_cap, hipStream_t s);
// keeps in[i] (rb_trigger, n of them) with sample + shift in [lo, hi), shifted, appended in order at
// out[*n_out ...] (entries beyond cap are counted, not written); *n_out is advanced
hipError_t launch_window(const void* in, int64_t n, int64_t shift, int64_t lo, int64_t hi, void* out, int64_t cap,
                         int64_t* n_out, hipStream_t s);
hipError_t launch_peaks_from_max(const unsigned long long* tmax, int T, void* out_peaks,
                                 hipStream_t s);
hipError_t launch_cluster_peaks(const void* trig, int64_t n, int W, int64_t N, uint8_t* is_peak,
                                hipStream_t s);
struct SparseArgs {
  int64_t N;
  int s_lo;
  const float2* tlo;          // FP32 inter-pass twiddle tables (as the FFT's)
  const float2* thi;
  const int32_t* list;        // selected templates
  const int32_t* d_count;     // optional device count of `list`
  const int64_t* n1_dev;      // optional device stage-1 total: nothing runs when it exceeds n1_cap
  int64_t n1_cap;             //   (the grouped records were not written)
  const int32_t* offsets;     // stage-1 records grouped by template: offsets / counts
  const int32_t* counts;
  const TrigRec* recs;
  const float2* d;            // whitened data from kb
  const float2* tmpl;         // bank templates (stride nbs, from kb)
  int64_t kb, nbs;
  const int32_t* sup_lo;
  const int32_t* sup_hi;
  float thr2;                 // squared final threshold
  TrigRec* out;
  int64_t out_cap;
  unsigned long long* out_count;
  int32_t* tmpl_count;
  unsigned long long* tmpl_max;
  const int32_t* goff;        // optional: workgroup b takes group b - goff[i] of list[i] (goff[i] <= b < goff[i + 1])
  int32_t nlist;              //   over the nlist listed templates (else: gridDim.y groups per template)
};
// goff[0..n]: exclusive prefix sums of ceil(counts[list[i]] / per) (goff[n] = total).
hipError_t launch_group_offsets(const int32_t* list, int n, const int32_t* counts, int per, int32_t* goff,
                                hipStream_t s);
// grid: listed templates (upper bound with d_count); groups: workgroups that
// share one template's crossings (each takes every groups-th group of 8).
hipError_t launch_sparse_exact(const SparseArgs& a, int grid, int groups, hipStream_t s);
int sparse_crossings_per_group();

// ---------------------------------------------------------------- binned first stage
// Rows of one pass-2 workgroup (consecutive samples of an n1 slice).
inline int pass2_rows(int N1) { return N1 >= 4096 ? 1 : 4096 / N1; }

struct BinReduceArgs {
  const float2* part;        // OUT_ZBIN partial sums, [vec][N2/G][N1]
  int64_t N;
  int N1, N2;
  int G, w;                  // samples per partial sum, per bin (powers of two, G | w)
  int vec_base, nvec;
  void* zavg;                // planar bin means [2Kp][N/w] in `dtype` (as the GEMM's Z)
  int dtype;                 // 0 f32, 1 bf16, 2 f16, 3 bf16 hi + lo planes
  float zscale;              // 16-bit: value scale
  int64_t zplane;            // dtype 3: offset (16-bit elements) of the lo plane
};
hipError_t launch_bin_reduce(const BinReduceArgs& a, hipStream_t s);
hipError_t launch_copy_u64(const unsigned long long* src, unsigned long long* dst, hipStream_t s);

struct FineArgs {
  const void* z;             // OUT_ZBIN Z, row k of stride N: complex64, or 16-bit pairs
  int z16;                   //   0 complex64, 1 bf16 pairs, 2 f16 pairs
  int64_t N;
  int N1, N2, F;             // FFT split; F = pass2_rows(N1)
  int K, w;
  const float2* C;           // local T x K complex64, C = conj(c), unscaled
  int t0;                    // global index of local template 0
  const TrigRec* bins;       // triggering (template, bin) records: sample = bin index
  const unsigned long long* begin;   // device: first record of this basis (NULL: begin_h)
  const unsigned long long* end;     // device: records appended so far (NULL: end_h)
  int64_t begin_h, end_h;            // host-known record range
  int64_t bins_cap;
  float thr_sq;              // candidate threshold, squared
  TrigRec* out;
  int64_t out_cap;
  unsigned long long* out_count;
  int32_t* tmpl_count;       // per global template
};
// grid: workgroups of four waves, each wave taking every (4 grid)-th record
hipError_t launch_fine_recon(const FineArgs& a, int grid, hipStream_t s);
// n_bound: an upper bound of the record count used to size the launch
hipError_t launch_select_final(const TrigRec* in, const unsigned long long* n_in, int64_t cap_in,
                               const float* inv_scale, float thr2_sq, TrigRec* out, int64_t out_cap,
                               unsigned long long* out_count, int32_t* tmpl_count,
                               unsigned long long* tmpl_max, int64_t n_bound, hipStream_t s);

// ---------------------------------------------------------------- FP64 complex GEMM
// C[m][n] (+)= sum_k opA(A)[m][k] * opB(B)[k][n], complex128 accumulation.
// Operands are complex64 or complex128 with arbitrary row/col strides (in
// elements) and an optional conjugation.  `workspace` (workspace_elems
// complex128) holds split-reduction partials; it may be NULL (no split).
struct ZOperand {
  const void* p;
  int is_c64;        // 1: complex64 elements, 0: complex128
  int64_t rs, cs;    // strides of (row, col) of the *logical* operand
  int conj;
};
hipError_t launch_zgemm(int64_t M, int64_t Nn, int64_t Kd, ZOperand A, ZOperand B, double2* C,
                        int64_t ldc, int accumulate, double2* workspace, int64_t workspace_elems,
                        hipStream_t s);
hipError_t launch_c128_to_c64_rows(const double2* in, int64_t rows, int64_t cols, int64_t ld_in,
                                   const double* row_scale, int conj, float2* out, int64_t ld_out,
                                   hipStream_t s);
hipError_t launch_basis_rows(const double2* BS, int64_t nb, int K, int64_t ld, const double* scale,
                             int64_t off, int64_t nbs, float2* out, hipStream_t s);
hipError_t launch_row_norms(const float2* w, int64_t rows, int64_t len, int64_t ld, double* out,
                            hipStream_t s);
// B: nt x K complex128 (row-major); idx[f] in [0, nt - 2] for f < nb.
hipError_t launch_interp_rows(const double2* B, int64_t nt, int K, const int32_t* idx, const double* frac,
                              const double* r, const double* scale, int64_t nb, double2* out, hipStream_t s);

// ---------------------------------------------------------------- allocation-free entry point
// Bytes of the fixed per-GPU device scratch of mf_full_noalloc.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
// Device address of `device`'s copy of that scratch, looked up once per device
// (call with the device current).
hipError_t noalloc_scratch_init(int device, void** out);
// Held by an mf_full_noalloc call for as long as its work uses the scratch.
std::mutex& noalloc_scratch_lock(int device);

// ---------------------------------------------------------------- misc
hipError_t launch_check_finite(const float* x, int64_t n, int64_t* flag, hipStream_t s);
// dtype 0 FP32, 1 BF16, 2 FP16 planar Z (one plane) -> complex64 natural order
hipError_t launch_z_to_natural(const void* z, int dtype, float inv_scale, int64_t N, int K, int N1,
                               int N2, float2* out, hipStream_t s);

// ---------------------------------------------------------------- adjoint
hipError_t launch_rho_at(const float* z, int64_t N, int K, int N1, int N2, const float2* C,
                         const int32_t* tmpl, const int32_t* samp, int64_t n, float2* rho,
                         hipStream_t s);
hipError_t launch_grad_c(const float* z, int64_t N, int K, int N1, int N2, const int32_t* order,
                         const int32_t* seg_off, int nseg, const int32_t* tmpl,
                         const int32_t* samp, const float2* rho, const float* g, float2* gC,
                         hipStream_t s);
hipError_t launch_scatter_a(int K, int64_t N, const int32_t* order, const int32_t* seg_off, int nseg,
                            const int32_t* tmpl, const int32_t* samp, const float2* rho,
                            const float* g, const float2* C, float2* A, hipStream_t s);
hipError_t launch_bsum(const float2* Ahat, const float2* P, const double* wd, int K, int64_t N,
                       int64_t kb, int64_t nbs, int64_t k_lo, int64_t k_hi, float2* B,
                       hipStream_t s);
hipError_t launch_real2(const float2* x, int64_t N, float* out, hipStream_t s);

// ---------------------------------------------------------------- refinement
// Per trigger (local template rows[i], sample samp[i]; n triggers): the m
// nearest bank neighbours by |<c_j, c_l>|, an orthonormal basis of the span
// of their coefficient rows and the trigger's own, and `iters` steps of
// projected gradient ascent of |rho|^2 from C_j.  Scratch: ov (n x T
// doubles), Q (n x (m + 1) x K complex128).  Outputs: c_out (n x K),
// nbr_out (n x m global indices), p_out (n x 2).
int refine_max_rank();
hipError_t launch_refine(const float* z, int64_t N, int N1, int N2, int K, int T, int t0, const float2* C,
                         const int32_t* rows, const int32_t* samp, int n, int m, int iters, double* ov,
                         double2* Q, float2* c_out, int32_t* nbr_out, float* p_out, hipStream_t s);

}  // namespace rbmf
