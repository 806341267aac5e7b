/*
 * rbmf.h -- C ABI of the reduced-basis hierarchical matched filter for
 * AMD Instinct MI355X (gfx950).
 *
 * The search it implements (Dhurkunde, Fehrmann & Nitz, "A hierarchical
 * approach to matched filtering using a reduced basis", arXiv:2110.13115):
 *
 *   - the noise-weighted inner product <s|h> = 4 int s~ h~* / Sn df
 *     (Sec. II, Eq. MF_def) and the SNR normalised by <h|h>^{1/2} with the
 *     unknown phase maximised by the modulus (Eq. SNR_def and the text after
 *     Eq. hf_eqn);
 *   - the SNR time series of one template by an inverse FFT of the weighted
 *     correlation (Eq. IFFT); a trigger is a sample whose SNR reaches a
 *     threshold (Sec. II);
 *   - an orthonormal basis of the whitened, unit-norm bank from its
 *     covariance / SVD (Sec. II.A, Eqs. Eq-PCA, Eq-SVD; Sec. III.B), truncated
 *     by the retained energy (Eq. SNR_loss);
 *   - per-basis filter outputs beta_k = IFFT(<s|p_k>) and the reconstruction
 *     rho_j = sum_k c*_{jk} beta_k (Eqs. basis_SNR, Beta_eqn);
 *   - a two-stage hierarchy (Sec. III.C): a first stage over the whole bank
 *     with a lowered threshold, and an exact second stage restricted to what
 *     the first stage selected.
 *
 * Conventions shared by every call
 * --------------------------------
 *   Grid      N samples (a power of two, 2^12..2^21) at fs Hz; dt = 1/fs,
 *             df = fs/N.  Band: bins k_lo = ceil(f_low/df) .. N/2-1
 *             inclusive (DC and Nyquist excluded).
 *   Spectra   s~[k] = dt * sum_n s[n] e^{-2 pi i k n/N}.
 *   Filter    rho_j[n] = 4 df sum_{k in band} s~[k] conj(h_j[k]) / Sn[k]
 *                        e^{+2 pi i k n/N} / sigma_j,
 *             sigma_j^2 = 4 df sum_{k in band} |h_j[k]|^2 / Sn[k];
 *             SNR = |rho_j[n]|, phase = arg rho_j[n].
 *   Pointers  "host or device" arguments are classified with
 *             hipPointerGetAttributes; device pointers must belong to the
 *             context's device.  Host arrays are read/written synchronously.
 *   Streams   all device work of a context is ordered on the stream given to
 *             rb_ctx_create (NULL = the null stream).  Calls that return
 *             counts synchronise that stream before returning.
 *   Errors    every call returns rb_status and never aborts; argument checks
 *             run on the host before any device work.  rb_last_error() gives a
 *             thread-local message for the last failure.
 *   Ownership the caller owns every array it passes; the library copies what
 *             it keeps into handles.  Handles own their device memory and are
 *             freed explicitly; free banks and bases before their context.
 *   Threads   one context per host thread; handles are not thread-safe.
 */
#ifndef RBMF_H
#define RBMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RB_OK = 0,
  RB_ERR_ARG = 1,          /* invalid argument (shape, range, null, PSD)      */
  RB_ERR_OOM = 2,          /* device or host allocation failed                 */
  RB_ERR_DEVICE = 3,       /* a HIP runtime call failed                        */
  RB_ERR_CAPACITY = 4,     /* output buffer too small; *n_out = required size  */
  RB_ERR_NUMERIC = 5,      /* non-finite input or degenerate numerics          */
  RB_ERR_UNSUPPORTED = 6,  /* valid but not supported by this build            */
  RB_ERR_CALLBACK = 7      /* the bank fill callback returned non-zero         */
} rb_status;

/* Storage type of the reconstruction operands C and Z (accumulation is FP32
 * in every case; basis construction, sigma and PSD products are FP64).
 * RB_BF16X3 keeps FP32 accuracy on the BF16 matrix cores: every FP32 value x
 * of C and Z is stored as hi = bf16(x) and lo = bf16(x - hi), and the product
 * sums the three leading partial products Ch Zh + Ch Zl + Cl Zh (the dropped
 * Cl Zl and the rounding of lo are ~2^-16 relative to each term). */
typedef enum { RB_F32 = 0, RB_BF16 = 1, RB_F16 = 2, RB_BF16X3 = 3 } rb_dtype;

/* Second-stage variant of rb_filter. */
typedef enum {
  RB_STAGE2_FULL = 0,      /* full matched filter (all N samples) of every
                              template with a first-stage crossing            */
  RB_STAGE2_SPARSE = 1,    /* exact SNR evaluated only at the first-stage
                              crossing samples (direct frequency sums)        */
  RB_STAGE2_AUTO = 2,      /* per template: FULL when it has at least
                              RBMF_STAGE2_SPLIT (default 32) first-stage
                              crossings, SPARSE otherwise (rb_filter only;
                              rb_filter_batch returns RB_ERR_UNSUPPORTED)     */
  RB_STAGE2_RECON = 3      /* the paper's own second stage (Sec. III.C): no
                              exact filter; the final triggers are the
                              candidates whose reconstructed |rho_RB| reaches
                              thr2, with that SNR (rb_filter only)            */
} rb_stage2_mode;

typedef struct rb_ctx_s*   rb_ctx;
typedef struct rb_bank_s*  rb_bank;
typedef struct rb_basis_s* rb_basis;

typedef struct {
  int64_t N;               /* samples per segment, power of two 2^12..2^21   */
  double  fs;              /* sampling rate, Hz (> 0)                        */
  double  f_low;           /* lower band edge, Hz, 0 < f_low < fs/2          */
} rb_grid;

/* One trigger: a (template, sample) pair whose SNR reaches the threshold. */
typedef struct {
  int32_t tmpl;            /* template index in the bank                     */
  int32_t sample;          /* sample index n in [0, N) (natural time order)  */
  float   snr;             /* |rho|                                          */
  float   phase;           /* arg rho in (-pi, pi]                           */
} rb_trigger;

/* Per-template maximum of |rho| over the samples a call evaluated. */
typedef struct {
  float   snr;             /* max |rho|; -1 if the template was not evaluated
                              by the exact filter in this call               */
  int32_t sample;          /* argmax (ties to the lowest n); -1 if none       */
} rb_peak;

typedef struct {
  int64_t n_stage1;        /* candidates: first-stage crossings of |rho_RB|
                              (rb_filter; with bins, those of the fine
                              reconstruction)                                */
  int32_t n_refiltered;    /* templates passed to the second stage           */
  int32_t rank;            /* basis rank used                                */
  float   ms[8];           /* device time per stage, ms: [0] strain FFT,
                              [1] correlation + basis IFFTs (+ bin means),
                              [2] reconstruction GEMM + first-stage threshold,
                              [3] selection, [4] second stage / full MF,
                              [5] sort + output, [6] total, [7] of [2], the
                              fine reconstruction of triggering bins         */
  int64_t n_bins;          /* triggering (template, bin) pairs (bin_w >= 2)  */
  double  min_energy;      /* smallest retained energy sum_k |c_jk|^2 of any
                              template of the bases used (1 for mf_full).
                              The part of a unit template outside its basis
                              has norm r = sqrt(1 - min_energy): a signal
                              matching the template at optimal SNR A loses
                              at most A r in the first stage, and noise adds
                              a Rayleigh term of scale r.  The second stages
                              that evaluate the exact SNR only where the
                              first stage crossed (SPARSE, AUTO) therefore
                              keep every final trigger while A r plus that
                              noise term stays below thr2 - thr1; FULL
                              needs only a crossing anywhere in the
                              template's series.                             */
  double  gemm_mfma_flop;  /* rb_filter: floating-point operations its
                              first-stage reconstruction GEMMs issued on the
                              matrix cores (the time of ms[2]), padding rows
                              and steps included: 6 K' T' N for the FP32
                              three-product kernel (below the 8 K T N of a
                              complex product), 8 K T' N for the realified
                              FP32 kernels, 8 K' T' N (x 3 split-BF16) for
                              the 16-bit ones.  0 from the other calls.      */
} rb_stats;

typedef struct {
  double  thr1;            /* candidate threshold on |rho_RB| (> 0)          */
  double  thr2;            /* final threshold (>= thr1): on the exact |rho|,
                              or on |rho_RB| with RB_STAGE2_RECON            */
  int32_t stage2;          /* rb_stage2_mode                                 */
  int32_t bin_w;           /* 0 or 1: rho_RB at every sample (first stage =
                              candidates); 2..64, a power of two with
                              N / bin_w >= 256: the binned first stage of
                              Sec. III.C (see rb_filter)                     */
  double  thr_bin;         /* bin_w >= 2: threshold rho_I on the averaged
                              |rho_avg| (> 0); ignored otherwise             */
  int32_t bin_source;      /* bin_w >= 2: 0 = the averaged series from the
                              basis (C beta_avg, Sec. III.C); 1 = from the
                              templates (Sec. III.D, Eq. avg_fft2: each
                              template's band product folded onto N/bin_w
                              bins and inverse transformed; the exact bin
                              means; needs N / bin_w >= 4096)                */
  int32_t flags;           /* 0, or RB_OPT_FP16_INTERMEDIATE                 */
} rb_filter_opts;

/* rb_filter_opts.flags.  RB_OPT_FP16_INTERMEDIATE: for BF16 and FP16 bases,
 * the four-step FFT intermediate between the passes that produce beta is
 * kept as FP16 pairs scaled by a power of two chosen from max |d| of the
 * segment (by Cauchy-Schwarz no pass-1 output of a unit-norm basis vector
 * reaches 2^15, so none overflows), halving that round trip's HBM traffic.
 * Its rounding (2^-11 of each intermediate element) spreads over the whole
 * segment: next to a signal of SNR 4000 the first-stage error at quiet
 * samples reaches 2.3e-2 of sum_k |c_jk| |beta_k(n)| (about 0.1 in |rho_RB|),
 * so thr2 - thr1 must cover it.  Ignored for FP32 and split-BF16 bases;
 * other bits are RB_ERR_ARG. */
#define RB_OPT_FP16_INTERMEDIATE 1

/* Bank source.  Fills out[(t1-t0) * (k1-k0) * 2] with the complex128 values
 * h_j[k] (interleaved re, im; row-major over templates) of templates
 * [t0, t1) at rfft bins [k0, k1).  Returns 0 on success.  Called from the
 * thread that called rb_bank_create, never concurrently. */
typedef int (*rb_bank_fill_fn)(void* user, int32_t t0, int32_t t1, int64_t k0, int64_t k1,
                               double* out);

/* Template source at arbitrary frequencies.  Fills out[(t1-t0) * nf * 2]
 * with the complex128 values h_j(f[i]) (interleaved re, im; row-major over
 * templates) of templates [t0, t1) at the nf host frequencies f (Hz).
 * Returns 0 on success.  Called from the thread that called the builder,
 * never concurrently. */
typedef int (*rb_fill_at_fn)(void* user, int32_t t0, int32_t t1, const double* f, int64_t nf,
                             double* out);

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`, ordering all work on `hip_stream`
 * (a hipStream_t, or NULL for the null stream; the stream stays owned by the
 * caller and must outlive the context).  RB_ERR_DEVICE if the device does not
 * exist or is not gfx950. */
rb_status rb_ctx_create(int device, void* hip_stream, rb_ctx* out);

/* Destroy a context.  RB_ERR_ARG if banks or bases created on it are still
 * alive. */
rb_status rb_ctx_destroy(rb_ctx ctx);

/* Thread-local text of the last failure ("" if none). */
const char* rb_last_error(void);

/* ------------------------------------------------------------------ bank */

/* Whiten and normalise a template bank and upload it (Sec. III.B: templates
 * whitened with the PSD and normalised to unity).
 *   grid  segment grid; psd: host, N/2+1 one-sided PSD values Sn[k] (1/Hz),
 *         finite and > 0 on the band (other bins are not read).
 *   T     number of templates, 1..2^24.
 *   fill  template source, called with chunks of templates over the bins
 *         [k_base, N/2) where k_base <= k_lo.
 * In FP64 on the host: sigma_j, the whitened unit templates
 * w_j[k] = h_j[k] sqrt(4 df/Sn[k]) / sigma_j; then rounded to complex64 and
 * uploaded.  RB_ERR_ARG for a bad grid or PSD, or a template with sigma = 0;
 * RB_ERR_CALLBACK if fill fails. */
rb_status rb_bank_create(rb_ctx ctx, const rb_grid* grid, const double* psd, int32_t T,
                         rb_bank_fill_fn fill, void* user, rb_bank* out);

rb_status rb_bank_free(rb_bank bank);

/* Bank facts.  Any output may be NULL.  sigma: host, T doubles (FP64 sigma_j
 * of the unwhitened templates, i.e. their optimal-SNR normalisation). */
rb_status rb_bank_info(rb_bank bank, int32_t* T, int64_t* k_lo, int64_t* k_hi, double* sigma);

/* ------------------------------------------------------------------ basis */

/* Reduced basis of a bank (Sec. II.A, III.B; Eqs. Eq-SVD, SNR_loss).
 *   rank  > 0: keep exactly min(rank, T) vectors;  0: the smallest K whose
 *         retained energy sum_{k<K} lambda_k / sum lambda is >= 1 - tol.
 *   tol   in (0, 1) when rank == 0.
 *   dtype storage of C and Z in rb_filter (RB_F32, RB_BF16, RB_F16).
 * FP64 throughout: Gram products of the stored templates, subspace iteration
 * with Rayleigh-Ritz, basis rows v_k = lambda_k^{-1/2} sum_j conj(U_jk) w_j,
 * coefficients c_jk = <w_j, v_k>.  The basis is stored complex64, the
 * coefficients as C = conj(c) in `dtype` (with power-of-two row scales for
 * FP16).  rank_out / energy_out: host, may be NULL.  Equivalent to
 * rb_build_basis_range over [0, T). */
rb_status rb_build_basis(rb_ctx ctx, rb_bank bank, int32_t rank, double tol, rb_dtype dtype,
                         rb_basis* out, int32_t* rank_out, double* energy_out);

/* Basis of the sub-bank of templates [t0, t1) (0 <= t0 < t1 <= T): the
 * paper splits a bank into sub-banks (along tau0) and builds one basis per
 * sub-bank (Sec. III.B).  Template indices stay global everywhere (triggers,
 * rb_rho_at / rb_backward trigger lists); per-template arrays of a range basis
 * (coefficients, gradients, dumps) have t1 - t0 rows. */
rb_status rb_build_basis_range(rb_ctx ctx, rb_bank bank, int32_t t0, int32_t t1, int32_t rank,
                               double tol, rb_dtype dtype, rb_basis* out, int32_t* rank_out,
                               double* energy_out);

/* Eigensolvers of the basis construction. */
typedef enum {
  RB_EIG_SUBSPACE = 0, /* randomized subspace iteration with Rayleigh-Ritz (the default) */
  RB_EIG_LANCZOS = 1   /* block Lanczos with full reorthogonalisation (Sec. III.B runs a Lanczos
                          eigensolver on the covariance) */
} rb_eig_solver;

/* rb_build_basis_range with a choice of FP64 eigensolver for the leading
 * eigenpairs of the Gram matrix W W^H of the sub-bank's whitened unit
 * templates (applied as W (W^H X), never formed).  RB_EIG_LANCZOS: Krylov
 * blocks of b = 32 columns (rank / 4 clamped to [16, 64] for a fixed rank),
 * each G X_j orthogonalised against every earlier block by two passes of
 * classical Gram-Schmidt (columns reduced below 1e-10 of their norm
 * dropped), Rayleigh-Ritz on the whole space after each block, stopping when
 * the pairs the rank rule keeps have residual norms |G u - theta u| <=
 * 1e-10 theta_1 (residuals formed directly) with at least b spare columns,
 * or the space reaches t1 - t0.
 * Both solvers feed the same basis rows, coefficients and storage.
 * RB_ERR_ARG for a bad solver; other arguments as rb_build_basis_range. */
rb_status rb_build_basis_solver(rb_ctx ctx, rb_bank bank, int32_t t0, int32_t t1, int32_t rank,
                                double tol, rb_dtype dtype, int32_t solver, rb_basis* out,
                                int32_t* rank_out, double* energy_out);

/* Non-uniform frequency set for the PCA (Sec. III.A, PCA using non-uniform
 * sampling).  Host only: touches no device.
 *   f, h_re  host, n >= 2 samples of one reference template (the longest
 *            of the bank) over [f[0], f[n-1]]: strictly increasing finite
 *            frequencies and the finite real part of h there.  The samples
 *            must resolve its oscillation (several per half-cycle).
 *   per_bin  frequencies per bin, 1..1024 (the paper takes five).
 *   df_min   floor on the spacing (> 0; the paper takes 1/128 Hz, the grid
 *            step of its 128 s segments).
 *   extra    host, n_extra frequencies merged into the set where they fall
 *            strictly inside (f[0], f[n-1]) (may be NULL when n_extra == 0);
 *            e.g. the uniform frequencies on either side of each template's
 *            f_ISCO cut, which linear interpolation could not follow else.
 * The zero crossings of h_re (a sign change between consecutive samples,
 * located by linear interpolation, or an interior sample exactly zero) cut
 * [f[0], f[n-1]] into bins [e_b, e_{b+1}); a bin takes the per_bin
 * frequencies e_b + m (e_{b+1} - e_b) / per_bin, or, when that spacing is
 * below df_min, the multiples k df_min inside it (so with df_min equal to a
 * segment's grid step the dense part of the set is that grid itself); f[n-1]
 * closes the set.  Output: the strictly increasing set in out[0 .. *n_out).
 * RB_ERR_CAPACITY (with *n_out = the size needed) when it has more than
 * cap entries; out may be NULL with cap == 0 to ask for the size.
 * RB_ERR_ARG for bad arguments. */
rb_status rb_nonuniform_freqs(const double* f, const double* h_re, int64_t n, int32_t per_bin, double df_min,
                              const double* extra, int64_t n_extra, double* out, int64_t cap,
                              int64_t* n_out);

/* Basis of templates [t0, t1) built by PCA on a non-uniform frequency set
 * and interpolated onto the bank's uniform grid (Sec. III.A; the
 * interpolation step of Sec. III.C).
 *   nodes      host, nt >= 2 strictly increasing frequencies covering the
 *              band: nodes[0] <= k_lo df and nodes[nt-1] >= k_hi df
 *              (typically from rb_nonuniform_freqs).
 *   psd_nodes  host, nt one-sided PSD values Sn(nodes[i]), finite and > 0.
 *   fill       the templates [t0, t1) at the nodes (the bank's own
 *              templates, global indices).
 *   rank, tol, dtype  as rb_build_basis_range (the rank rule runs on the
 *              eigenvalues on the set).
 * FP64 throughout: node i weighs omega_i, the width of its cell between the
 * midpoints to its neighbours (end cells mirrored); the templates are
 * whitened and normalised in that inner product,
 * V[j][i] = h_j(f_i) sqrt(4 omega_i / Sn_i) / sigma_j, rounded to complex64
 * on the device; the leading right singular vectors of V (eigenvectors of
 * the covariance V^H V) by the same subspace iteration as the uniform
 * basis; each, divided by sqrt(omega_i), interpolated linearly to the
 * uniform frequencies k df of the band and multiplied by sqrt(df); the K
 * interpolated vectors orthonormalised on the uniform grid; coefficients
 * c_jk = <w_j, v_k> against the bank's uniform templates.  The rank can
 * drop below the requested one only if interpolation made vectors linearly
 * dependent.  energy_out: sum |c|^2 / sum |w_j|^2 on the uniform grid.
 * rb_basis_export's lambda are the eigenvalues on the set.
 * RB_ERR_ARG for bad nodes, PSD or range; RB_ERR_CALLBACK if fill fails. */
rb_status rb_build_basis_nonuniform(rb_ctx ctx, rb_bank bank, int32_t t0, int32_t t1, const double* nodes,
                                    int64_t nt, const double* psd_nodes, rb_fill_at_fn fill, void* user,
                                    int32_t rank, double tol, rb_dtype dtype, rb_basis* out,
                                    int32_t* rank_out, double* energy_out);

/* Basis facts (outputs may be NULL). */
rb_status rb_basis_info(rb_basis basis, int32_t* t0, int32_t* t1, int32_t* rank, double* energy);

rb_status rb_basis_free(rb_basis basis);

/* Copy the basis out (host arrays, any may be NULL): V: K x nb complex128
 * (rows over bins k_lo..k_hi), c: (t1-t0) x K complex128 coefficients (FP64,
 * before storage rounding), lambda: K eigenvalues (FP64, descending). */
rb_status rb_basis_export(rb_basis basis, double* V, double* c, double* lambda);

/* ------------------------------------------------------------------ search */

/* Hierarchical reduced-basis search of one segment (Sec. III.C):
 *   1. s~ of the strain (forward FFT), whitened on the band;
 *   2. beta_k = IFFT(d conj(v_k)) for every basis vector of every sub-bank;
 *   3. bin_w <= 1: rho_RB = C beta (MFMA GEMM) at every sample, candidates
 *      |rho_RB| >= thr1.
 *      bin_w = w >= 2 (the binned first stage): the bin means
 *      beta_avg_k[i] = (1/w) sum_{r<w} beta_k[i w + r] (Eq. for beta^avg),
 *      rho_avg = C beta_avg (MFMA GEMM on N/w samples), triggering bins
 *      |rho_avg| >= thr_bin; then rho_RB at every sample of every
 *      triggering (template, bin) (FP32), candidates |rho_RB| >= thr1;
 *      with bin_source = 1 the averaged series comes from the templates
 *      instead (the fast first stage of Sec. III.D) and the basis serves
 *      the fine reconstruction only;
 *   4. second stage (opts->stage2) on the candidates: the exact |rho|
 *      (FULL, SPARSE, AUTO) or the reconstruction itself (RECON); final
 *      triggers reach thr2.
 *   With bin_w >= 2 the candidate set only holds samples of triggering bins:
 *   averaging lowers |rho| (the complex SNR rotates within a bin), so thr_bin
 *   must sit well below thr1 to keep a given recovery (Sec. IV.B).
 *   bases   nbases (>= 1) bases of this bank whose template ranges partition
 *           [0, T) (one basis of the whole bank, or one per sub-bank).
 *   strain  host or device, N floats.
 *   out     host or device, cap entries; triggers sorted by (tmpl, sample).
 *   n_out   host; number of final triggers.  If it exceeds cap the call
 *           returns RB_ERR_CAPACITY with the required count in *n_out.
 *   peaks   host or device, T entries, or NULL (with RECON: the maximum
 *           |rho_RB| over the template's candidates).
 *   stats   host or NULL.
 * RB_ERR_ARG for a bad threshold, mode, bin_w or thr_bin. */
rb_status rb_filter(rb_ctx ctx, const rb_basis* bases, int32_t nbases, rb_bank bank,
                    const float* strain, const rb_filter_opts* opts, rb_trigger* out, int64_t cap,
                    int64_t* n_out, rb_peak* peaks, rb_stats* stats);

/* Overlap-save search of a long strain (Sec. III.E): segments of N samples
 * (the bank's grid), each overlapping the previous one by N/2, searched with
 * rb_filter.  Segment i starts at i N/2 (the last one at n - N) and reports
 * the final triggers of its central half [start + N/4, start + 3N/4); the
 * first segment's window starts at 0, the last one's ends at n, and where
 * the last segment was moved back the previous window ends where its half
 * begins, so every stream sample is reported by exactly one segment.
 *   strain  host or device, n floats, N <= n < 2^31.  Segments are cut
 *           without tapering: condition the stream first (no power far below
 *           f_low), or the out-of-band power leaks into the band at every
 *           segment edge.
 *   out     host or device, cap entries; sample = index in the stream; in
 *           segment order, sorted by (tmpl, sample) within a segment.
 *   n_out   host; RB_ERR_CAPACITY (with the required count) if it exceeds cap.
 *   stats   host or NULL: counts and device times summed over the segments.
 * Other arguments and errors as rb_filter. */
rb_status rb_filter_stream(rb_ctx ctx, const rb_basis* bases, int32_t nbases, rb_bank bank,
                           const float* strain, int64_t n, const rb_filter_opts* opts, rb_trigger* out,
                           int64_t cap, int64_t* n_out, rb_stats* stats);

/* One work item of a batched search: a segment and the bank (on that
 * segment's grid) with the bases of its sub-banks. */
typedef struct {
  const float* strain;       /* device pointer, N floats of the bank's grid     */
  rb_bank bank;
  const rb_basis* bases;     /* bases partitioning the bank's templates         */
  int32_t nbases;
} rb_batch_item;

/* Batched hierarchical search (Sec. III.B sub-banks x segments of any length;
 * one item per (segment, bank)).  Each item runs the same steps as rb_filter
 * (FULL, SPARSE or RECON second stage, any bin_w with bin_source 0;
 * RB_ERR_UNSUPPORTED for AUTO or bin_source 1) with device-side counts, so
 * the whole batch is a sequence of kernel launches with no host
 * synchronisation inside.
 *   use_graph  1: the batch is captured once into a hipGraph (keyed by the
 *              item pointers, thresholds and capacities) and replayed on later
 *              calls with the same key: refill the strain buffers and call
 *              again.  0: launched eagerly.
 *   out        host or device, nitems x cap_item triggers; item i's sorted
 *              triggers start at out + i * cap_item.
 *   n_out      host, nitems counts.  RB_ERR_CAPACITY (with every count set)
 *              if some item has more than cap_item triggers.
 *   stats      host or NULL: summed counts and ms[6] = device time of the
 *              batch. */
rb_status rb_filter_batch(rb_ctx ctx, int32_t nitems, const rb_batch_item* items,
                          const rb_filter_opts* opts, int32_t use_graph, rb_trigger* out,
                          int64_t cap_item, int64_t* n_out, rb_stats* stats);

/* Template method (Sec. II, Eq. IFFT): the full SNR series of every template
 * by an inverse FFT, thresholded at thr (> 0).  Arguments as for rb_filter. */
rb_status mf_full(rb_ctx ctx, rb_bank bank, const float* strain, double thr, rb_trigger* out,
                  int64_t cap, int64_t* n_out, rb_peak* peaks, rb_stats* stats);

/* mf_full without device allocation, for callers that cannot allocate
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same kernels and the same sorted triggers as mf_full.
 *   strain  device, N floats.
 *   out     device, cap triggers (may be NULL when cap == 0).
 *   n_out   host: the number of triggers.
 * Scratch: every intermediate (whitened data, FFT intermediate, counters,
 * trigger records and their sort buffers) lives in one fixed device array of
 * RB_NOALLOC_SCRATCH_BYTES per GPU that the library holds until the process
 * ends; the call allocates nothing.  The array keeps the previous call's
 * contents (the call clears what must start at zero).  Calls on one GPU share
 * it, so overlapping calls would race: the library serialises them (a call
 * holds the GPU's array until its work has finished, and it synchronises the
 * context's stream before returning).
 * Precondition: the context already holds the FFT plan of the bank's grid
 * (any earlier mf_full or rb_filter call on a bank of the same N prepares
 * it), else RB_ERR_ARG.
 * Limits: RB_ERR_ARG when N and T need more than the array (N double2 of
 * FFT work, the whitened data, 16 bytes per template and 16 MiB of trigger
 * records: every supported N up to 2^21 fits with banks of up to 10^5
 * templates); RB_ERR_UNSUPPORTED, with *n_out = the count, when the
 * crossings exceed the records the array holds (at least 349 525, from
 * 16 MiB over three record arrays); RB_ERR_CAPACITY (with *n_out) when they
 * exceed cap. */
#define RB_NOALLOC_SCRATCH_BYTES (64ull << 20)
rb_status mf_full_noalloc(rb_ctx ctx, rb_bank bank, const float* strain, double thr, rb_trigger* out,
                          int64_t cap, int64_t* n_out);

/* First-stage reconstruction at given (template, sample) points:
 *   rho_i = sum_k C_{j_i k} beta_k[n_i]      (Eq. Beta_eqn, C = conj(c))
 * with beta from `strain` (FP32 path whatever the basis storage type).
 *   S    host or device, n triggers (only tmpl and sample are read; tmpl in
 *        the basis's range [t0, t1), sample in [0, N), else RB_ERR_ARG).
 *   C    host or device, (t1-t0) x K complex64 coefficients replacing the
 *        basis's own conj(c), or NULL to use them.
 *   rho  host or device, n complex64 (interleaved). */
rb_status rb_rho_at(rb_ctx ctx, rb_basis basis, const float* strain, const rb_trigger* S,
                    int64_t n, const float* C, float* rho);

/* Adjoint of correlation plus reconstruction.  For the loss
 *   L = sum_i g_i |rho_{j_i}[n_i]|^2      (S = {(j_i, n_i)} frozen, rho as in
 *                                          rb_rho_at)
 * computes dL/dC ((t1-t0) x K complex64, interleaved, torch's convention for a
 * complex leaf: dL/dRe + i dL/dIm; rows without triggers are zero) and dL/ds
 * (N floats).  Reductions run in a fixed order (bitwise reproducible).
 *   S, C     as for rb_rho_at.
 *   seed     host or device, n floats g_i, or NULL for all ones.
 *   grad_C   host or device or NULL; grad_strain host or device or NULL.
 *   loss     host or NULL: L. */
rb_status rb_backward(rb_ctx ctx, rb_basis basis, const float* strain, const rb_trigger* S,
                      const float* seed, int64_t n, const float* C, float* grad_C,
                      float* grad_strain, double* loss);

/* Refinement of trigger coefficient vectors between bank points (Sec. II.A:
 * the basis spans the bank, so a unit coefficient vector near a template's
 * describes a template between bank points; the gradient is the adjoint of
 * the reconstruction, Eq. Beta_eqn).  For each trigger i = (j, n):
 *   1. the `neighbours` templates l != j of the basis with the largest
 *      |<c_j, c_l>| (ties to the lower index);
 *   2. an orthonormal basis (FP64, modified Gram-Schmidt twice, dependent
 *      rows dropped) of the span of the coefficient rows C_j, C_l (C = conj(c));
 *   3. `iters` steps of projected gradient ascent of |rho|^2,
 *      rho = sum_k C_k beta_k[n], from C = C_j:
 *        C <- C + (2 rho conj(beta[:, n])) / (2 |rho|^2); C <- Proj C; C <- C / |C|.
 *      The maximiser over unit vectors of the span is the normalised
 *      projection of conj(beta[:, n]) onto it (Cauchy-Schwarz).
 * beta from `strain` on the FP32 path, whatever the basis storage type.
 *   S         host or device, n triggers (tmpl in the basis's range, sample in
 *             [0, N), else RB_ERR_ARG).
 *   neighbours 0 ... min(32, t1 - t0 - 1); iters 0 ... 100000.
 *   c_out     host or device, n x K complex64 (interleaved): refined rows of C.
 *   nbr_out   host or device or NULL: n x neighbours global template indices,
 *             nearest first.
 *   p_out     host or device or NULL: n x 2 floats, |rho|^2 of the trigger's
 *             own row C_j and of the refined row.
 * RB_ERR_UNSUPPORTED for ranks above 2048.  Outputs are written only on
 * success. */
rb_status rb_refine(rb_ctx ctx, rb_basis basis, const float* strain, const rb_trigger* S, int64_t n,
                    int32_t neighbours, int32_t iters, float* c_out, int32_t* nbr_out, float* p_out);

/* Clustered peaks of a (tmpl, sample)-sorted trigger list: is_peak[i] = 1 if
 * no trigger of the same template within +-W samples (circular over N) has a
 * larger SNR, or an equal SNR at a lower sample.  trig / is_peak: host or
 * device. */
rb_status rb_cluster_peaks(rb_ctx ctx, const rb_trigger* trig, int64_t n, int32_t W, int64_t N,
                           uint8_t* is_peak);

/* ------------------------------------------------------------------ debug */

/* Dump the complex SNR series (small T*N only): rho (host or device,
 * rows x N x 2 floats, natural time order).  basis == NULL: exact template
 * method for all T templates; otherwise the first-stage reconstruction
 * rho_RB = C beta for the basis's t1 - t0 templates. */
rb_status rb_debug_rho(rb_ctx ctx, rb_basis basis, rb_bank bank, const float* strain, float* rho);

/* Dump the averaged series of the binned first stage (small T*N only):
 * rho_avg = C beta_avg for the basis's t1 - t0 templates as rb_filter
 * computes it with bin_w = w (Sec. III.C), rows x (N/w) x 2 floats (host or
 * device), bins in natural order, storage scales removed. */
rb_status rb_debug_rho_binned(rb_ctx ctx, rb_basis basis, const float* strain, int32_t w, float* rho);

/* Dump the per-basis filter outputs beta (K x N x 2 floats, natural time
 * order, host or device) as stored for the reconstruction (after any 16-bit
 * rounding and with its scale removed).  For RB_BF16X3 bases beta holds
 * 2 x K x N x 2 floats: the high parts, then the low parts. */
rb_status rb_debug_basis_outputs(rb_ctx ctx, rb_basis basis, const float* strain, float* beta);

#ifdef __cplusplus
}
#endif
#endif /* RBMF_H */
