// C-ABI host layer: argument validation, handles, device buffers, and the
// orchestration of the kernels for each entry point of include/rbmf.h.
#include "../../include/rbmf.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"
#include "linalg.h"
#include "nonuniform.h"

namespace rbmf {

hipError_t launch_pack_c(const float2* C, int T, int Tp, int K, int Kp, int dtype, const float* row_scale,
                         void* cpk, hipStream_t stream);
int gemm_tile_templates();

namespace {
thread_local std::string g_err;
}
void set_error(const std::string& msg) { g_err = msg; }
const char* last_error_cstr() { return g_err.c_str(); }

}  // namespace rbmf

using namespace rbmf;
using cd = std::complex<double>;

// ====================================================================== helpers
namespace {

#define RB_CHECK(cond, code, msg)       \
  do {                                  \
    if (!(cond)) {                      \
      set_error(msg);                   \
      return code;                      \
    }                                   \
  } while (0)

#define RB_TRY(expr)                    \
  do {                                  \
    rb_status st_ = (expr);             \
    if (st_ != RB_OK) return st_;       \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  rb_status ensure(size_t need) {
    if (need <= bytes && p) return RB_OK;
    release();
    if (need == 0) need = 256;
    if (hipMalloc(&p, need) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      set_error("device allocation of " + std::to_string(need) + " bytes failed");
      return RB_ERR_OOM;
    }
    bytes = need;
    return RB_OK;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

struct HostPinned {
  void* p = nullptr;
  size_t bytes = 0;
  ~HostPinned() {
    if (p) (void)hipHostFree(p);
  }
  rb_status ensure(size_t need) {
    if (need <= bytes && p) return RB_OK;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    if (hipHostMalloc(&p, need, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      set_error("pinned host allocation failed");
      return RB_ERR_OOM;
    }
    bytes = need;
    return RB_OK;
  }
};

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

template <class F>
void parallel_for(int64_t n, F&& f) {
  int nt = (int)std::min<int64_t>(n, std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int64_t> next(0);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (int64_t i; (i = next.fetch_add(1)) < n;) f(i);
    });
  for (auto& t : th) t.join();
}

struct TwTables {
  DevBuf pyr, tlo, thi, pyr64, tlo64, thi64;
};

}  // namespace

// ====================================================================== handles
struct rb_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  int live = 0;
  std::map<int64_t, std::unique_ptr<TwTables>> tw;
  // scratch
  DevBuf work, work64, dspec, strain, z, z32, recs1, thr_inf, adjA, adjAhat, adjB, adjT, adjS, adjRho, adjG, adjC, adjGC,
      adjOrd, adjSeg, trig1, trig2, recs, tmp, final_out, cnt1, cnt2, off1, off2, fill1, fill2,
      list1, list2, tmax, summary, counters, thr_row, peaks, flag, rho_tmp, zws, listH, listL, nsplit,
      zfine, zpart, trigB, cntB, snap, tinv, gfold, offB, fillB, listB, recsB, sstrain, segout, wout, wcount, goffB,
      refOv, refQ, refC, refN, refP, hscale;
  // dspec is rewritten by each spectrum (dspec_gen counts them); the FP16
  // intermediate's scale in hscale belongs to spectrum hscale_gen
  uint64_t dspec_gen = 0, hscale_gen = ~uint64_t(0);
  int hscale_n2 = 0;
  int64_t gfold_N = 0;             // grid and bin width of the table in gfold
  int gfold_w = 0;
  hipEvent_t ev[8] = {};
  std::vector<hipEvent_t> evs;
  std::map<int64_t, int> fft_n2;   // autotuned four-step split per N (log2 N2)
  std::string arch;                // device architecture name (tuning cache key prefix)
  bool want_peaks = false;         // the current call returns per-template peaks (tmax is needed)
  double mfma_flop = 0;            // matrix-core flop of the reconstruction GEMMs launched since reset
  // batch search: per-item summaries and outputs, captured graph
  DevBuf bsum, bout;
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::string gkey;
  void* noalloc = nullptr;         // this device's fixed scratch (device address) for mf_full_noalloc
  ~rb_ctx_s() {
    for (auto e : evs) (void)hipEventDestroy(e);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (gstream) (void)hipStreamDestroy(gstream);
  }
};

struct rb_bank_s {
  rb_ctx ctx = nullptr;
  rb_grid grid{};
  int32_t T = 0;
  int64_t k_lo = 0, k_hi = 0, kb = 0, nbs = 0;
  std::vector<double> sigma;
  DevBuf w;          // T x nbs complex64 whitened unit templates
  DevBuf wd;         // nbs double: dt * sqrt(4 df / Sn) (0 below k_lo)
  DevBuf sup_lo, sup_hi;
  int live_bases = 0;
};

struct rb_basis_s {
  rb_ctx ctx = nullptr;
  rb_bank bank = nullptr;
  int32_t t0 = 0, T = 0;       // template range [t0, t0 + T) of the bank
  int32_t K = 0, Kp = 0, Tp = 0;
  rb_dtype dtype = RB_F32;
  double energy = 0.0, trace = 0.0;
  double min_energy = 1.0;     // smallest per-template retained energy sum_k |c_jk|^2
  std::vector<double> lambda;
  std::vector<cd> c;           // T x K FP64 coefficients
  std::vector<float> row_scale;  // per-template power-of-two scale (16-bit), 1 otherwise
  DevBuf P;                    // K x nbs complex64
  DevBuf cpk;                  // packed realified C
  DevBuf cpk3;                 // FP32: C packed for the three-product GEMM
  DevBuf cpkc;                 // 16-bit: C packed for the compact-coefficient GEMM variants
  DevBuf C32;                  // T x K complex64 (conj(c)), unscaled, for the adjoint
  DevBuf row_inv;              // Tp floats 1/row_scale
  DevBuf row_scale_dev;        // Tp floats
  DevBuf thr_row;              // Tp floats: squared first-stage threshold per template
  float thr_cached = -1.f;
  std::map<int64_t, int> gemm_variant;   // autotuned reconstruction kernel variant per column count
};

// ====================================================================== shared steps
namespace {

rb_status get_tables(rb_ctx ctx, const FftGeom& g, FftTables& out, FftTables64* out64 = nullptr) {
  auto it = ctx->tw.find(g.N);
  if (it == ctx->tw.end()) {
    auto t = std::make_unique<TwTables>();
    std::vector<float2> pyr(4096, make_float2(0.f, 0.f));
    for (int L = 2; L <= 2048; L <<= 1)
      for (int i = 0; i < L; ++i) {
        const double a = 2.0 * M_PI * (double)i / (double)L;
        pyr[L + i] = make_float2((float)std::cos(a), (float)std::sin(a));
      }
    const int64_t nlo = int64_t(1) << g.s_lo, nhi = g.N >> g.s_lo;
    std::vector<float2> tlo(nlo), thi(std::max<int64_t>(nhi, 1));
    for (int64_t e = 0; e < nlo; ++e) {
      const double a = 2.0 * M_PI * (double)e / (double)g.N;
      tlo[e] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    for (int64_t e = 0; e < nhi; ++e) {
      const double a = 2.0 * M_PI * (double)(e << g.s_lo) / (double)g.N;
      thi[e] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    std::vector<double2> pyr64(4096, make_double2(0.0, 0.0)), tlo64(nlo), thi64(thi.size());
    for (int L = 2; L <= 2048; L <<= 1)
      for (int i = 0; i < L; ++i) {
        const double a = 2.0 * M_PI * (double)i / (double)L;
        pyr64[L + i] = make_double2(std::cos(a), std::sin(a));
      }
    for (int64_t e = 0; e < nlo; ++e) {
      const double a = 2.0 * M_PI * (double)e / (double)g.N;
      tlo64[e] = make_double2(std::cos(a), std::sin(a));
    }
    for (int64_t e = 0; e < nhi; ++e) {
      const double a = 2.0 * M_PI * (double)(e << g.s_lo) / (double)g.N;
      thi64[e] = make_double2(std::cos(a), std::sin(a));
    }
    RB_TRY(t->pyr64.ensure(pyr64.size() * sizeof(double2)));
    RB_TRY(t->tlo64.ensure(tlo64.size() * sizeof(double2)));
    RB_TRY(t->thi64.ensure(thi64.size() * sizeof(double2)));
    RB_HIP(hipMemcpy(t->pyr64.p, pyr64.data(), pyr64.size() * sizeof(double2), hipMemcpyHostToDevice));
    RB_HIP(hipMemcpy(t->tlo64.p, tlo64.data(), tlo64.size() * sizeof(double2), hipMemcpyHostToDevice));
    RB_HIP(hipMemcpy(t->thi64.p, thi64.data(), thi64.size() * sizeof(double2), hipMemcpyHostToDevice));
    RB_TRY(t->pyr.ensure(pyr.size() * sizeof(float2)));
    RB_TRY(t->tlo.ensure(tlo.size() * sizeof(float2)));
    RB_TRY(t->thi.ensure(thi.size() * sizeof(float2)));
    RB_HIP(hipMemcpy(t->pyr.p, pyr.data(), pyr.size() * sizeof(float2), hipMemcpyHostToDevice));
    RB_HIP(hipMemcpy(t->tlo.p, tlo.data(), tlo.size() * sizeof(float2), hipMemcpyHostToDevice));
    RB_HIP(hipMemcpy(t->thi.p, thi.data(), thi.size() * sizeof(float2), hipMemcpyHostToDevice));
    it = ctx->tw.emplace(g.N, std::move(t)).first;
  }
  out.pyr = it->second->pyr.as<float2>();
  out.tlo = it->second->tlo.as<float2>();
  out.thi = it->second->thi.as<float2>();
  if (out64) {
    out64->pyr = it->second->pyr64.as<double2>();
    out64->tlo = it->second->tlo64.as<double2>();
    out64->thi = it->second->thi64.as<double2>();
  }
  return RB_OK;
}

rb_status fill32(rb_ctx ctx, void* p, uint32_t v, int64_t n) {
  RB_HIP(launch_fill_u32(static_cast<uint32_t*>(p), v, n, ctx->stream));
  return RB_OK;
}

// vectors per FFT batch: keep the [B][N] intermediate near 256 MB so the
// pass-1 -> pass-2 round trip can stay in the Infinity Cache.
// Vectors per FFT launch pair: the pass-1 -> pass-2 intermediate ([B][N]
// complex64) holds RBMF_WORK_MB megabytes (default 512).  Larger batches mean
// fewer launch pairs and fewer partly filled last waves of workgroups.
int64_t work_budget_bytes() {
  const char* e = std::getenv("RBMF_WORK_MB");
  const int64_t mb = e ? std::atoll(e) : 512;
  return std::max<int64_t>(8, std::min<int64_t>(mb, 4096)) << 20;
}

// RB_STAGE2_AUTO: crossings from which a template takes the full matched
// filter (RBMF_STAGE2_SPLIT, default 32: four groups of direct sums cost about
// as much as the two FFT passes of one template).
int stage2_split() {
  const char* e = std::getenv("RBMF_STAGE2_SPLIT");
  const int v = e ? std::atoi(e) : 32;
  return v < 1 ? 1 : v;
}

int batch_vectors(int64_t N, int64_t nvec) {
  int64_t b = work_budget_bytes() / (N * 8);
  b = std::max<int64_t>(1, std::min<int64_t>(b, 1024));
  return (int)std::min<int64_t>(b, std::max<int64_t>(nvec, 1));
}

PassArgs base_args(rb_bank bank, const FftGeom& g, const FftTables& tw) {
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.g = g;
  a.tw = tw;
  a.kb = bank->kb;
  a.nbs = bank->nbs;
  a.band_lo = (int32_t)bank->k_lo;
  a.band_hi = (int32_t)bank->k_hi;
  a.k_lo = (int32_t)bank->k_lo;
  a.k_hi = (int32_t)bank->k_hi;
  a.wd64 = bank->wd.as<double>();
  a.zscale = 1.f;
  return a;
}

// Persistent tuning cache.  With RBMF_TUNE_FILE set, tuned choices (FFT split
// per N, GEMM variant per dtype / K / T / N) are read from and written back to
// that file, a flat JSON object {"<arch>/<kind>/<key>": <int>, ...}; without
// it choices live for the process only.  A process-wide table shared by all
// contexts.
class TuneCache {
 public:
  bool get(const std::string& key, int* v) {
    std::lock_guard<std::mutex> lk(mu_);
    load();
    auto it = map_.find(key);
    if (it == map_.end()) return false;
    *v = it->second;
    return true;
  }
  void put(const std::string& key, int v) {
    std::lock_guard<std::mutex> lk(mu_);
    load();
    map_[key] = v;
    const char* f = std::getenv("RBMF_TUNE_FILE");
    if (!f || !*f) return;
    const std::string tmp = std::string(f) + ".tmp";
    FILE* fp = std::fopen(tmp.c_str(), "w");
    if (!fp) return;
    std::fprintf(fp, "{\n");
    size_t i = 0;
    for (const auto& kv : map_)
      std::fprintf(fp, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < map_.size() ? "," : "");
    std::fprintf(fp, "}\n");
    const bool ok = std::fclose(fp) == 0;
    if (ok) (void)std::rename(tmp.c_str(), f);
  }

 private:
  void load() {   // once; a missing or malformed file is an empty cache
    if (loaded_) return;
    loaded_ = true;
    const char* f = std::getenv("RBMF_TUNE_FILE");
    if (!f || !*f) return;
    FILE* fp = std::fopen(f, "r");
    if (!fp) return;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), fp)) > 0) text.append(buf, n);
    std::fclose(fp);
    size_t p = 0;
    while ((p = text.find('"', p)) != std::string::npos) {
      const size_t q = text.find('"', p + 1);
      if (q == std::string::npos) break;
      const std::string key = text.substr(p + 1, q - p - 1);
      const size_t c = text.find(':', q);
      if (c == std::string::npos) break;
      char* end = nullptr;
      const long v = std::strtol(text.c_str() + c + 1, &end, 10);
      if (end != text.c_str() + c + 1) map_[key] = (int)v;
      p = end ? (size_t)(end - text.c_str()) : q + 1;
    }
  }
  std::mutex mu_;
  bool loaded_ = false;
  std::map<std::string, int> map_;
};

TuneCache& tune_cache() {
  static TuneCache c;
  return c;
}

// ---------------------------------------------------------------- autotuner
// The four-step split N = N1 N2 of the FFT passes is chosen per N by timing
// the candidate splits (balanced, and one step either way) on a batch of
// correlation + inverse transforms of the bank's own templates, once per
// context.  RBMF_FFT_SPLIT=<log2 N2> forces a split, RBMF_AUTOTUNE=0 keeps
// the balanced one.
rb_status geom_for(rb_ctx ctx, rb_bank bank, FftGeom* out) {
  const int64_t N = bank->grid.N;
  auto it = ctx->fft_n2.find(N);
  if (it != ctx->fft_n2.end()) {
    *out = make_geom(N, it->second);
    return RB_OK;
  }
  const FftGeom g0 = make_geom(N);
  int choice = g0.log2N / 2;
  const char* force = std::getenv("RBMF_FFT_SPLIT");
  const char* at = std::getenv("RBMF_AUTOTUNE");
  const std::string key = ctx->arch + "/fft/N=" + std::to_string(N);
  int cached = -1;
  if (force) {
    const FftGeom gf = make_geom(N, std::atoi(force));
    RB_CHECK(geom_supported(gf), RB_ERR_ARG, "RBMF_FFT_SPLIT gives an unsupported split");
    choice = std::atoi(force);
  } else if (tune_cache().get(key, &cached) && geom_supported(make_geom(N, cached))) {
    choice = cached;
  } else if (!(at && std::strcmp(at, "0") == 0)) {
    std::vector<int> cand;
    for (int c : {g0.log2N / 2, g0.log2N - g0.log2N / 2, g0.log2N / 2 - 1})
      if (geom_supported(make_geom(N, c)) && std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
    if (cand.size() > 1) {
      const int B = std::min<int64_t>(batch_vectors(N, bank->T), 32);
      RB_TRY(ctx->work.ensure((size_t)B * N * 8));
      RB_TRY(ctx->dspec.ensure((size_t)bank->nbs * 8));
      RB_TRY(ctx->z32.ensure((size_t)2 * B * N * 4));
      RB_TRY(fill32(ctx, ctx->dspec.p, 0u, bank->nbs * 2));
      ctx->dspec_gen++;
      hipEvent_t e0, e1;
      RB_HIP(hipEventCreate(&e0));
      RB_HIP(hipEventCreate(&e1));
      float best = 1e30f;
      for (int c : cand) {
        const FftGeom g = make_geom(N, c);
        FftTables tw;
        RB_TRY(get_tables(ctx, g, tw));
        PassArgs a = base_args(bank, g, tw);
        a.sign = +1;
        a.nvec = B;
        a.d = ctx->dspec.as<float2>();
        a.src = bank->w.as<float2>();
        a.work = ctx->work.as<float2>();
        a.zout = ctx->z32.as<float>();
        float ms_min = 1e30f;
        for (int rep = 0; rep < 4; ++rep) {
          RB_HIP(hipEventRecord(e0, ctx->stream));
          RB_HIP(launch_pass1(a, IN_CORR, ctx->stream));
          RB_HIP(launch_pass2(a, OUT_Z32, ctx->stream));
          RB_HIP(hipEventRecord(e1, ctx->stream));
          RB_HIP(hipEventSynchronize(e1));
          float ms = 0.f;
          RB_HIP(hipEventElapsedTime(&ms, e0, e1));
          if (rep > 0) ms_min = std::min(ms_min, ms);   // first run warms up
        }
        if (ms_min < best) {
          best = ms_min;
          choice = c;
        }
        if (std::getenv("RBMF_VERBOSE"))
          std::fprintf(stderr, "[rbmf] N=%lld split N1=%d N2=%d: %.4f ms / %d vectors\n", (long long)N, g.N1, g.N2,
                       ms_min, B);
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      tune_cache().put(key, choice);
    }
  }
  ctx->fft_n2[N] = choice;
  *out = make_geom(N, choice);
  return RB_OK;
}


// Split for the binned first stage: the pass-2 workgroup rows F should cover
// a whole bin (F >= w) so that the pass writes the bin means itself; take the
// tuned split when it does, else the supported split nearest to it that does,
// else the one with the most rows.  A split forced with RBMF_FFT_SPLIT is kept.
FftGeom binned_geom(const FftGeom& g, int w) {
  if (pass2_rows(g.N1) >= w || std::getenv("RBMF_FFT_SPLIT")) return g;
  for (int n1 = 4096 / w; n1 >= 64; n1 >>= 1) {
    const FftGeom c = make_geom(g.N, g.log2N - __builtin_ctz((unsigned)n1));
    if (geom_supported(c)) return c;
  }
  for (int n2log = g.log2N; n2log >= 0; --n2log) {
    const FftGeom c = make_geom(g.N, n2log);
    if (geom_supported(c)) return c;   // largest N2, smallest N1: most rows
  }
  return g;
}

// strain -> device pointer (copied into ctx scratch if it is a host array)
rb_status strain_device(rb_ctx ctx, const float* strain, int64_t N, const float** out) {
  RB_CHECK(strain != nullptr, RB_ERR_ARG, "strain is NULL");
  if (is_device_ptr(strain)) {
    *out = strain;
    return RB_OK;
  }
  RB_TRY(ctx->strain.ensure(N * sizeof(float)));
  RB_HIP(hipMemcpyAsync(ctx->strain.p, strain, N * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
  *out = ctx->strain.as<float>();
  return RB_OK;
}

// a1 into caller-provided buffers: work64 (N double2), dspec (nbs float2)
rb_status spectrum_into(rb_ctx ctx, rb_bank bank, const FftGeom& g, const FftTables& tw, const FftTables64& tw64,
                        const float* s, double2* work64, float2* dspec) {
  RB_TRY(fill32(ctx, dspec, 0u, bank->nbs * 2));
  PassArgs a = base_args(bank, g, tw);
  a.sign = -1;
  a.nvec = 1;
  a.real_in = s;
  a.tw64 = tw64;
  a.work64 = work64;
  RB_HIP(launch_pass1(a, IN_REAL, ctx->stream));
  a.cout = dspec;
  RB_HIP(launch_pass2(a, OUT_SPECTRUM, ctx->stream));
  return RB_OK;
}

// a1: whitened band spectrum d[k - kb] = dt w[k] DFT(s)[k] (zero below k_lo)
rb_status step_spectrum(rb_ctx ctx, rb_bank bank, const FftGeom& g, const FftTables& tw, const float* s) {
  FftTables tw32;
  FftTables64 tw64;
  RB_TRY(get_tables(ctx, g, tw32, &tw64));
  RB_TRY(ctx->work64.ensure((size_t)g.N * 16));
  RB_TRY(ctx->dspec.ensure((size_t)bank->nbs * 8));
  ctx->dspec_gen++;
  return spectrum_into(ctx, bank, g, tw, tw64, s, ctx->work64.as<double2>(), ctx->dspec.as<float2>());
}

// Pass 1 / pass 2 over nvec vectors in batches of B (one [B][N] work buffer,
// the context's stream).  Measured: running pass 2 of batch b on a second
// stream beside pass 1 of batch b + 1 (two buffers small enough for the
// Infinity Cache) was slower at every buffer size tried (4.1 ms against
// 3.4 ms for the headline Z stage), the cross-stream ordering costing more
// than the overlap gains.
rb_status pass_pairs(rb_ctx ctx, PassArgs a, int64_t nvec, InKind in, OutKind out) {
  const int64_t N = a.g.N;
  const int B = batch_vectors(N, nvec);
  RB_TRY(ctx->work.ensure((size_t)B * N * 8));
  a.work = ctx->work.as<float2>();
  for (int64_t v0 = 0; v0 < nvec; v0 += B) {
    a.vec_base = (int)v0;
    a.nvec = (int)std::min<int64_t>(B, nvec - v0);
    RB_HIP(launch_pass1(a, in, ctx->stream));
    RB_HIP(launch_pass2(a, out, ctx->stream));
  }
  return RB_OK;
}

// The FP16 intermediate's {s, 1 / s} for the current spectrum in ctx->dspec
// (computed once per spectrum; the bound depends on the split's N2).
rb_status half_scale(rb_ctx ctx, rb_bank bank, const FftGeom& g, const float** hs) {
  if (ctx->hscale_gen != ctx->dspec_gen || ctx->hscale_n2 != g.N2) {
    RB_TRY(ctx->hscale.ensure((size_t)(2 + kHalfScaleParts) * 4));
    RB_HIP(launch_half_scale(ctx->dspec.as<float2>(), bank->nbs, g.N2, ctx->hscale.as<float>() + 2,
                             ctx->hscale.as<float>(), ctx->stream));
    ctx->hscale_gen = ctx->dspec_gen;
    ctx->hscale_n2 = g.N2;
  }
  *hs = ctx->hscale.as<float>();
  return RB_OK;
}

// a2 + a3: Z = IFFT(d conj(P_k)) for all basis vectors, planar storage
// (the basis's storage type, or FP32 into ctx->z32 when force_f32).  With
// fp16_inter and BF16 / FP16 storage the four-step intermediate between the
// passes is kept as FP16 pairs scaled by a power of two chosen from max |d|
// (no overflow for unit-norm vectors), half the intermediate's HBM traffic;
// its rounding spreads over the segment (an error floor that scales with the
// loudest signal), so it is the caller's option, not the default.
rb_status step_basis_outputs(rb_ctx ctx, rb_basis basis, const FftGeom& g, const FftTables& tw,
                             bool force_f32 = false, bool fp16_inter = false) {
  rb_bank bank = basis->bank;
  const int K = basis->K, Kp = force_f32 ? basis->K : basis->Kp;
  const rb_dtype dt = force_f32 ? RB_F32 : basis->dtype;
  DevBuf& zb = force_f32 ? ctx->z32 : ctx->z;
  const size_t esz = dt == RB_F32 ? 4 : 2;
  const int planes = dt == RB_BF16X3 ? 2 : 1;           // BF16X3: hi plane, then lo plane
  const size_t plane_bytes = (size_t)2 * Kp * g.N * esz;
  RB_TRY(zb.ensure(plane_bytes * planes));
  if (Kp > K) {   // zero the padded rows so that 0 * pad never produces NaN
    const size_t off = (size_t)2 * K * g.N * esz, bytes = (size_t)2 * (Kp - K) * g.N * esz;
    for (int p = 0; p < planes; ++p)
      RB_TRY(fill32(ctx, static_cast<char*>(zb.p) + p * plane_bytes + off, 0u, (int64_t)(bytes / 4)));
  }
  PassArgs a = base_args(bank, g, tw);
  a.sign = +1;
  a.d = ctx->dspec.as<float2>();
  a.src = basis->P.as<float2>();
  a.zout = zb.as<float>();
  a.zdtype = (int)dt;
  a.zplane = (int64_t)2 * Kp * g.N;
  if (fp16_inter && (dt == RB_BF16 || dt == RB_F16)) {
    RB_TRY(half_scale(ctx, bank, g, &a.hscale));
    return pass_pairs(ctx, a, K, IN_CORR_H, OUT_Z16_H);
  }
  return pass_pairs(ctx, a, K, IN_CORR, dt == RB_F32 ? OUT_Z32 : OUT_Z16);
}

int64_t trig_capacity(const DevBuf& b) { return (int64_t)(b.bytes / sizeof(TrigRec)); }

// Binned first stage (Sec. III.C): FP32 Z of every basis vector in the
// OUT_ZBIN layout (ctx->zfine, read by the fine reconstruction) and the bin
// means beta_avg in the reconstruction dtype (ctx->z, planar [2Kp][N/w], the
// GEMM's operand), from partial sums written by the same pass-2 launch.
rb_status step_basis_outputs_binned(rb_ctx ctx, rb_basis basis, const FftGeom& g, const FftTables& tw, int w,
                                    bool fp16_inter = false) {
  rb_bank bank = basis->bank;
  const int K = basis->K, Kp = basis->Kp;
  const rb_dtype dt = basis->dtype;
  const int64_t Nb = g.N / w;
  const int G = std::min(pass2_rows(g.N1), w);
  const size_t esz = dt == RB_F32 ? 4 : 2;
  const int planes = dt == RB_BF16X3 ? 2 : 1;
  const size_t plane_bytes = (size_t)2 * Kp * Nb * esz;
  RB_TRY(ctx->z.ensure(plane_bytes * planes));
  if (Kp > K) {
    const size_t off = (size_t)2 * K * Nb * esz, bytes = (size_t)2 * (Kp - K) * Nb * esz;
    for (int p = 0; p < planes; ++p)
      RB_TRY(fill32(ctx, static_cast<char*>(ctx->z.p) + p * plane_bytes + off, 0u, (int64_t)(bytes / 4)));
  }
  // the fine reconstruction reads Z in the basis's storage precision (FP32 for split BF16)
  const int z16 = dt == RB_BF16 ? 1 : dt == RB_F16 ? 2 : 0;
  RB_TRY(ctx->zfine.ensure((size_t)K * g.N * (z16 ? 4 : 8)));
  if (G < w) RB_TRY(ctx->zpart.ensure((size_t)K * (g.N / G) * 8));
  const int B = batch_vectors(g.N, K);
  RB_TRY(ctx->work.ensure((size_t)B * g.N * 8));
  PassArgs a = base_args(bank, g, tw);
  a.sign = +1;
  a.d = ctx->dspec.as<float2>();
  a.src = basis->P.as<float2>();
  a.work = ctx->work.as<float2>();
  a.zfine = ctx->zfine.p;
  a.zfine16 = z16;
  a.zout = ctx->z.as<float>();
  a.zdtype = (int)dt;
  a.zplane = (int64_t)2 * Kp * Nb;
  a.zpart = G < w ? ctx->zpart.as<float2>() : nullptr;
  a.bin_g = G;
  a.bin_w = w;
  // 16-bit storage: the FP16 intermediate, as in step_basis_outputs
  const bool h = fp16_inter && (dt == RB_BF16 || dt == RB_F16);
  if (h) RB_TRY(half_scale(ctx, bank, g, &a.hscale));
  for (int v0 = 0; v0 < K; v0 += B) {
    a.vec_base = v0;
    a.nvec = std::min(B, K - v0);
    RB_HIP(launch_pass1(a, h ? IN_CORR_H : IN_CORR, ctx->stream));
    RB_HIP(launch_pass2(a, h ? OUT_ZBIN_H : OUT_ZBIN, ctx->stream));
  }
  if (G == w) return RB_OK;   // the pass wrote the bin means itself
  BinReduceArgs r;
  std::memset(&r, 0, sizeof(r));
  r.part = ctx->zpart.as<float2>();
  r.N = g.N;
  r.N1 = g.N1;
  r.N2 = g.N2;
  r.G = G;
  r.w = w;
  r.vec_base = 0;
  r.nvec = K;
  r.zavg = ctx->z.p;
  r.dtype = (int)dt;
  r.zscale = 1.f;
  r.zplane = (int64_t)2 * Kp * Nb;
  RB_HIP(launch_bin_reduce(r, ctx->stream));
  return RB_OK;
}

// rho_RB at every sample of the triggering bins appended by basis `basis`
// since the snapshot `snap` of the bin counter; candidates into trig1 / cnt1.
rb_status step_fine(rb_ctx ctx, rb_basis basis, const FftGeom& g, int w, float thr1sq,
                    const unsigned long long* snap, const TrigRec* bins = nullptr, int64_t begin_h = 0,
                    int64_t end_h = 0) {
  FineArgs f;
  std::memset(&f, 0, sizeof(f));
  f.z = ctx->zfine.p;
  f.z16 = basis->dtype == RB_BF16 ? 1 : basis->dtype == RB_F16 ? 2 : 0;
  f.N = g.N;
  f.N1 = g.N1;
  f.N2 = g.N2;
  f.F = pass2_rows(g.N1);
  f.K = basis->K;
  f.w = w;
  f.C = basis->C32.as<float2>();
  f.t0 = basis->t0;
  f.bins = bins ? bins : ctx->trigB.as<TrigRec>();
  f.begin = bins ? nullptr : snap;
  f.end = bins ? nullptr : ctx->counters.as<unsigned long long>() + 2;
  f.begin_h = begin_h;
  f.end_h = end_h;
  f.bins_cap = trig_capacity(ctx->trigB);
  f.thr_sq = thr1sq;
  f.out = ctx->trig1.as<TrigRec>();
  f.out_cap = trig_capacity(ctx->trig1);
  f.out_count = ctx->counters.as<unsigned long long>();
  f.tmpl_count = ctx->cnt1.as<int32_t>();
  RB_HIP(launch_fine_recon(f, 1024, ctx->stream));
  return RB_OK;
}

// Template-method first stage of the binned search (Sec. III.D, Eq. avg_fft2):
// for every template, the band product with the whitened data folded onto
// M = N / w bins with the geometric-sum weights G, an M-point inverse
// transform (the bin means of its SNR series, exactly), and the threshold
// |<rho>_b|^2 >= thr_sq into trigB / cntB (the bin index as the sample).
rb_status step_fold(rb_ctx ctx, rb_bank bank, const FftGeom& gM, int w, float thr_sq) {
  const int64_t N = bank->grid.N;
  if (ctx->gfold_N != N || ctx->gfold_w != w) {   // G[F] for F < N/2, FP64 on the host
    std::vector<float2> G((size_t)(N / 2));
    for (int64_t F = 0; F < N / 2; ++F) {
      if (F == 0) {
        G[0] = make_float2((float)w, 0.f);
        continue;
      }
      // (1 - z^w) / (1 - z), z = e^{2 pi i F / N}
      const double a = 2.0 * M_PI * (double)F / (double)N;
      const cd z(std::cos(a), std::sin(a)), zw(std::cos(a * w), std::sin(a * w));
      const cd g = (1.0 - zw) / (1.0 - z);
      G[(size_t)F] = make_float2((float)g.real(), (float)g.imag());
    }
    RB_TRY(ctx->gfold.ensure(G.size() * sizeof(float2)));
    RB_HIP(hipMemcpyAsync(ctx->gfold.p, G.data(), G.size() * sizeof(float2), hipMemcpyHostToDevice, ctx->stream));
    RB_HIP(hipStreamSynchronize(ctx->stream));
    ctx->gfold_N = N;
    ctx->gfold_w = w;
  }
  FftTables tw;
  RB_TRY(get_tables(ctx, gM, tw));
  const int T = bank->T;
  const int B = batch_vectors(gM.N, T);
  RB_TRY(ctx->work.ensure((size_t)B * gM.N * 8));
  PassArgs a = base_args(bank, gM, tw);
  a.sign = +1;
  a.d = ctx->dspec.as<float2>();
  a.src = bank->w.as<float2>();
  a.sup_lo = bank->sup_lo.as<int32_t>();
  a.sup_hi = bank->sup_hi.as<int32_t>();
  a.gfold = ctx->gfold.as<float2>();
  a.fold_half = w / 2;
  a.fold_inv = 1.f / (float)w;
  a.work = ctx->work.as<float2>();
  a.thr2 = thr_sq;
  a.trig = ctx->trigB.as<TrigRec>();
  a.trig_cap = trig_capacity(ctx->trigB);
  a.trig_count = ctx->counters.as<unsigned long long>() + 2;
  a.tmpl_count = ctx->cntB.as<int32_t>();
  a.tmpl_max = nullptr;
  for (int64_t i0 = 0; i0 < T; i0 += B) {
    a.vec_base = (int)i0;
    a.nvec = (int)std::min<int64_t>(B, T - i0);
    RB_HIP(launch_pass1(a, IN_FOLD, ctx->stream));
    RB_HIP(launch_pass2(a, OUT_THRESH, ctx->stream));
  }
  return RB_OK;
}

// Records of a context's trigger buffers when they are first allocated;
// RBMF_TRIG_RECORDS=<n> starts every buffer at n records instead (the growth
// paths then run on small searches too).
int64_t initial_records(int64_t dflt) {
  const char* e = std::getenv("RBMF_TRIG_RECORDS");
  const int64_t n = e ? std::atoll(e) : dflt;
  return std::max<int64_t>(1, std::min<int64_t>(n, int64_t(1) << 28));
}

rb_status ensure_trigger_scratch(rb_ctx ctx, int T) {
  RB_TRY(ctx->cnt1.ensure((size_t)T * 4));
  RB_TRY(ctx->cnt2.ensure((size_t)T * 4));
  RB_TRY(ctx->off1.ensure((size_t)T * 4));
  RB_TRY(ctx->off2.ensure((size_t)T * 4));
  RB_TRY(ctx->fill1.ensure((size_t)T * 4));
  RB_TRY(ctx->fill2.ensure((size_t)T * 4));
  RB_TRY(ctx->list1.ensure((size_t)T * 4));
  RB_TRY(ctx->list2.ensure((size_t)T * 4));
  RB_TRY(ctx->tmax.ensure((size_t)T * 8));
  RB_TRY(ctx->summary.ensure(8 * 8));
  RB_TRY(ctx->counters.ensure(4 * 8));
  RB_TRY(ctx->cntB.ensure((size_t)T * 4));
  RB_TRY(ctx->flag.ensure(8));
  if (ctx->trig1.bytes == 0) RB_TRY(ctx->trig1.ensure((size_t)initial_records(1 << 22) * sizeof(TrigRec)));
  if (ctx->trig2.bytes == 0) RB_TRY(ctx->trig2.ensure((size_t)initial_records(1 << 20) * sizeof(TrigRec)));
  if (ctx->trigB.bytes == 0) RB_TRY(ctx->trigB.ensure((size_t)initial_records(1 << 20) * sizeof(TrigRec)));
  return RB_OK;
}

// Full matched filter of a template list (or all templates) with the
// threshold epilogue; counts in cnt2, records in trig2, maxima in tmax.
// With d_count (graph mode) nlist is an upper bound and list entries at or
// beyond *d_count are skipped on the device.
// Buffers of the template method's passes: the [B][N] intermediate, the
// whitened data, the trigger records and their counters.
struct MfBufs {
  float2* work;
  int B;
  const float2* d;
  TrigRec* trig;
  int64_t trig_cap;
  unsigned long long* trig_count;
  int32_t* tmpl_count;
  unsigned long long* tmpl_max;   // NULL: no per-template maxima
};

rb_status mf_passes(rb_ctx ctx, rb_bank bank, const FftGeom& g, const FftTables& tw, const int32_t* list,
                    int64_t nlist, float thr2sq, const int32_t* d_count, const MfBufs& b) {
  PassArgs a = base_args(bank, g, tw);
  a.sign = +1;
  a.d = b.d;
  a.src = bank->w.as<float2>();
  a.sup_lo = bank->sup_lo.as<int32_t>();
  a.sup_hi = bank->sup_hi.as<int32_t>();
  a.work = b.work;
  a.vec_list = list;
  a.d_count = d_count;
  a.thr2 = thr2sq;
  a.trig = b.trig;
  a.trig_cap = b.trig_cap;
  a.trig_count = b.trig_count;
  a.tmpl_count = b.tmpl_count;
  a.tmpl_max = b.tmpl_max;
  for (int64_t i0 = 0; i0 < nlist; i0 += b.B) {
    a.vec_base = (int)i0;
    a.nvec = (int)std::min<int64_t>(b.B, nlist - i0);
    RB_HIP(launch_pass1(a, IN_CORR, ctx->stream));
    RB_HIP(launch_pass2(a, OUT_THRESH, ctx->stream));
  }
  return RB_OK;
}

rb_status step_mf(rb_ctx ctx, rb_bank bank, const FftGeom& g, const FftTables& tw, const int32_t* list,
                  int64_t nlist, float thr2sq, const int32_t* d_count = nullptr) {
  PassArgs a = base_args(bank, g, tw);
  a.sign = +1;
  a.d = ctx->dspec.as<float2>();
  a.src = bank->w.as<float2>();
  a.sup_lo = bank->sup_lo.as<int32_t>();
  a.sup_hi = bank->sup_hi.as<int32_t>();
  a.vec_list = list;
  a.d_count = d_count;
  a.thr2 = thr2sq;
  a.trig = ctx->trig2.as<TrigRec>();
  a.trig_cap = trig_capacity(ctx->trig2);
  a.trig_count = ctx->counters.as<unsigned long long>() + 1;
  a.tmpl_count = ctx->cnt2.as<int32_t>();
  a.tmpl_max = ctx->want_peaks ? ctx->tmax.as<unsigned long long>() : nullptr;
  return pass_pairs(ctx, a, nlist, IN_CORR, OUT_THRESH);
}

// scan cnt -> offsets/list and read the summary {total, nlist, maxcount, flag}
rb_status scan_and_read(rb_ctx ctx, int T, DevBuf& cnt, DevBuf& off, DevBuf& fill, DevBuf& list,
                        int64_t sum_host[3]) {
  RB_HIP(launch_scan_counts(cnt.as<int32_t>(), T, off.as<int32_t>(), fill.as<int32_t>(), list.as<int32_t>(),
                            ctx->summary.as<int64_t>(), ctx->stream));
  RB_HIP(hipMemcpyAsync(sum_host, ctx->summary.p, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  RB_HIP(hipStreamSynchronize(ctx->stream));
  return RB_OK;
}

// Stage-2 records (trig2, cnt2, off2, list2) -> sorted rb_trigger in final_out
rb_status step_sort(rb_ctx ctx, int T, int64_t total, int64_t nlist) {
  RB_TRY(ctx->recs.ensure(std::max<size_t>(16, (size_t)total * sizeof(TrigRec))));
  RB_TRY(ctx->tmp.ensure(std::max<size_t>(16, (size_t)total * sizeof(TrigRec))));
  RB_TRY(ctx->final_out.ensure(std::max<size_t>(16, (size_t)total * sizeof(rb_trigger))));
  RB_HIP(launch_scatter_triggers(ctx->trig2.as<TrigRec>(), total, nullptr, ctx->off2.as<int32_t>(),
                                 ctx->fill2.as<int32_t>(), ctx->recs.as<TrigRec>(), ctx->stream));
  RB_HIP(launch_segment_sort(ctx->recs.as<TrigRec>(), ctx->tmp.as<TrigRec>(), ctx->off2.as<int32_t>(),
                             ctx->cnt2.as<int32_t>(), ctx->list2.as<int32_t>(), (int)nlist, ctx->final_out.p,
                             nullptr, 0, ctx->stream));
  (void)T;
  return RB_OK;
}

rb_status copy_out(rb_ctx ctx, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return RB_OK;
  const hipMemcpyKind kind = is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  RB_HIP(hipMemcpyAsync(dst, src, bytes, kind, ctx->stream));
  return RB_OK;
}

void record(rb_ctx ctx, rb_stats* st, int i) {
  if (st) (void)hipEventRecord(ctx->ev[i], ctx->stream);
}

rb_status validate_ctx(rb_ctx ctx) {
  RB_CHECK(ctx != nullptr, RB_ERR_ARG, "context is NULL");
  RB_HIP(hipSetDevice(ctx->device));
  return RB_OK;
}

// Second stage + sort + output shared by rb_filter and mf_full.
rb_status finish_stage2(rb_ctx ctx, rb_bank bank, rb_trigger* out, int64_t cap, int64_t* n_out, rb_peak* peaks,
                        int64_t sum2[3]) {
  const int T = bank->T;
  const int64_t total = sum2[0];
  *n_out = total;
  if (peaks) {
    RB_TRY(ctx->peaks.ensure((size_t)T * sizeof(rb_peak)));
    RB_HIP(launch_peaks_from_max(ctx->tmax.as<unsigned long long>(), T, ctx->peaks.p, ctx->stream));
    RB_TRY(copy_out(ctx, peaks, ctx->peaks.p, (size_t)T * sizeof(rb_peak)));
  }
  if (total > cap) {
    RB_HIP(hipStreamSynchronize(ctx->stream));
    set_error("trigger capacity " + std::to_string(cap) + " < required " + std::to_string(total));
    return RB_ERR_CAPACITY;
  }
  RB_CHECK(out != nullptr || total == 0, RB_ERR_ARG, "out is NULL");
  RB_TRY(step_sort(ctx, T, total, sum2[1]));
  RB_TRY(copy_out(ctx, out, ctx->final_out.p, (size_t)total * sizeof(rb_trigger)));
  return RB_OK;
}

}  // namespace

// ====================================================================== context
extern "C" const char* rb_last_error(void) { return rbmf::last_error_cstr(); }

extern "C" rb_status rb_ctx_create(int device, void* hip_stream, rb_ctx* out) {
  RB_CHECK(out != nullptr, RB_ERR_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  RB_HIP(hipGetDeviceCount(&n));
  RB_CHECK(device >= 0 && device < n, RB_ERR_DEVICE, "no HIP device " + std::to_string(device));
  hipDeviceProp_t prop;
  RB_HIP(hipGetDeviceProperties(&prop, device));
  RB_CHECK(std::strncmp(prop.gcnArchName, "gfx950", 6) == 0, RB_ERR_DEVICE,
           std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
  RB_HIP(hipSetDevice(device));
  void* noalloc = nullptr;
  RB_HIP(noalloc_scratch_init(device, &noalloc));
  auto c = new (std::nothrow) rb_ctx_s;
  RB_CHECK(c != nullptr, RB_ERR_OOM, "host allocation failed");
  c->device = device;
  c->noalloc = noalloc;
  c->arch = prop.gcnArchName;
  c->stream = static_cast<hipStream_t>(hip_stream);
  for (auto& e : c->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      delete c;
      set_error("hipEventCreate failed");
      return RB_ERR_DEVICE;
    }
  }
  *out = c;
  return RB_OK;
}

extern "C" rb_status rb_ctx_destroy(rb_ctx ctx) {
  RB_CHECK(ctx != nullptr, RB_ERR_ARG, "context is NULL");
  RB_CHECK(ctx->live == 0, RB_ERR_ARG, "context still has live banks or bases");
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& e : ctx->ev) (void)hipEventDestroy(e);
  delete ctx;
  return RB_OK;
}

// ====================================================================== bank
extern "C" rb_status rb_bank_create(rb_ctx ctx, const rb_grid* grid, const double* psd, int32_t T,
                                    rb_bank_fill_fn fill, void* user, rb_bank* out) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(out != nullptr && grid != nullptr && psd != nullptr && fill != nullptr, RB_ERR_ARG,
           "NULL argument");
  *out = nullptr;
  const int64_t N = grid->N;
  RB_CHECK(N >= 4096 && N <= (int64_t(1) << 21) && (N & (N - 1)) == 0, RB_ERR_ARG,
           "N must be a power of two in [2^12, 2^21]");
  RB_CHECK(std::isfinite(grid->fs) && grid->fs > 0, RB_ERR_ARG, "fs must be > 0");
  RB_CHECK(std::isfinite(grid->f_low) && grid->f_low > 0 && grid->f_low < grid->fs / 2, RB_ERR_ARG,
           "f_low must be in (0, fs/2)");
  RB_CHECK(T >= 1 && T <= (1 << 24), RB_ERR_ARG, "T must be in [1, 2^24]");
  const double df = grid->fs / (double)N, dt = 1.0 / grid->fs;
  const int64_t k_lo = (int64_t)std::ceil(grid->f_low / df - 1e-9), k_hi = N / 2 - 1;
  RB_CHECK(k_lo >= 1 && k_lo <= k_hi, RB_ERR_ARG, "empty band");
  for (int64_t k = k_lo; k <= k_hi; ++k)
    RB_CHECK(std::isfinite(psd[k]) && psd[k] > 0, RB_ERR_ARG,
             "PSD must be finite and positive on the band (bin " + std::to_string(k) + ")");
  std::unique_ptr<rb_bank_s> b(new (std::nothrow) rb_bank_s);
  RB_CHECK(b != nullptr, RB_ERR_OOM, "host allocation failed");
  b->ctx = ctx;
  b->grid = *grid;
  b->T = T;
  b->k_lo = k_lo;
  b->k_hi = k_hi;
  b->kb = (k_lo / 16) * 16;
  b->nbs = N / 2 - b->kb;
  const int64_t nbs = b->nbs, kb = b->kb;
  std::vector<double> w(nbs, 0.0);
  std::vector<double> wd(nbs, 0.0);
  for (int64_t k = k_lo; k <= k_hi; ++k) {
    w[k - kb] = std::sqrt(4.0 * df / psd[k]);
    wd[k - kb] = dt * w[k - kb];
  }
  RB_TRY(b->wd.ensure(nbs * sizeof(double)));
  RB_HIP(hipMemcpy(b->wd.p, wd.data(), nbs * sizeof(double), hipMemcpyHostToDevice));
  RB_TRY(b->w.ensure((size_t)T * nbs * sizeof(float2)));
  RB_TRY(b->sup_lo.ensure((size_t)T * 4));
  RB_TRY(b->sup_hi.ensure((size_t)T * 4));
  b->sigma.assign(T, 0.0);
  std::vector<int32_t> slo(T), shi(T);
  // templates per fill callback: 512 MB of FP64 host values (enough rows for a
  // multi-threaded generator at N = 2^20)
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(T, (int64_t(512) << 20) / (nbs * 16)));
  std::vector<double> hbuf((size_t)chunk * nbs * 2);
  HostPinned stage;
  RB_TRY(stage.ensure((size_t)chunk * nbs * sizeof(float2)));
  std::string bad;
  for (int64_t t0 = 0; t0 < T; t0 += chunk) {
    const int64_t t1 = std::min<int64_t>(T, t0 + chunk);
    RB_HIP(hipStreamSynchronize(ctx->stream));   // staging buffer reuse
    const int rc = fill(user, (int32_t)t0, (int32_t)t1, kb, N / 2, hbuf.data());
    RB_CHECK(rc == 0, RB_ERR_CALLBACK, "bank fill callback returned " + std::to_string(rc));
    float2* st = static_cast<float2*>(stage.p);
    std::atomic<int> nbad(0);
    parallel_for(t1 - t0, [&](int64_t i) {
      const double* h = &hbuf[(size_t)i * nbs * 2];
      double s2 = 0.0;
      int64_t lo = -1, hi = -1;
      for (int64_t k = k_lo; k <= k_hi; ++k) {
        const double re = h[2 * (k - kb)], im = h[2 * (k - kb) + 1];
        const double a2 = (re * re + im * im) * w[k - kb] * w[k - kb];
        s2 += a2;
        if (a2 > 0.0) {
          if (lo < 0) lo = k;
          hi = k;
        }
      }
      const double sg = std::sqrt(s2);
      b->sigma[t0 + i] = sg;
      if (!(sg > 0.0) || !std::isfinite(sg)) {
        nbad++;
        return;
      }
      float2* o = st + (size_t)i * nbs;
      for (int64_t k = kb; k < k_lo; ++k) o[k - kb] = make_float2(0.f, 0.f);
      for (int64_t k = k_lo; k <= k_hi; ++k) {
        const double f = w[k - kb] / sg;
        o[k - kb] = make_float2((float)(h[2 * (k - kb)] * f), (float)(h[2 * (k - kb) + 1] * f));
      }
      slo[t0 + i] = (int32_t)lo;
      shi[t0 + i] = (int32_t)hi;
    });
    RB_CHECK(nbad.load() == 0, RB_ERR_ARG, "a template has zero or non-finite norm on the band");
    RB_HIP(hipMemcpyAsync(b->w.as<float2>() + (size_t)t0 * nbs, st, (size_t)(t1 - t0) * nbs * sizeof(float2),
                          hipMemcpyHostToDevice, ctx->stream));
  }
  RB_HIP(hipMemcpy(b->sup_lo.p, slo.data(), (size_t)T * 4, hipMemcpyHostToDevice));
  RB_HIP(hipMemcpy(b->sup_hi.p, shi.data(), (size_t)T * 4, hipMemcpyHostToDevice));
  RB_HIP(hipStreamSynchronize(ctx->stream));
  ctx->live++;
  *out = b.release();
  return RB_OK;
}

extern "C" rb_status rb_bank_free(rb_bank bank) {
  RB_CHECK(bank != nullptr, RB_ERR_ARG, "bank is NULL");
  RB_CHECK(bank->live_bases == 0, RB_ERR_ARG, "bank still has live bases");
  (void)hipSetDevice(bank->ctx->device);
  (void)hipStreamSynchronize(bank->ctx->stream);
  bank->ctx->live--;
  delete bank;
  return RB_OK;
}

extern "C" rb_status rb_bank_info(rb_bank bank, int32_t* T, int64_t* k_lo, int64_t* k_hi, double* sigma) {
  RB_CHECK(bank != nullptr, RB_ERR_ARG, "bank is NULL");
  if (T) *T = bank->T;
  if (k_lo) *k_lo = bank->k_lo;
  if (k_hi) *k_hi = bank->k_hi;
  if (sigma) {
    // sigma of the unwhitened templates (the bank stores w_j = h_j w / sigma_j)
    std::memcpy(sigma, bank->sigma.data(), bank->sigma.size() * sizeof(double));
  }
  return RB_OK;
}

// ====================================================================== basis
namespace {

struct BasisWork {
  DevBuf Q, Y, B, M, R, ws, norms, scale;
};

// Orthonormalise the columns of Y (T x L, complex128, row-major ld = L) in
// place of Q: `passes` times "scale, Gram, eigen-decompose" (SVQB).  Returns
// the kept column count in *Lout.
rb_status svqb(rb_ctx ctx, BasisWork& bw, const double2* Y, int64_t T, int L, double2* Qout, int* Lout,
               int passes = 2) {
  const double2* src = Y;
  int Lc = L;
  for (int pass = 0; pass < passes; ++pass) {
    RB_TRY(bw.M.ensure((size_t)Lc * Lc * 16));
    ZOperand A{src, 0, 1, Lc, 1};
    ZOperand Bo{src, 0, Lc, 1, 0};
    RB_HIP(launch_zgemm(Lc, Lc, T, A, Bo, bw.M.as<double2>(), Lc, 0, bw.ws.as<double2>(),
                        (int64_t)(bw.ws.bytes / 16), ctx->stream));
    std::vector<cd> G((size_t)Lc * Lc);
    RB_HIP(hipMemcpyAsync(G.data(), bw.M.p, G.size() * 16, hipMemcpyDeviceToHost, ctx->stream));
    RB_HIP(hipStreamSynchronize(ctx->stream));
    std::vector<double> dsc(Lc);
    for (int i = 0; i < Lc; ++i) {
      const double g = G[(size_t)i * Lc + i].real();
      dsc[i] = g > 0 ? 1.0 / std::sqrt(g) : 0.0;
    }
    for (int i = 0; i < Lc; ++i)
      for (int j = 0; j < Lc; ++j) G[(size_t)i * Lc + j] *= dsc[i] * dsc[j];
    std::vector<double> th;
    std::vector<cd> W;
    RB_CHECK(herm_eig_desc(Lc, G, th, W), RB_ERR_NUMERIC, "eigensolver did not converge");
    int keep = 0;
    while (keep < Lc && th[keep] > 1e-12 * th[0]) ++keep;
    RB_CHECK(keep > 0, RB_ERR_NUMERIC, "rank-zero subspace");
    std::vector<cd> Rm((size_t)Lc * keep);
    for (int i = 0; i < Lc; ++i)
      for (int j = 0; j < keep; ++j) Rm[(size_t)i * keep + j] = dsc[i] * W[(size_t)i * Lc + j] / std::sqrt(th[j]);
    RB_TRY(bw.R.ensure(Rm.size() * 16));
    RB_HIP(hipMemcpyAsync(bw.R.p, Rm.data(), Rm.size() * 16, hipMemcpyHostToDevice, ctx->stream));
    RB_HIP(hipStreamSynchronize(ctx->stream));   // Rm is pageable and local
    // pass 0: Y -> Qout; pass 1: Qout -> Y (then copied back to Qout)
    double2* outp = (pass == 0) ? Qout : bw.Y.as<double2>();
    ZOperand A2{src, 0, Lc, 1, 0};
    ZOperand B2{bw.R.p, 0, keep, 1, 0};
    RB_HIP(launch_zgemm(T, keep, Lc, A2, B2, outp, keep, 0, bw.ws.as<double2>(), (int64_t)(bw.ws.bytes / 16),
                        ctx->stream));
    src = outp;
    Lc = keep;
  }
  // after an even number of passes the result is in Y
  if (src != Qout) RB_HIP(hipMemcpyAsync(Qout, src, (size_t)T * Lc * 16, hipMemcpyDeviceToDevice, ctx->stream));
  *Lout = Lc;
  return RB_OK;
}

}  // namespace

extern "C" rb_status rb_build_basis(rb_ctx ctx, rb_bank bank, int32_t rank, double tol, rb_dtype dtype,
                                    rb_basis* out, int32_t* rank_out, double* energy_out) {
  RB_CHECK(bank != nullptr, RB_ERR_ARG, "bank is NULL");
  return rb_build_basis_range(ctx, bank, 0, bank->T, rank, tol, dtype, out, rank_out, energy_out);
}

extern "C" rb_status rb_basis_info(rb_basis basis, int32_t* t0, int32_t* t1, int32_t* rank, double* energy) {
  RB_CHECK(basis != nullptr, RB_ERR_ARG, "basis is NULL");
  if (t0) *t0 = basis->t0;
  if (t1) *t1 = basis->t0 + basis->T;
  if (rank) *rank = basis->K;
  if (energy) *energy = basis->energy;
  return RB_OK;
}

namespace {

// Leading right singular subspace of the stored rows W (T x n complex64, row
// stride ld), i.e. the leading eigenvectors of the covariance W^H W
// (Sec. II.A; Sec. III.A-B): randomized subspace iteration with SVQB
// orthonormalisation and a Rayleigh-Ritz step, the subspace doubled until
// the rank rule is met with spare vectors.  On return bw.B = W^H Q (n x Lc),
// theta / S the Ritz values and vectors of Q^H W W^H Q, K the kept rank.
rb_status subspace_pca(rb_ctx ctx, BasisWork& bw, const float2* W, int64_t T, int64_t n, int64_t ld, double trace,
                       int32_t rank, double tol, std::vector<double>& theta, std::vector<cd>& S, int& Lc, int& K) {
  hipStream_t s = ctx->stream;
  const ZOperand Wop{W, 1, ld, 1, 0};    // T x n
  const ZOperand WHop{W, 1, 1, ld, 1};   // n x T  (conjugate transpose)
  const int over = 32;
  int L = (int)std::min<int64_t>(T, rank > 0 ? (int64_t)rank + std::max(over, rank / 4) : 160);
  const int q = 4;
  Lc = 0;
  K = 0;
  std::mt19937_64 rng(0x2110131150ull);
  std::normal_distribution<double> nd;
  for (;;) {
    // random start, orthonormalised
    std::vector<cd> Om((size_t)T * L);
    for (auto& v : Om) v = cd(nd(rng), nd(rng));
    RB_TRY(bw.Q.ensure((size_t)T * L * 16));
    RB_TRY(bw.Y.ensure((size_t)T * L * 16));
    RB_HIP(hipMemcpyAsync(bw.Y.p, Om.data(), Om.size() * 16, hipMemcpyHostToDevice, s));
    RB_TRY(svqb(ctx, bw, bw.Y.as<double2>(), T, L, bw.Q.as<double2>(), &Lc));
    RB_TRY(bw.B.ensure((size_t)n * Lc * 16));
    if (Lc < T) {
      for (int it = 0; it < q; ++it) {
        ZOperand Qop{bw.Q.p, 0, Lc, 1, 0};
        RB_HIP(launch_zgemm(n, Lc, T, WHop, Qop, bw.B.as<double2>(), Lc, 0, bw.ws.as<double2>(),
                            (int64_t)(bw.ws.bytes / 16), s));
        ZOperand Bop{bw.B.p, 0, Lc, 1, 0};
        RB_HIP(launch_zgemm(T, Lc, n, Wop, Bop, bw.Y.as<double2>(), Lc, 0, bw.ws.as<double2>(),
                            (int64_t)(bw.ws.bytes / 16), s));
        int Ln = 0;   // one SVQB pass between products, two after the last
        RB_TRY(svqb(ctx, bw, bw.Y.as<double2>(), T, Lc, bw.Q.as<double2>(), &Ln, it + 1 < q ? 1 : 2));
        Lc = Ln;
      }
    }
    // Rayleigh-Ritz: B = W^H Q, M = B^H B = Q^H G Q
    {
      ZOperand Qop{bw.Q.p, 0, Lc, 1, 0};
      RB_HIP(launch_zgemm(n, Lc, T, WHop, Qop, bw.B.as<double2>(), Lc, 0, bw.ws.as<double2>(),
                          (int64_t)(bw.ws.bytes / 16), s));
      RB_TRY(bw.M.ensure((size_t)Lc * Lc * 16));
      ZOperand BH{bw.B.p, 0, 1, Lc, 1};
      ZOperand Bo{bw.B.p, 0, Lc, 1, 0};
      RB_HIP(launch_zgemm(Lc, Lc, n, BH, Bo, bw.M.as<double2>(), Lc, 0, bw.ws.as<double2>(),
                          (int64_t)(bw.ws.bytes / 16), s));
      std::vector<cd> Mh((size_t)Lc * Lc);
      RB_HIP(hipMemcpyAsync(Mh.data(), bw.M.p, Mh.size() * 16, hipMemcpyDeviceToHost, s));
      RB_HIP(hipStreamSynchronize(s));
      RB_CHECK(herm_eig_desc(Lc, Mh, theta, S), RB_ERR_NUMERIC, "eigensolver did not converge");
    }
    int npos = 0;
    while (npos < Lc && theta[npos] > 1e-14 * theta[0]) ++npos;
    if (std::getenv("RBMF_VERBOSE")) {
      double cs = 0.0;
      for (int k = 0; k < npos; ++k) cs += theta[k];
      std::fprintf(stderr, "[rbmf] basis T=%lld: subspace %d, captured energy %.6f\n", (long long)T, Lc,
                   cs / trace);
    }
    if (rank > 0) {
      K = std::min(rank, npos);
      break;
    }
    double cum = 0.0;
    K = 0;
    while (K < npos && cum < (1.0 - tol) * trace) cum += theta[K++];
    // enough: the tolerance is met with `over` spare Ritz vectors, or the
    // subspace already spans every direction above the round-off floor
    // (the orthonormalisation dropped columns: the bank's numerical rank is Lc)
    if (cum >= (1.0 - tol) * trace && (K + over <= Lc || Lc >= T || Lc < L)) break;
    if (Lc >= T || L >= T || Lc < L) break;   // cannot grow further (or nothing left to find)
    L = (int)std::min<int64_t>(T, 2 * (int64_t)L);
  }
  RB_CHECK(K >= 1, RB_ERR_NUMERIC, "basis has rank zero");
  return RB_OK;
}

// The K leading Ritz vectors BS = B S[:, :K] (n x K, complex128).
rb_status ritz_vectors(rb_ctx ctx, BasisWork& bw, int64_t n, int Lc, int K, const std::vector<cd>& S, DevBuf& BS,
                       int64_t ldb = 0) {
  hipStream_t s = ctx->stream;
  std::vector<cd> Sk((size_t)Lc * K);
  for (int i = 0; i < Lc; ++i)
    for (int k = 0; k < K; ++k) Sk[(size_t)i * K + k] = S[(size_t)i * Lc + k];
  DevBuf Sd;
  RB_TRY(Sd.ensure(Sk.size() * 16));
  RB_HIP(hipMemcpyAsync(Sd.p, Sk.data(), Sk.size() * 16, hipMemcpyHostToDevice, s));
  RB_TRY(BS.ensure((size_t)n * K * 16));
  ZOperand Bo{bw.B.p, 0, ldb > 0 ? ldb : Lc, 1, 0};
  ZOperand So{Sd.p, 0, K, 1, 0};
  RB_HIP(launch_zgemm(n, K, Lc, Bo, So, BS.as<double2>(), K, 0, bw.ws.as<double2>(), (int64_t)(bw.ws.bytes / 16),
                      s));
  RB_HIP(hipStreamSynchronize(s));   // Sk is pageable and local
  return RB_OK;
}

// Block Lanczos with full reorthogonalisation for the leading eigenpairs of
// the Gram matrix G = W W^H (T x T) of the stored rows (Sec. II.A: its
// eigenvectors give the basis; the paper runs a Lanczos eigensolver on the
// covariance, Sec. III.B), applied as G X = W (W^H X) without forming G.
// Krylov blocks X_0, X_1, ... of `b` columns: X_{j+1} orthonormalises
// G X_j after two passes of classical Gram-Schmidt against every earlier
// block (columns that vanish are dropped; an empty block means the Krylov
// space is invariant).  After each block the Rayleigh-Ritz problem
// M = V^H G V is solved on the host; the residuals G V s - theta V s of the
// Ritz pairs that the rank rule keeps are formed on the device.  Stops when
// their norms are <= 1e-10 theta_1 (or the space reaches T).  On return bw.B holds W^H V (n x ldb, ldb >= Lc), and
// theta / S / Lc / K as subspace_pca's.
rb_status lanczos_pca(rb_ctx ctx, BasisWork& bw, const float2* W, int64_t T, int64_t n, int64_t ld, double trace,
                      int32_t rank, double tol, std::vector<double>& theta, std::vector<cd>& S, int& Lc, int& K,
                      int64_t& ldb) {
  hipStream_t s = ctx->stream;
  const ZOperand Wop{W, 1, ld, 1, 0};    // T x n
  const ZOperand WHop{W, 1, 1, ld, 1};   // n x T  (conjugate transpose)
  const int b = (int)std::min<int64_t>(T, rank > 0 ? std::max(16, std::min(64, rank / 4)) : 32);
  // Krylov dimension cap: the rank (or a first guess) several times over, at most T
  const int64_t want = rank > 0 ? rank : 160;
  int64_t cap = std::min<int64_t>(T, std::max<int64_t>(4 * want + 4 * b, 8 * b));
  DevBuf V, GV, Y, H, P;
  auto grow = [&](int64_t c) -> rb_status {    // column capacity of V, GV, B
    cap = c;
    DevBuf v2, g2, b2;
    RB_TRY(v2.ensure((size_t)T * cap * 16));
    RB_TRY(g2.ensure((size_t)T * cap * 16));
    RB_TRY(b2.ensure((size_t)n * cap * 16));
    if (Lc > 0) {
      RB_HIP(hipMemcpy2DAsync(v2.p, cap * 16, V.p, ldb * 16, (size_t)Lc * 16, T, hipMemcpyDeviceToDevice, s));
      RB_HIP(hipMemcpy2DAsync(g2.p, cap * 16, GV.p, ldb * 16, (size_t)Lc * 16, T, hipMemcpyDeviceToDevice, s));
      RB_HIP(hipMemcpy2DAsync(b2.p, cap * 16, bw.B.p, ldb * 16, (size_t)Lc * 16, n, hipMemcpyDeviceToDevice, s));
      RB_HIP(hipStreamSynchronize(s));
    }
    V = std::move(v2);
    GV = std::move(g2);
    bw.B = std::move(b2);
    ldb = cap;
    return RB_OK;
  };
  Lc = 0;
  K = 0;
  ldb = 0;
  RB_TRY(grow(cap));
  RB_TRY(Y.ensure((size_t)T * b * 16));
  RB_TRY(bw.Y.ensure((size_t)T * b * 16));
  RB_TRY(bw.Q.ensure((size_t)T * b * 16));
  // random start block, orthonormalised
  std::mt19937_64 rng(0x2110131151ull);
  std::normal_distribution<double> nd;
  {
    std::vector<cd> Om((size_t)T * b);
    for (auto& v : Om) v = cd(nd(rng), nd(rng));
    RB_HIP(hipMemcpyAsync(Y.p, Om.data(), Om.size() * 16, hipMemcpyHostToDevice, s));
    int kept = 0;
    RB_TRY(svqb(ctx, bw, Y.as<double2>(), T, b, bw.Q.as<double2>(), &kept));
    RB_HIP(hipMemcpy2DAsync(V.p, ldb * 16, bw.Q.p, (size_t)kept * 16, (size_t)kept * 16, T, hipMemcpyDeviceToDevice,
                            s));
    RB_HIP(hipStreamSynchronize(s));   // Om is pageable and local
    Lc = kept;
  }
  int64_t c0 = 0;          // first column of the newest block
  bool final_pass = false; // the Krylov space stopped growing: solve once more on it and stop
  for (;;) {
    const int bj = (int)(Lc - c0);
    // W^H X_j -> B columns [c0, Lc); G X_j -> GV columns [c0, Lc)
    {
      ZOperand Xop{V.as<double2>() + c0, 0, ldb, 1, 0};
      RB_HIP(launch_zgemm(n, bj, T, WHop, Xop, bw.B.as<double2>() + c0, ldb, 0, bw.ws.as<double2>(),
                          (int64_t)(bw.ws.bytes / 16), s));
      ZOperand Bop{bw.B.as<double2>() + c0, 0, ldb, 1, 0};
      RB_HIP(launch_zgemm(T, bj, n, Wop, Bop, GV.as<double2>() + c0, ldb, 0, bw.ws.as<double2>(),
                          (int64_t)(bw.ws.bytes / 16), s));
    }
    const bool too_small = !final_pass && rank > 0 && Lc < std::min<int64_t>(T, (int64_t)rank + b) && Lc + b <= T;
    // Rayleigh-Ritz on V (Lc columns): M = V^H GV
    std::vector<cd> Mh((size_t)Lc * Lc);
    if (!too_small) {
      RB_TRY(H.ensure((size_t)Lc * Lc * 16));
      ZOperand VH{V.p, 0, 1, ldb, 1};
      ZOperand GVo{GV.p, 0, ldb, 1, 0};
      RB_HIP(launch_zgemm(Lc, Lc, T, VH, GVo, H.as<double2>(), Lc, 0, bw.ws.as<double2>(),
                          (int64_t)(bw.ws.bytes / 16), s));
      RB_HIP(hipMemcpyAsync(Mh.data(), H.p, Mh.size() * 16, hipMemcpyDeviceToHost, s));
      RB_HIP(hipStreamSynchronize(s));
    }
    double worst = 0.0;
    int npos = 0;
    if (!too_small) {
    // symmetrise (rounding) and solve
    for (int i = 0; i < Lc; ++i)
      for (int j = 0; j < i; ++j) {
        const cd a = 0.5 * (Mh[(size_t)i * Lc + j] + std::conj(Mh[(size_t)j * Lc + i]));
        Mh[(size_t)i * Lc + j] = a;
        Mh[(size_t)j * Lc + i] = std::conj(a);
      }
    RB_CHECK(herm_eig_desc((int)Lc, Mh, theta, S), RB_ERR_NUMERIC, "eigensolver did not converge");
    npos = 0;
    while (npos < Lc && theta[npos] > 1e-14 * theta[0]) ++npos;
    if (rank > 0) {
      K = (int)std::min<int64_t>(rank, npos);
    } else {
      double cum = 0.0;
      K = 0;
      while (K < npos && cum < (1.0 - tol) * trace) cum += theta[K++];
    }
    // residuals of the pairs that are kept, formed directly (the difference
    // s^H (GV)^H GV s - theta^2 cannot resolve residuals below ~1e-8 theta_1):
    // R = GV S_K - V S_K diag(theta) (T x K), |R e_k| from the diagonal of R^H R
    {
      std::vector<cd> Sk((size_t)Lc * K), St((size_t)Lc * K);
      for (int i = 0; i < Lc; ++i)
        for (int k = 0; k < K; ++k) {
          Sk[(size_t)i * K + k] = S[(size_t)i * Lc + k];
          St[(size_t)i * K + k] = -theta[k] * S[(size_t)i * Lc + k];
        }
      DevBuf Sd, Std, Rd, RR;
      RB_TRY(Sd.ensure(Sk.size() * 16));
      RB_TRY(Std.ensure(St.size() * 16));
      RB_TRY(Rd.ensure((size_t)T * K * 16));
      RB_TRY(RR.ensure((size_t)K * K * 16));
      RB_HIP(hipMemcpyAsync(Sd.p, Sk.data(), Sk.size() * 16, hipMemcpyHostToDevice, s));
      RB_HIP(hipMemcpyAsync(Std.p, St.data(), St.size() * 16, hipMemcpyHostToDevice, s));
      ZOperand GVo{GV.p, 0, ldb, 1, 0};
      ZOperand Vo{V.p, 0, ldb, 1, 0};
      ZOperand So{Sd.p, 0, K, 1, 0};
      ZOperand Sto{Std.p, 0, K, 1, 0};
      RB_HIP(launch_zgemm(T, K, Lc, GVo, So, Rd.as<double2>(), K, 0, bw.ws.as<double2>(),
                          (int64_t)(bw.ws.bytes / 16), s));
      RB_HIP(launch_zgemm(T, K, Lc, Vo, Sto, Rd.as<double2>(), K, 1, bw.ws.as<double2>(),
                          (int64_t)(bw.ws.bytes / 16), s));
      ZOperand RH{Rd.p, 0, 1, K, 1};
      ZOperand Ro{Rd.p, 0, K, 1, 0};
      RB_HIP(launch_zgemm(K, K, T, RH, Ro, RR.as<double2>(), K, 0, bw.ws.as<double2>(),
                          (int64_t)(bw.ws.bytes / 16), s));
      std::vector<cd> rr((size_t)K * K);
      RB_HIP(hipMemcpyAsync(rr.data(), RR.p, rr.size() * 16, hipMemcpyDeviceToHost, s));
      RB_HIP(hipStreamSynchronize(s));   // Sk / St are pageable and local
      for (int k = 0; k < K; ++k) worst = std::max(worst, std::sqrt(std::max(0.0, rr[(size_t)k * K + k].real())));
    }
    }
    const bool energy_ok = too_small || rank > 0 || K < npos || Lc >= T;   // the rule is met inside the space
    const bool spare = Lc >= K + b;
    if (std::getenv("RBMF_VERBOSE") && !too_small)
      std::fprintf(stderr, "[rbmf] lanczos T=%lld: %d columns, K %d, worst residual %.3e theta_1 %.3e\n",
                   (long long)T, Lc, K, worst, theta[0]);
    if (final_pass || (!too_small && ((energy_ok && spare && worst <= 1e-10 * theta[0]) || Lc >= T))) break;
    // next block: G X_j orthogonalised against every block (two passes), then orthonormalised
    const int64_t nb_next = std::min<int64_t>(b, T - Lc);
    if (Lc + nb_next > cap) RB_TRY(grow(std::min<int64_t>(T, 2 * cap)));
    RB_HIP(hipMemcpy2DAsync(Y.p, (size_t)bj * 16, GV.as<double2>() + c0, ldb * 16, (size_t)bj * 16, T,
                            hipMemcpyDeviceToDevice, s));
    auto col_norms = [&](std::vector<double>& out) -> rb_status {   // |Y e_i|^2
      RB_TRY(P.ensure((size_t)bj * bj * 16));
      ZOperand YH{Y.p, 0, 1, bj, 1};
      ZOperand Yo{Y.p, 0, bj, 1, 0};
      RB_HIP(launch_zgemm(bj, bj, T, YH, Yo, P.as<double2>(), bj, 0, bw.ws.as<double2>(),
                          (int64_t)(bw.ws.bytes / 16), s));
      std::vector<cd> g((size_t)bj * bj);
      RB_HIP(hipMemcpyAsync(g.data(), P.p, g.size() * 16, hipMemcpyDeviceToHost, s));
      RB_HIP(hipStreamSynchronize(s));
      out.resize(bj);
      for (int i = 0; i < bj; ++i) out[i] = g[(size_t)i * bj + i].real();
      return RB_OK;
    };
    std::vector<double> n0, n1;
    RB_TRY(col_norms(n0));
    for (int pass = 0; pass < 2; ++pass) {
      RB_TRY(H.ensure((size_t)Lc * bj * 16));
      ZOperand VH{V.p, 0, 1, ldb, 1};
      ZOperand Yo{Y.p, 0, bj, 1, 0};
      RB_HIP(launch_zgemm(Lc, bj, T, VH, Yo, H.as<double2>(), bj, 0, bw.ws.as<double2>(),
                          (int64_t)(bw.ws.bytes / 16), s));
      std::vector<cd> Hh((size_t)Lc * bj);
      RB_HIP(hipMemcpyAsync(Hh.data(), H.p, Hh.size() * 16, hipMemcpyDeviceToHost, s));
      RB_HIP(hipStreamSynchronize(s));
      for (auto& v : Hh) v = -v;
      RB_HIP(hipMemcpyAsync(H.p, Hh.data(), Hh.size() * 16, hipMemcpyHostToDevice, s));
      ZOperand Vo{V.p, 0, ldb, 1, 0};
      ZOperand Ho{H.p, 0, bj, 1, 0};
      RB_HIP(launch_zgemm(T, bj, Lc, Vo, Ho, Y.as<double2>(), bj, 1, bw.ws.as<double2>(),
                          (int64_t)(bw.ws.bytes / 16), s));
      RB_HIP(hipStreamSynchronize(s));   // Hh is pageable and local
    }
    // a column reduced below 1e-10 of its norm is rounding noise, not a new direction: zero it, so the
    // orthonormalisation drops it
    RB_TRY(col_norms(n1));
    for (int i = 0; i < bj; ++i)
      if (!(n1[i] > 1e-20 * n0[i]))
        RB_HIP(hipMemset2DAsync(Y.as<double2>() + i, (size_t)bj * 16, 0, 16, T, s));
    int kept = 0;
    const rb_status st = svqb(ctx, bw, Y.as<double2>(), T, bj, bw.Q.as<double2>(), &kept);
    // a block that vanishes entirely (the Krylov space is invariant) ends the iteration
    if (st != RB_OK) {
      final_pass = true;
      continue;
    }
    kept = (int)std::min<int64_t>(kept, nb_next);
    RB_HIP(hipMemcpy2DAsync(V.as<double2>() + Lc, ldb * 16, bw.Q.p, (size_t)kept * 16, (size_t)kept * 16, T,
                            hipMemcpyDeviceToDevice, s));
    c0 = Lc;
    Lc += kept;
  }
  RB_CHECK(K >= 1, RB_ERR_NUMERIC, "basis has rank zero");
  RB_CHECK(rank > 0 || K < Lc || Lc >= T, RB_ERR_NUMERIC, "Lanczos space exhausted before the rank rule was met");
  set_error("");
  return RB_OK;
}

// Stores the basis of templates [t0, t0 + T): rows v_k = conj(BS[:, k]) sc[k]
// over the band (BS: nb x K complex128 on the device), coefficients
// c = W BS diag(sc) against the bank's uniform templates, C = conj(c) packed
// for the reconstruction GEMM in `dtype`.  lambda: K values kept for export;
// energy < 0: take sum |c|^2 / trace.
rb_status finish_basis(rb_ctx ctx, rb_bank bank, int32_t t0, int64_t T, int K, const double2* BS,
                       const std::vector<double>& sc, const double* lambda, double trace, double energy,
                       rb_dtype dtype, BasisWork& bw, rb_basis* out, int32_t* rank_out, double* energy_out) {
  hipStream_t s = ctx->stream;
  const int64_t nb = bank->k_hi - bank->k_lo + 1, off = bank->k_lo - bank->kb, nbs = bank->nbs;
  const float2* W = bank->w.as<float2>() + (size_t)t0 * nbs + off;
  const ZOperand Wop{W, 1, nbs, 1, 0};
  std::unique_ptr<rb_basis_s> bs(new (std::nothrow) rb_basis_s);
  RB_CHECK(bs != nullptr, RB_ERR_OOM, "host allocation failed");
  bs->ctx = ctx;
  bs->bank = bank;
  bs->t0 = t0;
  bs->T = (int32_t)T;
  bs->K = K;
  bs->Kp = (dtype == RB_F32) ? K : ((K + 7) / 8) * 8;
  const int tile = gemm_tile_templates();
  bs->Tp = (int)(((T + tile - 1) / tile) * tile);
  bs->dtype = dtype;
  bs->trace = trace;
  bs->lambda.assign(lambda, lambda + K);
  DevBuf cdev, scale;
  RB_TRY(scale.ensure(K * 8));
  RB_HIP(hipMemcpyAsync(scale.p, sc.data(), K * 8, hipMemcpyHostToDevice, s));
  RB_TRY(bs->P.ensure((size_t)K * nbs * sizeof(float2)));
  RB_HIP(launch_basis_rows(BS, nb, K, K, scale.as<double>(), off, nbs, bs->P.as<float2>(), s));
  // c = W BS diag(theta^-1/2)  (T x K)
  RB_TRY(cdev.ensure((size_t)T * K * 16));
  {
    ZOperand BSo{BS, 0, K, 1, 0};
    RB_HIP(launch_zgemm(T, K, nb, Wop, BSo, cdev.as<double2>(), K, 0, bw.ws.as<double2>(),
                        (int64_t)(bw.ws.bytes / 16), s));
  }
  bs->c.resize((size_t)T * K);
  RB_HIP(hipMemcpyAsync(bs->c.data(), cdev.p, bs->c.size() * 16, hipMemcpyDeviceToHost, s));
  RB_HIP(hipStreamSynchronize(s));
  double csum = 0.0, cmin = 1.0;
  for (int64_t j = 0; j < T; ++j) {
    double cj = 0.0;
    for (int k = 0; k < K; ++k) {
      bs->c[(size_t)j * K + k] *= sc[k];
      cj += std::norm(bs->c[(size_t)j * K + k]);
    }
    csum += cj;
    cmin = std::min(cmin, cj);
  }
  bs->energy = energy >= 0 ? energy : csum / trace;
  bs->min_energy = std::min(1.0, cmin);
  // C = conj(c) as complex64 (unscaled), row scales for FP16
  std::vector<float2> C32((size_t)T * K);
  bs->row_scale.assign(bs->Tp, 1.f);
  for (int64_t j = 0; j < T; ++j) {
    double mx = 0.0;
    for (int k = 0; k < K; ++k) {
      const cd v = std::conj(bs->c[(size_t)j * K + k]);
      C32[(size_t)j * K + k] = make_float2((float)v.real(), (float)v.imag());
      mx = std::max(mx, std::max(std::fabs(v.real()), std::fabs(v.imag())));
    }
    if (dtype == RB_F16 && mx > 0) {
      int ex;
      (void)std::frexp(mx, &ex);      // mx = m 2^ex, m in [0.5, 1)
      bs->row_scale[j] = (float)std::ldexp(1.0, -ex);
    }
  }
  std::vector<float> rinv(bs->Tp);
  for (int j = 0; j < bs->Tp; ++j) rinv[j] = 1.f / bs->row_scale[j];
  RB_TRY(bs->C32.ensure(C32.size() * sizeof(float2)));
  RB_HIP(hipMemcpyAsync(bs->C32.p, C32.data(), C32.size() * sizeof(float2), hipMemcpyHostToDevice, s));
  RB_TRY(bs->row_inv.ensure((size_t)bs->Tp * 4));
  RB_TRY(bs->row_scale_dev.ensure((size_t)bs->Tp * 4));
  RB_HIP(hipMemcpyAsync(bs->row_inv.p, rinv.data(), (size_t)bs->Tp * 4, hipMemcpyHostToDevice, s));
  RB_HIP(hipMemcpyAsync(bs->row_scale_dev.p, bs->row_scale.data(), (size_t)bs->Tp * 4, hipMemcpyHostToDevice, s));
  const size_t cpk_bytes = (dtype == RB_F32) ? (size_t)(bs->Tp / 32) * ((K + 1) / 2) * 64 * 4 * 4
                                             : (size_t)(bs->Tp / 16) * (bs->Kp / 8) * 64 * 8 * 2 *
                                                   (dtype == RB_BF16X3 ? 2 : 1);
  RB_TRY(bs->cpk.ensure(cpk_bytes));
  RB_HIP(launch_pack_c(bs->C32.as<float2>(), (int)T, bs->Tp, K, bs->Kp, (int)dtype,
                       dtype == RB_F16 ? bs->row_scale_dev.as<float>() : nullptr, bs->cpk.p, s));
  if (dtype == RB_F32) {
    RB_TRY(bs->cpk3.ensure((size_t)(bs->Tp / 32) * ((K + 1) / 2) * 64 * 16));
    RB_HIP(launch_pack_c3(bs->C32.as<float2>(), (int)T, bs->Tp, K, bs->cpk3.p, s));
  } else {
    RB_TRY(bs->cpkc.ensure((size_t)(bs->Tp / 32) * (bs->Kp / 8) * 64 * 8 * 2 * (dtype == RB_BF16X3 ? 2 : 1)));
    RB_HIP(launch_pack_c16c(bs->C32.as<float2>(), (int)T, bs->Tp, K, bs->Kp, (int)dtype,
                            dtype == RB_F16 ? bs->row_scale_dev.as<float>() : nullptr, bs->cpkc.p, s));
  }
  RB_HIP(hipStreamSynchronize(s));
  if (rank_out) *rank_out = K;
  if (energy_out) *energy_out = bs->energy;
  bank->live_bases++;
  ctx->live++;
  *out = bs.release();
  return RB_OK;
}

}  // namespace

extern "C" rb_status rb_build_basis_range(rb_ctx ctx, rb_bank bank, int32_t t0, int32_t t1, int32_t rank,
                                          double tol, rb_dtype dtype, rb_basis* out, int32_t* rank_out,
                                          double* energy_out) {
  return rb_build_basis_solver(ctx, bank, t0, t1, rank, tol, dtype, RB_EIG_SUBSPACE, out, rank_out, energy_out);
}

extern "C" rb_status rb_build_basis_solver(rb_ctx ctx, rb_bank bank, int32_t t0, int32_t t1, int32_t rank,
                                           double tol, rb_dtype dtype, int32_t solver, rb_basis* out,
                                           int32_t* rank_out, double* energy_out) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(solver == RB_EIG_SUBSPACE || solver == RB_EIG_LANCZOS, RB_ERR_ARG, "bad eigensolver");
  RB_CHECK(bank != nullptr && out != nullptr, RB_ERR_ARG, "NULL argument");
  RB_CHECK(bank->ctx == ctx, RB_ERR_ARG, "bank belongs to another context");
  RB_CHECK(t0 >= 0 && t0 < t1 && t1 <= bank->T, RB_ERR_ARG, "template range must satisfy 0 <= t0 < t1 <= T");
  RB_CHECK(rank >= 0, RB_ERR_ARG, "rank must be >= 0");
  RB_CHECK(rank > 0 || (tol > 0 && tol < 1), RB_ERR_ARG, "tol must be in (0, 1) when rank == 0");
  RB_CHECK(dtype == RB_F32 || dtype == RB_BF16 || dtype == RB_F16 || dtype == RB_BF16X3, RB_ERR_ARG,
           "bad dtype");
  *out = nullptr;
  const int64_t T = t1 - t0;
  const int64_t nb = bank->k_hi - bank->k_lo + 1, off = bank->k_lo - bank->kb, nbs = bank->nbs;
  hipStream_t s = ctx->stream;
  BasisWork bw;
  RB_TRY(bw.ws.ensure((size_t)64 << 20 << 4));   // 64 Mi complex128 split-K partials (1 GiB)
  // trace of the Gram = sum of stored squared norms
  RB_TRY(bw.norms.ensure((size_t)T * 8));
  const float2* W = bank->w.as<float2>() + (size_t)t0 * nbs + off;
  RB_HIP(launch_row_norms(W, T, nb, nbs, bw.norms.as<double>(), s));
  std::vector<double> norms(T);
  RB_HIP(hipMemcpyAsync(norms.data(), bw.norms.p, T * 8, hipMemcpyDeviceToHost, s));
  RB_HIP(hipStreamSynchronize(s));
  double trace = 0.0;
  for (double v : norms) trace += v;
  std::vector<double> theta;
  std::vector<cd> S;
  int Lc = 0, K = 0;
  int64_t ldb = 0;
  if (solver == RB_EIG_LANCZOS)
    RB_TRY(lanczos_pca(ctx, bw, W, T, nb, nbs, trace, rank, tol, theta, S, Lc, K, ldb));
  else
    RB_TRY(subspace_pca(ctx, bw, W, T, nb, nbs, trace, rank, tol, theta, S, Lc, K));
  DevBuf BS;
  RB_TRY(ritz_vectors(ctx, bw, nb, Lc, K, S, BS, ldb));
  std::vector<double> sc(K);
  double e = 0.0;
  for (int k = 0; k < K; ++k) {
    sc[k] = 1.0 / std::sqrt(theta[k]);
    e += theta[k];
  }
  return finish_basis(ctx, bank, t0, T, K, BS.as<double2>(), sc, theta.data(), trace, e / trace, dtype, bw, out,
                      rank_out, energy_out);
}

extern "C" rb_status rb_build_basis_nonuniform(rb_ctx ctx, rb_bank bank, int32_t t0, int32_t t1,
                                               const double* nodes, int64_t nt, const double* psd_nodes,
                                               rb_fill_at_fn fill, void* user, int32_t rank, double tol,
                                               rb_dtype dtype, rb_basis* out, int32_t* rank_out,
                                               double* energy_out) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(bank != nullptr && out != nullptr && nodes != nullptr && psd_nodes != nullptr && fill != nullptr,
           RB_ERR_ARG, "NULL argument");
  RB_CHECK(bank->ctx == ctx, RB_ERR_ARG, "bank belongs to another context");
  RB_CHECK(t0 >= 0 && t0 < t1 && t1 <= bank->T, RB_ERR_ARG, "template range must satisfy 0 <= t0 < t1 <= T");
  RB_CHECK(rank >= 0, RB_ERR_ARG, "rank must be >= 0");
  RB_CHECK(rank > 0 || (tol > 0 && tol < 1), RB_ERR_ARG, "tol must be in (0, 1) when rank == 0");
  RB_CHECK(dtype == RB_F32 || dtype == RB_BF16 || dtype == RB_F16 || dtype == RB_BF16X3, RB_ERR_ARG,
           "bad dtype");
  RB_CHECK(nt >= 2 && nt <= (int64_t(1) << 26), RB_ERR_ARG, "nt must be in [2, 2^26]");
  *out = nullptr;
  const double df = bank->grid.fs / (double)bank->grid.N;
  for (int64_t i = 0; i < nt; ++i) {
    RB_CHECK(std::isfinite(nodes[i]) && (i == 0 || nodes[i] > nodes[i - 1]), RB_ERR_ARG,
             "nodes must be finite and strictly increasing");
    RB_CHECK(std::isfinite(psd_nodes[i]) && psd_nodes[i] > 0, RB_ERR_ARG,
             "PSD at the nodes must be finite and positive");
  }
  RB_CHECK(nodes[0] <= (double)bank->k_lo * df && nodes[nt - 1] >= (double)bank->k_hi * df, RB_ERR_ARG,
           "nodes must cover the band [k_lo df, k_hi df]");
  const int64_t T = t1 - t0;
  const int64_t nb = bank->k_hi - bank->k_lo + 1, off = bank->k_lo - bank->kb, nbs = bank->nbs;
  hipStream_t s = ctx->stream;
  // whitened unit templates on the set, V[j][i] = h_j(f_i) g_i / sigma_j with
  // g_i = sqrt(4 omega_i / Sn_i), FP64 on the host, complex64 on the device
  std::vector<double> om, g(nt);
  cell_weights(nodes, nt, om);
  for (int64_t i = 0; i < nt; ++i) g[i] = std::sqrt(4.0 * om[i] / psd_nodes[i]);
  DevBuf V;
  RB_TRY(V.ensure((size_t)T * nt * sizeof(float2)));
  const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(T, (int64_t(64) << 20) / (nt * 16)));
  std::vector<double> hbuf((size_t)chunk * nt * 2);
  HostPinned stage;
  RB_TRY(stage.ensure((size_t)chunk * nt * sizeof(float2)));
  for (int64_t c0 = 0; c0 < T; c0 += chunk) {
    const int64_t c1 = std::min<int64_t>(T, c0 + chunk);
    RB_HIP(hipStreamSynchronize(s));   // staging buffer reuse
    const int rc = fill(user, (int32_t)(t0 + c0), (int32_t)(t0 + c1), nodes, nt, hbuf.data());
    RB_CHECK(rc == 0, RB_ERR_CALLBACK, "template fill callback returned " + std::to_string(rc));
    float2* st = static_cast<float2*>(stage.p);
    std::atomic<int> nbad(0);
    parallel_for(c1 - c0, [&](int64_t r) {
      const double* h = &hbuf[(size_t)r * nt * 2];
      double s2 = 0.0;
      for (int64_t i = 0; i < nt; ++i) {
        const double re = h[2 * i] * g[i], im = h[2 * i + 1] * g[i];
        s2 += re * re + im * im;
      }
      const double sg = std::sqrt(s2);
      if (!(sg > 0.0) || !std::isfinite(sg)) {
        nbad++;
        return;
      }
      float2* o = st + (size_t)r * nt;
      for (int64_t i = 0; i < nt; ++i) {
        const double fct = g[i] / sg;
        o[i] = make_float2((float)(h[2 * i] * fct), (float)(h[2 * i + 1] * fct));
      }
    });
    RB_CHECK(nbad.load() == 0, RB_ERR_ARG, "a template has zero or non-finite norm on the nodes");
    RB_HIP(hipMemcpyAsync(V.as<float2>() + (size_t)c0 * nt, st, (size_t)(c1 - c0) * nt * sizeof(float2),
                          hipMemcpyHostToDevice, s));
  }
  BasisWork bw;
  RB_TRY(bw.ws.ensure((size_t)64 << 20 << 4));
  RB_TRY(bw.norms.ensure((size_t)T * 8));
  std::vector<double> norms(T);
  RB_HIP(launch_row_norms(V.as<float2>(), T, nt, nt, bw.norms.as<double>(), s));
  RB_HIP(hipMemcpyAsync(norms.data(), bw.norms.p, T * 8, hipMemcpyDeviceToHost, s));
  RB_HIP(hipStreamSynchronize(s));
  double trace_set = 0.0;
  for (double v : norms) trace_set += v;
  std::vector<double> theta;
  std::vector<cd> S;
  int Lc = 0, K = 0;
  RB_TRY(subspace_pca(ctx, bw, V.as<float2>(), T, nt, nt, trace_set, rank, tol, theta, S, Lc, K));
  DevBuf BSn;
  RB_TRY(ritz_vectors(ctx, bw, nt, Lc, K, S, BSn));
  // interpolation onto the band: r_i = 1/sqrt(omega_i), per-vector scale
  // sqrt(df) theta_k^{-1/2} (unit vectors on the set -> densities -> grid)
  std::vector<int32_t> idx;
  std::vector<double> frac, r(nt), scv(K);
  interp_table(nodes, nt, bank->k_lo, bank->k_hi, df, idx, frac);
  for (int64_t i = 0; i < nt; ++i) r[i] = 1.0 / std::sqrt(om[i]);
  for (int k = 0; k < K; ++k) scv[k] = std::sqrt(df) / std::sqrt(theta[k]);
  DevBuf idx_d, frac_d, r_d, sc_d, BSu, BSo;
  RB_TRY(idx_d.ensure((size_t)nb * 4));
  RB_TRY(frac_d.ensure((size_t)nb * 8));
  RB_TRY(r_d.ensure((size_t)nt * 8));
  RB_TRY(sc_d.ensure((size_t)K * 8));
  RB_HIP(hipMemcpyAsync(idx_d.p, idx.data(), (size_t)nb * 4, hipMemcpyHostToDevice, s));
  RB_HIP(hipMemcpyAsync(frac_d.p, frac.data(), (size_t)nb * 8, hipMemcpyHostToDevice, s));
  RB_HIP(hipMemcpyAsync(r_d.p, r.data(), (size_t)nt * 8, hipMemcpyHostToDevice, s));
  RB_HIP(hipMemcpyAsync(sc_d.p, scv.data(), (size_t)K * 8, hipMemcpyHostToDevice, s));
  RB_TRY(BSu.ensure((size_t)nb * K * 16));
  RB_HIP(launch_interp_rows(BSn.as<double2>(), nt, K, idx_d.as<int32_t>(), frac_d.as<double>(), r_d.as<double>(),
                            sc_d.as<double>(), nb, BSu.as<double2>(), s));
  // orthonormal on the uniform grid (two SVQB passes over the nb x K columns)
  RB_TRY(BSo.ensure((size_t)nb * K * 16));
  RB_TRY(bw.Y.ensure((size_t)nb * K * 16));
  int K2 = 0;
  RB_TRY(svqb(ctx, bw, BSu.as<double2>(), nb, K, BSo.as<double2>(), &K2));
  RB_HIP(hipStreamSynchronize(s));   // host tables are local
  // trace of the uniform templates for the kept energy
  RB_TRY(bw.norms.ensure((size_t)T * 8));
  const float2* Wu = bank->w.as<float2>() + (size_t)t0 * nbs + off;
  RB_HIP(launch_row_norms(Wu, T, nb, nbs, bw.norms.as<double>(), s));
  RB_HIP(hipMemcpyAsync(norms.data(), bw.norms.p, T * 8, hipMemcpyDeviceToHost, s));
  RB_HIP(hipStreamSynchronize(s));
  double trace = 0.0;
  for (double v : norms) trace += v;
  std::vector<double> ones(K2, 1.0);
  return finish_basis(ctx, bank, t0, T, K2, BSo.as<double2>(), ones, theta.data(), trace, -1.0, dtype, bw, out,
                      rank_out, energy_out);
}

extern "C" rb_status rb_basis_free(rb_basis basis) {
  RB_CHECK(basis != nullptr, RB_ERR_ARG, "basis is NULL");
  (void)hipSetDevice(basis->ctx->device);
  (void)hipStreamSynchronize(basis->ctx->stream);
  basis->bank->live_bases--;
  basis->ctx->live--;
  delete basis;
  return RB_OK;
}

extern "C" rb_status rb_basis_export(rb_basis basis, double* V, double* c, double* lambda) {
  RB_CHECK(basis != nullptr, RB_ERR_ARG, "basis is NULL");
  RB_HIP(hipSetDevice(basis->ctx->device));
  rb_bank bank = basis->bank;
  const int K = basis->K;
  const int64_t nb = bank->k_hi - bank->k_lo + 1, off = bank->k_lo - bank->kb;
  if (V) {
    std::vector<float2> P((size_t)K * bank->nbs);
    RB_HIP(hipMemcpy(P.data(), basis->P.p, P.size() * sizeof(float2), hipMemcpyDeviceToHost));
    for (int k = 0; k < K; ++k)
      for (int64_t f = 0; f < nb; ++f) {
        const float2 v = P[(size_t)k * bank->nbs + off + f];
        V[2 * ((size_t)k * nb + f)] = v.x;
        V[2 * ((size_t)k * nb + f) + 1] = v.y;
      }
  }
  if (c) std::memcpy(c, basis->c.data(), basis->c.size() * 16);
  if (lambda) std::memcpy(lambda, basis->lambda.data(), basis->lambda.size() * 8);
  return RB_OK;
}

// ====================================================================== search
namespace {

// rho = C Z on the basis outputs (w = 1: every sample, crossings into trig1 /
// cnt1) or on their bin means (w >= 2: N/w columns, triggering bins into
// trigB / cntB with the bin index as the sample).
rb_status stage1_gemm(rb_ctx ctx, rb_basis basis, const FftGeom& g, float thr1sq, float2* rho_out, int w = 1) {
  const float want = rho_out ? std::numeric_limits<float>::infinity() : thr1sq;
  if (!(basis->thr_cached == want)) {
    RB_TRY(basis->thr_row.ensure((size_t)basis->Tp * 4));
    std::vector<float> thr(basis->Tp);
    for (int j = 0; j < basis->Tp; ++j) {
      const float a = basis->row_scale[j];
      thr[j] = want * a * a;
    }
    RB_HIP(hipMemcpyAsync(basis->thr_row.p, thr.data(), thr.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    RB_HIP(hipStreamSynchronize(ctx->stream));
    basis->thr_cached = want;
  }
  GemmArgs ga;
  std::memset(&ga, 0, sizeof(ga));
  ga.N = g.N / w;
  ga.T = basis->T;
  ga.Tp = basis->Tp;
  ga.K = basis->K;
  ga.Kp = basis->Kp;
  ga.dtype = (int)basis->dtype;
  ga.cpk = basis->cpk.p;
  ga.cpk3 = basis->cpk3.p;
  ga.cpkc = basis->cpkc.p;
  ga.z = ctx->z.p;
  ga.thr2_row = basis->thr_row.as<float>();
  ga.N1 = g.N1;
  ga.N2 = g.N2 / w;
  DevBuf& tb = w > 1 ? ctx->trigB : ctx->trig1;
  ga.trig = tb.as<TrigRec>();
  ga.trig_cap = trig_capacity(tb);
  ga.trig_count = ctx->counters.as<unsigned long long>() + (w > 1 ? 2 : 0);
  ga.tmpl_base = basis->t0;
  ga.tmpl_count = (w > 1 ? ctx->cntB : ctx->cnt1).as<int32_t>() + basis->t0;
  ga.rho_out = rho_out;
  ga.row_inv = basis->row_inv.as<float>();
  if (basis->gemm_variant.find(ga.N) == basis->gemm_variant.end()) {
    // autotune on this basis's first call: time every variant on the real Z
    // with infinite thresholds (no trigger is appended), keep the fastest
    const char* force = std::getenv("RBMF_GEMM_VARIANT");
    const char* at = std::getenv("RBMF_AUTOTUNE");
    const std::string key = ctx->arch + "/gemm3/dt=" + std::to_string(ga.dtype) + "/K=" + std::to_string(ga.K) +
                            "/T=" + std::to_string(ga.T) + "/N=" + std::to_string(ga.N);
    int choice = 0, cached = -1;
    if (force) {
      choice = std::max(0, std::min(recon_variants(ga.dtype) - 1, std::atoi(force)));
    } else if (tune_cache().get(key, &cached) && cached >= 0 && cached < recon_variants(ga.dtype)) {
      choice = cached;
    } else if (!(at && std::strcmp(at, "0") == 0)) {
      RB_TRY(ctx->thr_inf.ensure((size_t)basis->Tp * 4));
      RB_TRY(fill32(ctx, ctx->thr_inf.p, 0x7f800000u, basis->Tp));
      GemmArgs gt = ga;
      gt.thr2_row = ctx->thr_inf.as<float>();
      gt.rho_out = nullptr;
      hipEvent_t e0, e1;
      RB_HIP(hipEventCreate(&e0));
      RB_HIP(hipEventCreate(&e1));
      float best = 1e30f;
      for (int v = 0; v < recon_variants(ga.dtype); ++v) {
        gt.variant = v;
        float ms_min = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
          RB_HIP(hipEventRecord(e0, ctx->stream));
          RB_HIP(launch_recon_gemm(gt, ctx->stream));
          RB_HIP(hipEventRecord(e1, ctx->stream));
          RB_HIP(hipEventSynchronize(e1));
          float ms = 0.f;
          RB_HIP(hipEventElapsedTime(&ms, e0, e1));
          if (rep > 0) ms_min = std::min(ms_min, ms);
        }
        if (std::getenv("RBMF_VERBOSE"))
          std::fprintf(stderr, "[rbmf] GEMM dtype %d K=%d T=%d variant %d: %.4f ms\n", ga.dtype, ga.K, ga.T, v,
                       ms_min);
        if (ms_min < best) {
          best = ms_min;
          choice = v;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      tune_cache().put(key, choice);
    }
    basis->gemm_variant[ga.N] = choice;
  }
  ga.variant = basis->gemm_variant[ga.N];
  RB_HIP(launch_recon_gemm(ga, ctx->stream));
  ctx->mfma_flop += recon_mfma_flop(ga);
  return RB_OK;
}

rb_status event(rb_ctx ctx, size_t i) {
  while (ctx->evs.size() <= i) {
    hipEvent_t e;
    RB_HIP(hipEventCreate(&e));
    ctx->evs.push_back(e);
  }
  RB_HIP(hipEventRecord(ctx->evs[i], ctx->stream));
  return RB_OK;
}

float elapsed(rb_ctx ctx, size_t a, size_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, ctx->evs[a], ctx->evs[b]) != hipSuccess) {
    (void)hipGetLastError();
    return 0.f;
  }
  return ms;
}

// The bases must belong to `bank` and their ranges must partition [0, T).
rb_status check_partition(rb_ctx ctx, const rb_basis* bases, int32_t nb, rb_bank bank) {
  RB_CHECK(bases != nullptr && nb >= 1, RB_ERR_ARG, "need at least one basis");
  std::vector<std::pair<int32_t, int32_t>> r;
  for (int32_t i = 0; i < nb; ++i) {
    RB_CHECK(bases[i] != nullptr, RB_ERR_ARG, "basis is NULL");
    RB_CHECK(bases[i]->bank == bank && bases[i]->ctx == ctx, RB_ERR_ARG, "basis/bank/context mismatch");
    r.push_back({bases[i]->t0, bases[i]->t0 + bases[i]->T});
  }
  std::sort(r.begin(), r.end());
  int32_t at = 0;
  for (auto& x : r) {
    RB_CHECK(x.first == at, RB_ERR_ARG, "basis template ranges must partition [0, T)");
    at = x.second;
  }
  RB_CHECK(at == bank->T, RB_ERR_ARG, "basis template ranges must partition [0, T)");
  return RB_OK;
}

// Arguments of the sparse exact second stage over the stage-1 records grouped
// by template (list1 / off1 / cnt1 / recs1).  d_count and n1_dev are the
// device-side list length and stage-1 total of a captured search (NULL when
// the host knows them).
SparseArgs sparse_args(rb_ctx ctx, rb_bank bank, const FftGeom& g, const FftTables& tw, double thr2,
                       const int32_t* d_count, const int64_t* n1_dev, int64_t n1_cap) {
  SparseArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.N = g.N;
  sa.s_lo = g.s_lo;
  sa.tlo = tw.tlo;
  sa.thi = tw.thi;
  sa.list = ctx->list1.as<int32_t>();
  sa.d_count = d_count;
  sa.n1_dev = n1_dev;
  sa.n1_cap = n1_cap;
  sa.offsets = ctx->off1.as<int32_t>();
  sa.counts = ctx->cnt1.as<int32_t>();
  sa.recs = ctx->recs1.as<TrigRec>();
  sa.d = ctx->dspec.as<float2>();
  sa.tmpl = bank->w.as<float2>();
  sa.kb = bank->kb;
  sa.nbs = bank->nbs;
  sa.sup_lo = bank->sup_lo.as<int32_t>();
  sa.sup_hi = bank->sup_hi.as<int32_t>();
  sa.thr2 = (float)(thr2 * thr2);
  sa.out = ctx->trig2.as<TrigRec>();
  sa.out_cap = trig_capacity(ctx->trig2);
  sa.out_count = ctx->counters.as<unsigned long long>() + 1;
  sa.tmpl_count = ctx->cnt2.as<int32_t>();
  sa.tmpl_max = ctx->want_peaks ? ctx->tmax.as<unsigned long long>() : nullptr;
  return sa;
}

}  // namespace

extern "C" rb_status rb_filter(rb_ctx ctx, const rb_basis* bases, int32_t nbases, rb_bank bank,
                               const float* strain, const rb_filter_opts* opts, rb_trigger* out, int64_t cap,
                               int64_t* n_out, rb_peak* peaks, rb_stats* stats) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(bank != nullptr && opts != nullptr && n_out != nullptr, RB_ERR_ARG, "NULL argument");
  RB_CHECK(bank->ctx == ctx, RB_ERR_ARG, "bank belongs to another context");
  RB_TRY(check_partition(ctx, bases, nbases, bank));
  RB_CHECK(std::isfinite(opts->thr1) && opts->thr1 > 0, RB_ERR_ARG, "thr1 must be > 0");
  RB_CHECK(std::isfinite(opts->thr2) && opts->thr2 >= opts->thr1, RB_ERR_ARG, "thr2 must be >= thr1");
  RB_CHECK(opts->stage2 == RB_STAGE2_FULL || opts->stage2 == RB_STAGE2_SPARSE || opts->stage2 == RB_STAGE2_AUTO ||
               opts->stage2 == RB_STAGE2_RECON,
           RB_ERR_ARG, "bad stage2 mode");
  const int w = opts->bin_w >= 2 ? opts->bin_w : 1;
  RB_CHECK(opts->bin_w >= 0 && opts->bin_w <= 64 && (w & (w - 1)) == 0 && bank->grid.N / w >= 256, RB_ERR_ARG,
           "bin_w must be 0, 1 or a power of two <= 64 with N / bin_w >= 256");
  RB_CHECK(w == 1 || (std::isfinite(opts->thr_bin) && opts->thr_bin > 0), RB_ERR_ARG, "thr_bin must be > 0");
  RB_CHECK(opts->bin_source == 0 || (opts->bin_source == 1 && w > 1), RB_ERR_ARG,
           "bin_source must be 0, or 1 with bin_w >= 2");
  RB_CHECK((opts->flags & ~RB_OPT_FP16_INTERMEDIATE) == 0, RB_ERR_ARG, "unknown opts flag");
  const bool fold = opts->bin_source == 1;
  FftGeom gM{};
  if (fold) {
    gM = make_geom(bank->grid.N / w);
    RB_CHECK(geom_supported(gM), RB_ERR_ARG, "bin_source 1 needs N / bin_w >= 4096");
  }
  RB_CHECK(cap >= 0, RB_ERR_ARG, "cap must be >= 0");
  const int T = bank->T;
  ctx->want_peaks = peaks != nullptr;
  FftGeom g;
  RB_TRY(geom_for(ctx, bank, &g));
  FftTables tw;
  RB_TRY(get_tables(ctx, g, tw));
  const float* s;
  RB_TRY(strain_device(ctx, strain, g.N, &s));
  RB_TRY(ensure_trigger_scratch(ctx, T));
  const bool tm = stats != nullptr;
  // events: 0 start, 1 spectrum, 2+2m Z of basis m, 3+2m GEMM (+ fine) of basis m, then scan,
  // stage 2, end; with bins, e_end + 1 + m between the GEMM and the fine step of basis m
  const size_t e_scan = 2 + 2 * (size_t)nbases, e_s2 = e_scan + 1, e_end = e_s2 + 1;
  if (tm) RB_TRY(event(ctx, 0));
  RB_TRY(fill32(ctx, ctx->flag.p, 0u, 2));
  RB_HIP(launch_check_finite(s, g.N, ctx->flag.as<int64_t>(), ctx->stream));
  RB_TRY(step_spectrum(ctx, bank, g, tw, s));
  if (tm) RB_TRY(event(ctx, 1));
  int64_t sum1[3];
  int64_t nbins = 0;
  const float thr1sq = (float)(opts->thr1 * opts->thr1);
  const FftGeom gb = w > 1 ? binned_geom(g, w) : g;   // the twiddle tables depend on N only
  if (w > 1) RB_TRY(ctx->snap.ensure((size_t)nbases * 8));
  std::vector<int32_t> offB, cntB;   // template fold: bins grouped by template
  if (fold) {
    if (tm) RB_TRY(event(ctx, e_end + 1 + (size_t)nbases));
    for (;;) {
      RB_TRY(fill32(ctx, ctx->counters.as<unsigned long long>() + 2, 0u, 2));
      RB_TRY(fill32(ctx, ctx->cntB.p, 0u, T));
      RB_TRY(step_fold(ctx, bank, gM, w, (float)(opts->thr_bin * opts->thr_bin)));
      RB_HIP(hipMemcpyAsync(&nbins, ctx->counters.as<unsigned long long>() + 2, 8, hipMemcpyDeviceToHost,
                            ctx->stream));
      RB_HIP(hipStreamSynchronize(ctx->stream));
      if (nbins <= trig_capacity(ctx->trigB)) break;
      RB_TRY(ctx->trigB.ensure((size_t)(nbins + nbins / 4) * sizeof(TrigRec)));
    }
    RB_TRY(ctx->offB.ensure((size_t)T * 4));
    RB_TRY(ctx->fillB.ensure((size_t)T * 4));
    RB_TRY(ctx->listB.ensure((size_t)T * 4));
    RB_TRY(ctx->recsB.ensure(std::max<size_t>(16, (size_t)nbins * sizeof(TrigRec))));
    int64_t sumB[3];
    RB_TRY(scan_and_read(ctx, T, ctx->cntB, ctx->offB, ctx->fillB, ctx->listB, sumB));
    RB_HIP(launch_scatter_triggers(ctx->trigB.as<TrigRec>(), nbins, nullptr, ctx->offB.as<int32_t>(),
                                   ctx->fillB.as<int32_t>(), ctx->recsB.as<TrigRec>(), ctx->stream));
    offB.resize(T);
    cntB.resize(T);
    RB_HIP(hipMemcpyAsync(offB.data(), ctx->offB.p, (size_t)T * 4, hipMemcpyDeviceToHost, ctx->stream));
    RB_HIP(hipMemcpyAsync(cntB.data(), ctx->cntB.p, (size_t)T * 4, hipMemcpyDeviceToHost, ctx->stream));
    RB_HIP(hipStreamSynchronize(ctx->stream));
    if (tm) RB_TRY(event(ctx, e_end + 2 + (size_t)nbases));
  }
  for (;;) {
    ctx->mfma_flop = 0;   // (the GEMMs of the last attempt, the one the stage times cover)
    RB_TRY(fill32(ctx, ctx->counters.p, 0u, 2));
    RB_TRY(fill32(ctx, ctx->cnt1.p, 0u, T));
    if (w > 1 && !fold) {
      RB_TRY(fill32(ctx, ctx->counters.as<unsigned long long>() + 2, 0u, 2));
      RB_TRY(fill32(ctx, ctx->cntB.p, 0u, T));
    }
    const bool h16 = (opts->flags & RB_OPT_FP16_INTERMEDIATE) != 0;
    for (int32_t m = 0; m < nbases; ++m) {
      if (w == 1) {
        RB_TRY(step_basis_outputs(ctx, bases[m], g, tw, false, h16));
        if (tm) RB_TRY(event(ctx, 2 + 2 * (size_t)m));
        RB_TRY(stage1_gemm(ctx, bases[m], g, thr1sq, nullptr));
      } else if (fold) {   // the basis serves the fine stage only
        RB_TRY(step_basis_outputs_binned(ctx, bases[m], gb, tw, w, h16));
        if (tm) RB_TRY(event(ctx, 2 + 2 * (size_t)m));
        if (tm) RB_TRY(event(ctx, e_end + 1 + (size_t)m));
        const int t0 = bases[m]->t0, t1 = t0 + bases[m]->T;
        RB_TRY(step_fine(ctx, bases[m], gb, w, thr1sq, nullptr, ctx->recsB.as<TrigRec>(), offB[t0],
                         (int64_t)offB[t1 - 1] + cntB[t1 - 1]));
      } else {
        RB_TRY(step_basis_outputs_binned(ctx, bases[m], gb, tw, w, h16));
        if (tm) RB_TRY(event(ctx, 2 + 2 * (size_t)m));
        unsigned long long* snap = ctx->snap.as<unsigned long long>() + m;
        RB_HIP(launch_copy_u64(ctx->counters.as<unsigned long long>() + 2, snap, ctx->stream));
        RB_TRY(stage1_gemm(ctx, bases[m], gb, (float)(opts->thr_bin * opts->thr_bin), nullptr, w));
        if (tm) RB_TRY(event(ctx, e_end + 1 + (size_t)m));
        RB_TRY(step_fine(ctx, bases[m], gb, w, thr1sq, snap));
      }
      if (tm) RB_TRY(event(ctx, 3 + 2 * (size_t)m));
    }
    if (w > 1 && !fold)
      RB_HIP(hipMemcpyAsync(&nbins, ctx->counters.as<unsigned long long>() + 2, 8, hipMemcpyDeviceToHost,
                            ctx->stream));
    RB_TRY(scan_and_read(ctx, T, ctx->cnt1, ctx->off1, ctx->fill1, ctx->list1, sum1));
    if (nbins > trig_capacity(ctx->trigB)) {
      RB_TRY(ctx->trigB.ensure((size_t)(nbins + nbins / 4) * sizeof(TrigRec)));
      continue;
    }
    if (sum1[0] <= trig_capacity(ctx->trig1)) break;
    RB_TRY(ctx->trig1.ensure((size_t)(sum1[0] + sum1[0] / 4) * sizeof(TrigRec)));
  }
  if (tm) RB_TRY(event(ctx, e_scan));
  int64_t flag = 0;
  RB_HIP(hipMemcpyAsync(&flag, ctx->flag.p, 8, hipMemcpyDeviceToHost, ctx->stream));
  RB_HIP(hipStreamSynchronize(ctx->stream));
  RB_CHECK(flag == 0, RB_ERR_NUMERIC, "strain contains non-finite values");
  int64_t sum2[3];
  const bool recon = opts->stage2 == RB_STAGE2_RECON;
  const bool autom = opts->stage2 == RB_STAGE2_AUTO;
  const bool sparse = opts->stage2 == RB_STAGE2_SPARSE || autom;
  // RECON without bins reads the GEMM's records, which carry the 16-bit row
  // scales: gather every basis's inverse scales by global template
  const float* inv_scale = nullptr;
  if (recon && w == 1) {
    bool scaled = false;
    for (int32_t m = 0; m < nbases; ++m) scaled |= bases[m]->dtype != RB_F32;
    if (scaled) {
      RB_TRY(ctx->tinv.ensure((size_t)T * 4));
      for (int32_t m = 0; m < nbases; ++m)
        RB_HIP(hipMemcpyAsync(ctx->tinv.as<float>() + bases[m]->t0, bases[m]->row_inv.p, (size_t)bases[m]->T * 4,
                              hipMemcpyDeviceToDevice, ctx->stream));
      inv_scale = ctx->tinv.as<float>();
    }
  }
  if (sparse) {   // stage-1 records grouped by template (off1 / fill1 from the scan)
    RB_TRY(ctx->recs1.ensure(std::max<size_t>(16, (size_t)sum1[0] * sizeof(TrigRec))));
    RB_HIP(launch_scatter_triggers(ctx->trig1.as<TrigRec>(), sum1[0], nullptr, ctx->off1.as<int32_t>(),
                                   ctx->fill1.as<int32_t>(), ctx->recs1.as<TrigRec>(), ctx->stream));
  }
  // AUTO: templates with many crossings take the full matched filter (two FFT
  // passes), the rest the direct sums; nsplit = {heavy, light} list lengths
  int32_t nsplit[2] = {0, (int32_t)sum1[1]};
  const int split = stage2_split();
  if (autom) {
    RB_TRY(ctx->listH.ensure((size_t)T * 4));
    RB_TRY(ctx->listL.ensure((size_t)T * 4));
    RB_TRY(ctx->nsplit.ensure(16));
    RB_TRY(fill32(ctx, ctx->nsplit.p, 0u, 2));
    RB_HIP(launch_split_list(ctx->list1.as<int32_t>(), sum1[1], ctx->cnt1.as<int32_t>(), split,
                             ctx->listH.as<int32_t>(), ctx->listL.as<int32_t>(), ctx->nsplit.as<int32_t>(),
                             ctx->stream));
    RB_HIP(hipMemcpyAsync(nsplit, ctx->nsplit.p, 8, hipMemcpyDeviceToHost, ctx->stream));
    RB_HIP(hipStreamSynchronize(ctx->stream));
  }
  for (;;) {
    RB_TRY(fill32(ctx, ctx->counters.as<unsigned long long>() + 1, 0u, 2));
    RB_TRY(fill32(ctx, ctx->cnt2.p, 0u, T));
    RB_TRY(fill32(ctx, ctx->tmax.p, 0u, 2 * (int64_t)T));
    if (recon)
      RB_HIP(launch_select_final(ctx->trig1.as<TrigRec>(), ctx->counters.as<unsigned long long>(),
                                 trig_capacity(ctx->trig1), inv_scale, (float)(opts->thr2 * opts->thr2),
                                 ctx->trig2.as<TrigRec>(), trig_capacity(ctx->trig2),
                                 ctx->counters.as<unsigned long long>() + 1, ctx->cnt2.as<int32_t>(),
                                 ctx->want_peaks ? ctx->tmax.as<unsigned long long>() : nullptr, sum1[0],
                                 ctx->stream));
    if (sparse && nsplit[1] > 0) {
      SparseArgs sa = sparse_args(ctx, bank, g, tw, opts->thr2, nullptr, nullptr, 0);
      if (autom) sa.list = ctx->listL.as<int32_t>();
      // one workgroup per group of crossings: offsets on the device, the grid
      // an upper bound (sum of ceil(c / per) <= templates + crossings / per)
      const int64_t per = sparse_crossings_per_group();
      RB_TRY(ctx->goffB.ensure((size_t)(T + 1) * 4));
      RB_HIP(launch_group_offsets(sa.list, nsplit[1], sa.counts, (int)per, ctx->goffB.as<int32_t>(), ctx->stream));
      sa.goff = ctx->goffB.as<int32_t>();
      sa.nlist = nsplit[1];
      const int64_t grid = std::min<int64_t>((int64_t)nsplit[1] + sum1[0] / per, (int64_t(1) << 31) - 1);
      RB_HIP(launch_sparse_exact(sa, (int)grid, 1, ctx->stream));
    }
    if (!sparse && !recon)
      RB_TRY(step_mf(ctx, bank, g, tw, ctx->list1.as<int32_t>(), sum1[1], (float)(opts->thr2 * opts->thr2)));
    else if (sparse && nsplit[0] > 0)
      RB_TRY(step_mf(ctx, bank, g, tw, ctx->listH.as<int32_t>(), nsplit[0], (float)(opts->thr2 * opts->thr2)));
    if (tm) RB_TRY(event(ctx, e_s2));
    RB_TRY(scan_and_read(ctx, T, ctx->cnt2, ctx->off2, ctx->fill2, ctx->list2, sum2));
    if (sum2[0] <= trig_capacity(ctx->trig2)) break;
    RB_TRY(ctx->trig2.ensure((size_t)(sum2[0] + sum2[0] / 4) * sizeof(TrigRec)));
  }
  const rb_status st = finish_stage2(ctx, bank, out, cap, n_out, peaks, sum2);
  if (tm) RB_TRY(event(ctx, e_end));
  RB_HIP(hipStreamSynchronize(ctx->stream));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->n_stage1 = sum1[0];
    stats->n_refiltered = (int32_t)sum1[1];
    stats->n_bins = nbins;
    stats->gemm_mfma_flop = ctx->mfma_flop;
    int kmax = 0;
    stats->min_energy = 1.0;
    for (int32_t m = 0; m < nbases; ++m) {
      kmax = std::max(kmax, (int)bases[m]->K);
      stats->min_energy = std::min(stats->min_energy, bases[m]->min_energy);
    }
    stats->rank = kmax;
    stats->ms[0] = elapsed(ctx, 0, 1);
    for (int32_t m = 0; m < nbases; ++m) {
      stats->ms[1] += elapsed(ctx, m == 0 ? 1 : 3 + 2 * (size_t)(m - 1), 2 + 2 * (size_t)m);
      stats->ms[2] += elapsed(ctx, 2 + 2 * (size_t)m, 3 + 2 * (size_t)m);
    }
    if (w > 1)
      for (int32_t m = 0; m < nbases; ++m) stats->ms[7] += elapsed(ctx, e_end + 1 + (size_t)m, 3 + 2 * (size_t)m);
    if (fold) {   // the template fold is a first stage of its own: counted in [2]
      const float f = elapsed(ctx, e_end + 1 + (size_t)nbases, e_end + 2 + (size_t)nbases);
      stats->ms[2] += f;
      stats->ms[1] -= f;
    }
    stats->ms[3] = elapsed(ctx, 3 + 2 * (size_t)(nbases - 1), e_scan);
    stats->ms[4] = elapsed(ctx, e_scan, e_s2);
    stats->ms[5] = elapsed(ctx, e_s2, e_end);
    stats->ms[6] = elapsed(ctx, 0, e_end);
  }
  return st;
}

extern "C" rb_status rb_filter_stream(rb_ctx ctx, const rb_basis* bases, int32_t nbases, rb_bank bank,
                                      const float* strain, int64_t n, const rb_filter_opts* opts, rb_trigger* out,
                                      int64_t cap, int64_t* n_out, rb_stats* stats) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(bank != nullptr && opts != nullptr && n_out != nullptr && strain != nullptr, RB_ERR_ARG, "NULL argument");
  RB_CHECK(bank->ctx == ctx, RB_ERR_ARG, "bank belongs to another context");
  RB_CHECK(cap >= 0 && (out != nullptr || cap == 0), RB_ERR_ARG, "bad output buffer");
  const int64_t N = bank->grid.N;
  RB_CHECK(n >= N && n <= (int64_t)INT32_MAX, RB_ERR_ARG, "need N <= n < 2^31 samples");
  const float* sdev = strain;
  if (!is_device_ptr(strain)) {
    RB_TRY(ctx->sstrain.ensure((size_t)n * sizeof(float)));
    RB_HIP(hipMemcpyAsync(ctx->sstrain.p, strain, (size_t)n * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    sdev = ctx->sstrain.as<float>();
  }
  rb_trigger* odev = out;
  if (out != nullptr && !is_device_ptr(out)) {
    RB_TRY(ctx->wout.ensure(std::max<size_t>(16, (size_t)cap * sizeof(rb_trigger))));
    odev = ctx->wout.as<rb_trigger>();
  }
  RB_TRY(ctx->wcount.ensure(8));
  RB_TRY(fill32(ctx, ctx->wcount.p, 0u, 2));
  if (ctx->segout.bytes == 0) RB_TRY(ctx->segout.ensure((size_t)1 << 16 << 4));
  const int64_t hop = N / 2, count = (n - N + hop - 1) / hop + 1;
  rb_stats acc;
  std::memset(&acc, 0, sizeof(acc));
  int64_t lo = 0;
  for (int64_t i = 0; i < count; ++i) {
    const int64_t s0 = std::min(i * hop, n - N);
    const int64_t hi = i == count - 1 ? n : std::min((i + 1) * hop, n - N) + N / 4;
    int64_t ni = 0;
    rb_stats st;
    for (;;) {   // the segment's own search; grow the scratch output if it is short
      const int64_t segcap = (int64_t)(ctx->segout.bytes / sizeof(rb_trigger));
      const rb_status r = rb_filter(ctx, bases, nbases, bank, sdev + s0, opts, ctx->segout.as<rb_trigger>(), segcap,
                                    &ni, nullptr, stats ? &st : nullptr);
      if (r == RB_ERR_CAPACITY) {
        RB_TRY(ctx->segout.ensure((size_t)(ni + ni / 4) * sizeof(rb_trigger)));
        continue;
      }
      if (r != RB_OK) return r;
      break;
    }
    if (ni > 0)
      RB_HIP(launch_window(ctx->segout.p, ni, s0, lo, hi, odev, cap, ctx->wcount.as<int64_t>(), ctx->stream));
    if (stats) {
      acc.n_stage1 += st.n_stage1;
      acc.n_refiltered += st.n_refiltered;
      acc.rank = std::max(acc.rank, st.rank);
      acc.n_bins += st.n_bins;
      acc.min_energy = st.min_energy;
      for (int k = 0; k < 8; ++k) acc.ms[k] += st.ms[k];
    }
    lo = hi;
  }
  int64_t total = 0;
  RB_HIP(hipMemcpyAsync(&total, ctx->wcount.p, 8, hipMemcpyDeviceToHost, ctx->stream));
  RB_HIP(hipStreamSynchronize(ctx->stream));
  *n_out = total;
  if (stats) *stats = acc;
  if (total > cap) {
    set_error("trigger capacity " + std::to_string(cap) + " < required " + std::to_string(total));
    return RB_ERR_CAPACITY;
  }
  if (odev != out && total > 0) {
    RB_HIP(hipMemcpyAsync(out, odev, (size_t)total * sizeof(rb_trigger), hipMemcpyDeviceToHost, ctx->stream));
    RB_HIP(hipStreamSynchronize(ctx->stream));
  }
  return RB_OK;
}

extern "C" rb_status mf_full(rb_ctx ctx, rb_bank bank, const float* strain, double thr, rb_trigger* out,
                             int64_t cap, int64_t* n_out, rb_peak* peaks, rb_stats* stats) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(bank != nullptr && n_out != nullptr, RB_ERR_ARG, "NULL argument");
  RB_CHECK(bank->ctx == ctx, RB_ERR_ARG, "bank belongs to another context");
  RB_CHECK(std::isfinite(thr) && thr > 0, RB_ERR_ARG, "thr must be > 0");
  RB_CHECK(cap >= 0, RB_ERR_ARG, "cap must be >= 0");
  const int T = bank->T;
  ctx->want_peaks = peaks != nullptr;
  FftGeom g;
  RB_TRY(geom_for(ctx, bank, &g));
  FftTables tw;
  RB_TRY(get_tables(ctx, g, tw));
  const float* s;
  RB_TRY(strain_device(ctx, strain, g.N, &s));
  RB_TRY(ensure_trigger_scratch(ctx, T));
  record(ctx, stats, 0);
  RB_TRY(fill32(ctx, ctx->flag.p, 0u, 2));
  RB_HIP(launch_check_finite(s, g.N, ctx->flag.as<int64_t>(), ctx->stream));
  RB_TRY(step_spectrum(ctx, bank, g, tw, s));
  record(ctx, stats, 1);
  int64_t sum2[3];
  for (;;) {
    RB_TRY(fill32(ctx, ctx->counters.p, 0u, 4));
    RB_TRY(fill32(ctx, ctx->cnt2.p, 0u, T));
    RB_TRY(fill32(ctx, ctx->tmax.p, 0u, 2 * (int64_t)T));
    RB_TRY(step_mf(ctx, bank, g, tw, nullptr, T, (float)(thr * thr)));
    record(ctx, stats, 2);
    RB_TRY(scan_and_read(ctx, T, ctx->cnt2, ctx->off2, ctx->fill2, ctx->list2, sum2));
    if (sum2[0] <= trig_capacity(ctx->trig2)) break;
    RB_TRY(ctx->trig2.ensure((size_t)(sum2[0] + sum2[0] / 4) * sizeof(TrigRec)));
  }
  int64_t flag = 0;
  RB_HIP(hipMemcpyAsync(&flag, ctx->flag.p, 8, hipMemcpyDeviceToHost, ctx->stream));
  RB_HIP(hipStreamSynchronize(ctx->stream));
  RB_CHECK(flag == 0, RB_ERR_NUMERIC, "strain contains non-finite values");
  const rb_status st = finish_stage2(ctx, bank, out, cap, n_out, peaks, sum2);
  record(ctx, stats, 3);
  RB_HIP(hipStreamSynchronize(ctx->stream));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->n_refiltered = T;
    stats->min_energy = 1.0;     // the exact filter of every template
    float ms;
    if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]) == hipSuccess) stats->ms[0] = ms;
    if (hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]) == hipSuccess) stats->ms[4] = ms;
    if (hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]) == hipSuccess) stats->ms[5] = ms;
    if (hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[3]) == hipSuccess) stats->ms[6] = ms;
    (void)hipGetLastError();
  }
  return st;
}

// ====================================================================== allocation-free template method
// mf_full on a fixed per-GPU scratch (see include/rbmf.h).  Layout of the
// scratch, every part 256-byte aligned: flag, counter and scan summary;
// per-template counts, offsets, fill cursors and list; the whitened data; the
// FFT intermediate (first the FP64 strain transform's N double2, then the
// template passes' [B][N] complex64); three record arrays of R entries
// (unsorted records, grouped records, merge buffer).
extern "C" rb_status mf_full_noalloc(rb_ctx ctx, rb_bank bank, const float* strain, double thr, rb_trigger* out,
                                     int64_t cap, int64_t* n_out) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(bank != nullptr && n_out != nullptr, RB_ERR_ARG, "NULL argument");
  RB_CHECK(bank->ctx == ctx, RB_ERR_ARG, "bank belongs to another context");
  RB_CHECK(std::isfinite(thr) && thr > 0, RB_ERR_ARG, "thr must be > 0");
  RB_CHECK(cap >= 0, RB_ERR_ARG, "cap must be >= 0");
  RB_CHECK(strain != nullptr && is_device_ptr(strain), RB_ERR_ARG, "strain must be a device pointer");
  RB_CHECK(cap == 0 || (out != nullptr && is_device_ptr(out)), RB_ERR_ARG, "out must be a device pointer");
  RB_CHECK(ctx->noalloc != nullptr, RB_ERR_DEVICE, "no scratch address for this device");
  const int64_t N = bank->grid.N;
  const int T = bank->T;
  const auto gi = ctx->fft_n2.find(N);
  const auto ti = ctx->tw.find(N);
  RB_CHECK(gi != ctx->fft_n2.end() && ti != ctx->tw.end(), RB_ERR_ARG,
           "no FFT plan for N = " + std::to_string(N) +
               " in this context yet (one mf_full or rb_filter call on a bank of this grid prepares it)");
  const FftGeom g = make_geom(N, gi->second);
  const FftTables tw{ti->second->pyr.as<float2>(), ti->second->tlo.as<float2>(), ti->second->thi.as<float2>()};
  const FftTables64 tw64{ti->second->pyr64.as<double2>(), ti->second->tlo64.as<double2>(),
                         ti->second->thi64.as<double2>()};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t o_flag = take(8), o_cnt = take(8), o_sum = take(8 * sizeof(int64_t));
  const size_t o_count = take((size_t)T * 4), o_off = take((size_t)T * 4), o_fill = take((size_t)T * 4),
               o_list = take((size_t)T * 4);
  const size_t o_d = take((size_t)bank->nbs * 8);
  const size_t spec_bytes = (size_t)N * 16, vec_bytes = (size_t)N * 8;
  const size_t min_rec_bytes = (size_t(16) << 20) + 3 * 256;   // at least 349 525 records per array
  RB_CHECK(off + spec_bytes + min_rec_bytes <= kNoallocScratchBytes, RB_ERR_ARG,
           "N = " + std::to_string(N) + " with " + std::to_string(T) + " templates needs more than the " +
               std::to_string(kNoallocScratchBytes >> 20) + " MiB fixed scratch of mf_full_noalloc (use mf_full)");
  const int B = (int)std::max<int64_t>(
      1, std::min<int64_t>({16, (int64_t)T, (int64_t)((kNoallocScratchBytes - off - min_rec_bytes) / vec_bytes)}));
  const size_t o_work = take(std::max(spec_bytes, (size_t)B * vec_bytes));
  const int64_t R = (int64_t)((kNoallocScratchBytes - off - 3 * 256) / (3 * sizeof(TrigRec)));
  const size_t o_trig = take((size_t)R * sizeof(TrigRec)), o_recs = take((size_t)R * sizeof(TrigRec)),
               o_tmp = take((size_t)R * sizeof(TrigRec));
  RB_CHECK(off <= kNoallocScratchBytes && R * 3 * sizeof(TrigRec) >= (size_t(16) << 20), RB_ERR_ARG,
           "scratch layout does not fit");
  char* base = static_cast<char*>(ctx->noalloc);
  int64_t* flag = reinterpret_cast<int64_t*>(base + o_flag);
  unsigned long long* counter = reinterpret_cast<unsigned long long*>(base + o_cnt);
  int64_t* summary = reinterpret_cast<int64_t*>(base + o_sum);
  int32_t* counts = reinterpret_cast<int32_t*>(base + o_count);
  int32_t* offsets = reinterpret_cast<int32_t*>(base + o_off);
  int32_t* fill = reinterpret_cast<int32_t*>(base + o_fill);
  int32_t* list = reinterpret_cast<int32_t*>(base + o_list);
  float2* dspec = reinterpret_cast<float2*>(base + o_d);
  TrigRec* trig = reinterpret_cast<TrigRec*>(base + o_trig);
  TrigRec* recs = reinterpret_cast<TrigRec*>(base + o_recs);
  TrigRec* tmp = reinterpret_cast<TrigRec*>(base + o_tmp);

  // one call at a time per GPU: the scratch keeps the previous call's contents
  // and would be shared by overlapping calls
  std::lock_guard<std::mutex> lock(noalloc_scratch_lock(ctx->device));
  const rb_status st = [&]() -> rb_status {
    RB_TRY(fill32(ctx, flag, 0u, 2));
    RB_TRY(fill32(ctx, counter, 0u, 2));
    RB_TRY(fill32(ctx, counts, 0u, T));
    RB_HIP(launch_check_finite(strain, N, flag, ctx->stream));
    RB_TRY(spectrum_into(ctx, bank, g, tw, tw64, strain, reinterpret_cast<double2*>(base + o_work), dspec));
    const MfBufs b{reinterpret_cast<float2*>(base + o_work), B, dspec, trig, R, counter, counts, nullptr};
    RB_TRY(mf_passes(ctx, bank, g, tw, nullptr, T, (float)(thr * thr), nullptr, b));
    RB_HIP(launch_scan_counts(counts, T, offsets, fill, list, summary, ctx->stream));
    int64_t host[4] = {0, 0, 0, 0};
    RB_HIP(hipMemcpyAsync(host, summary, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    RB_HIP(hipMemcpyAsync(host + 3, flag, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    RB_HIP(hipStreamSynchronize(ctx->stream));
    RB_CHECK(host[3] == 0, RB_ERR_NUMERIC, "strain contains non-finite values");
    const int64_t total = host[0];
    *n_out = total;
    RB_CHECK(total <= R, RB_ERR_UNSUPPORTED,
             std::to_string(total) + " crossings exceed the " + std::to_string(R) +
                 " records of the fixed scratch of mf_full_noalloc (use mf_full)");
    RB_CHECK(total <= cap, RB_ERR_CAPACITY,
             "trigger capacity " + std::to_string(cap) + " < required " + std::to_string(total));
    if (total > 0) {
      RB_HIP(launch_scatter_triggers(trig, total, nullptr, offsets, fill, recs, ctx->stream));
      RB_HIP(launch_segment_sort(recs, tmp, offsets, counts, list, (int)host[1], out, nullptr, 0, ctx->stream));
    }
    RB_HIP(hipStreamSynchronize(ctx->stream));
    return RB_OK;
  }();
  (void)hipStreamSynchronize(ctx->stream);   // (error paths) no queued work may outlive the lock
  return st;
}

extern "C" rb_status rb_cluster_peaks(rb_ctx ctx, const rb_trigger* trig, int64_t n, int32_t W, int64_t N,
                                      uint8_t* is_peak) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(n >= 0 && W >= 0 && N > 0, RB_ERR_ARG, "bad sizes");
  if (n == 0) return RB_OK;
  RB_CHECK(trig != nullptr && is_peak != nullptr, RB_ERR_ARG, "NULL argument");
  DevBuf tdev, pdev;
  const void* tp = trig;
  if (!is_device_ptr(trig)) {
    RB_TRY(tdev.ensure((size_t)n * sizeof(rb_trigger)));
    RB_HIP(hipMemcpyAsync(tdev.p, trig, (size_t)n * sizeof(rb_trigger), hipMemcpyHostToDevice, ctx->stream));
    tp = tdev.p;
  }
  uint8_t* pp = is_peak;
  const bool dev_out = is_device_ptr(is_peak);
  if (!dev_out) {
    RB_TRY(pdev.ensure((size_t)n));
    pp = pdev.as<uint8_t>();
  }
  RB_HIP(launch_cluster_peaks(tp, n, W, N, pp, ctx->stream));
  if (!dev_out) RB_HIP(hipMemcpyAsync(is_peak, pp, (size_t)n, hipMemcpyDeviceToHost, ctx->stream));
  RB_HIP(hipStreamSynchronize(ctx->stream));
  return RB_OK;
}

// ====================================================================== debug
extern "C" rb_status rb_debug_rho(rb_ctx ctx, rb_basis basis, rb_bank bank, const float* strain, float* rho) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(bank != nullptr && rho != nullptr, RB_ERR_ARG, "NULL argument");
  RB_CHECK(bank->ctx == ctx && (basis == nullptr || basis->bank == bank), RB_ERR_ARG, "handle mismatch");
  const int T = bank->T;
  const int rows = basis ? basis->T : T;
  FftGeom g;
  RB_TRY(geom_for(ctx, bank, &g));
  RB_CHECK((double)rows * g.N <= 4e9, RB_ERR_ARG, "rows * N too large for a dump");
  FftTables tw;
  RB_TRY(get_tables(ctx, g, tw));
  const float* s;
  RB_TRY(strain_device(ctx, strain, g.N, &s));
  RB_TRY(ensure_trigger_scratch(ctx, T));
  float2* dst = reinterpret_cast<float2*>(rho);
  const bool dev = is_device_ptr(rho);
  if (!dev) {
    RB_TRY(ctx->rho_tmp.ensure((size_t)rows * g.N * 8));
    dst = ctx->rho_tmp.as<float2>();
  }
  RB_TRY(step_spectrum(ctx, bank, g, tw, s));
  if (basis == nullptr) {
    const int B = batch_vectors(g.N, T);
    RB_TRY(ctx->work.ensure((size_t)B * g.N * 8));
    PassArgs a = base_args(bank, g, tw);
    a.sign = +1;
    a.d = ctx->dspec.as<float2>();
    a.src = bank->w.as<float2>();
    a.sup_lo = bank->sup_lo.as<int32_t>();
    a.sup_hi = bank->sup_hi.as<int32_t>();
    a.work = ctx->work.as<float2>();
    a.cout = dst;
    for (int i0 = 0; i0 < T; i0 += B) {
      a.vec_base = i0;
      a.nvec = std::min(B, T - i0);
      RB_HIP(launch_pass1(a, IN_CORR, ctx->stream));
      RB_HIP(launch_pass2(a, OUT_NATURAL, ctx->stream));
    }
  } else {
    RB_TRY(step_basis_outputs(ctx, basis, g, tw));
    RB_TRY(fill32(ctx, ctx->counters.p, 0u, 2));
    RB_TRY(fill32(ctx, ctx->cnt1.p, 0u, T));
    RB_TRY(stage1_gemm(ctx, basis, g, 0.f, dst));   // rows [t0, t0 + T) of the basis
  }
  if (!dev) RB_HIP(hipMemcpyAsync(rho, dst, (size_t)rows * g.N * 8, hipMemcpyDeviceToHost, ctx->stream));
  RB_HIP(hipStreamSynchronize(ctx->stream));
  return RB_OK;
}

extern "C" rb_status rb_debug_rho_binned(rb_ctx ctx, rb_basis basis, const float* strain, int32_t w, float* rho) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(basis != nullptr && rho != nullptr, RB_ERR_ARG, "NULL argument");
  rb_bank bank = basis->bank;
  RB_CHECK(w >= 2 && w <= 64 && (w & (w - 1)) == 0 && bank->grid.N / w >= 256, RB_ERR_ARG,
           "w must be a power of two in [2, 64] with N / w >= 256");
  const int rows = basis->T;
  FftGeom g;
  RB_TRY(geom_for(ctx, bank, &g));
  const int64_t Nb = g.N / w;
  RB_CHECK((double)rows * Nb <= 4e9, RB_ERR_ARG, "rows * N / w too large for a dump");
  FftTables tw;
  RB_TRY(get_tables(ctx, g, tw));
  const float* s;
  RB_TRY(strain_device(ctx, strain, g.N, &s));
  RB_TRY(ensure_trigger_scratch(ctx, bank->T));
  float2* dst = reinterpret_cast<float2*>(rho);
  const bool dev = is_device_ptr(rho);
  if (!dev) {
    RB_TRY(ctx->rho_tmp.ensure((size_t)rows * Nb * 8));
    dst = ctx->rho_tmp.as<float2>();
  }
  RB_TRY(step_spectrum(ctx, bank, g, tw, s));
  const FftGeom gb = binned_geom(g, w);
  RB_TRY(step_basis_outputs_binned(ctx, basis, gb, tw, w));
  RB_TRY(fill32(ctx, ctx->counters.as<unsigned long long>() + 2, 0u, 2));
  RB_TRY(fill32(ctx, ctx->cntB.p, 0u, bank->T));
  RB_TRY(stage1_gemm(ctx, basis, gb, 0.f, dst, w));
  if (!dev) RB_HIP(hipMemcpyAsync(rho, dst, (size_t)rows * Nb * 8, hipMemcpyDeviceToHost, ctx->stream));
  RB_HIP(hipStreamSynchronize(ctx->stream));
  return RB_OK;
}

extern "C" rb_status rb_debug_basis_outputs(rb_ctx ctx, rb_basis basis, const float* strain, float* beta) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(basis != nullptr && beta != nullptr, RB_ERR_ARG, "NULL argument");
  rb_bank bank = basis->bank;
  FftGeom g;
  RB_TRY(geom_for(ctx, bank, &g));
  const int K = basis->K;
  FftTables tw;
  RB_TRY(get_tables(ctx, g, tw));
  const float* s;
  RB_TRY(strain_device(ctx, strain, g.N, &s));
  RB_TRY(step_spectrum(ctx, bank, g, tw, s));
  RB_TRY(step_basis_outputs(ctx, basis, g, tw));
  const int planes = basis->dtype == RB_BF16X3 ? 2 : 1;    // BF16X3: high parts, then low parts
  const size_t bytes = (size_t)planes * K * g.N * 8;
  float2* dst = reinterpret_cast<float2*>(beta);
  const bool dev = is_device_ptr(beta);
  if (!dev) {
    RB_TRY(ctx->rho_tmp.ensure(bytes));
    dst = ctx->rho_tmp.as<float2>();
  }
  const int dt = basis->dtype == RB_BF16X3 ? (int)RB_BF16 : (int)basis->dtype;
  for (int p = 0; p < planes; ++p)
    RB_HIP(launch_z_to_natural(static_cast<const uint16_t*>(ctx->z.p) + (size_t)p * 2 * basis->Kp * g.N, dt, 1.f,
                               g.N, K, g.N1, g.N2, dst + (size_t)p * K * g.N, ctx->stream));
  if (!dev) RB_HIP(hipMemcpyAsync(beta, dst, bytes, hipMemcpyDeviceToHost, ctx->stream));
  RB_HIP(hipStreamSynchronize(ctx->stream));
  return RB_OK;
}

namespace {

// Copies the trigger list (host or device) to host arrays and validates it.
rb_status host_triggers(rb_ctx ctx, const rb_trigger* S, int64_t n, int t0, int T, int64_t N,
                        std::vector<int32_t>& tm, std::vector<int32_t>& sp) {
  std::vector<rb_trigger> h((size_t)n);
  if (n > 0) {
    if (is_device_ptr(S)) {
      RB_HIP(hipMemcpyAsync(h.data(), S, (size_t)n * sizeof(rb_trigger), hipMemcpyDeviceToHost, ctx->stream));
      RB_HIP(hipStreamSynchronize(ctx->stream));
    } else {
      std::memcpy(h.data(), S, (size_t)n * sizeof(rb_trigger));
    }
  }
  tm.resize(n);
  sp.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    RB_CHECK(h[i].tmpl >= t0 && h[i].tmpl < t0 + T && h[i].sample >= 0 && h[i].sample < N, RB_ERR_ARG,
             "trigger " + std::to_string(i) + " outside the basis's templates or the segment");
    tm[i] = h[i].tmpl - t0;     // local row
    sp[i] = h[i].sample;
  }
  return RB_OK;
}

rb_status upload(rb_ctx ctx, DevBuf& b, const void* src, size_t bytes) {
  RB_TRY(b.ensure(std::max<size_t>(bytes, 16)));
  if (bytes) RB_HIP(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, ctx->stream));
  return RB_OK;
}

// Uploads C (host or device, T x K complex64) or points at the basis's own.
rb_status coeffs(rb_ctx ctx, rb_basis basis, const float* C, const float2** out) {
  if (C == nullptr) {
    *out = basis->C32.as<float2>();
    return RB_OK;
  }
  if (is_device_ptr(C)) {
    *out = reinterpret_cast<const float2*>(C);
    return RB_OK;
  }
  const size_t bytes = (size_t)basis->T * basis->K * sizeof(float2);
  RB_TRY(ctx->adjC.ensure(bytes));
  RB_HIP(hipMemcpyAsync(ctx->adjC.p, C, bytes, hipMemcpyHostToDevice, ctx->stream));
  RB_HIP(hipStreamSynchronize(ctx->stream));
  *out = ctx->adjC.as<float2>();
  return RB_OK;
}

// Groups trigger indices by key (stable): order and segment offsets.
void group_by(const std::vector<int32_t>& key, std::vector<int32_t>& order, std::vector<int32_t>& seg) {
  const int64_t n = (int64_t)key.size();
  order.resize(n);
  for (int64_t i = 0; i < n; ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  seg.clear();
  for (int64_t s = 0; s < n; ++s)
    if (s == 0 || key[order[s]] != key[order[s - 1]]) seg.push_back((int32_t)s);
  seg.push_back((int32_t)n);
}

// d, FP32 Z, uploaded triggers and rho at the trigger points.
rb_status adjoint_forward(rb_ctx ctx, rb_basis basis, const float* strain, const rb_trigger* S, int64_t n,
                          const float* C, const FftGeom& g, std::vector<int32_t>& tm, std::vector<int32_t>& sp,
                          const float2** Cd) {
  rb_bank bank = basis->bank;
  FftTables tw;
  RB_TRY(get_tables(ctx, g, tw));
  RB_TRY(host_triggers(ctx, S, n, basis->t0, basis->T, g.N, tm, sp));
  const float* s;
  RB_TRY(strain_device(ctx, strain, g.N, &s));
  RB_TRY(coeffs(ctx, basis, C, Cd));
  RB_TRY(step_spectrum(ctx, bank, g, tw, s));
  RB_TRY(step_basis_outputs(ctx, basis, g, tw, true));
  RB_TRY(upload(ctx, ctx->adjT, tm.data(), tm.size() * 4));
  RB_TRY(upload(ctx, ctx->adjS, sp.data(), sp.size() * 4));
  RB_TRY(ctx->adjRho.ensure(std::max<size_t>(16, (size_t)n * sizeof(float2))));
  RB_HIP(launch_rho_at(ctx->z32.as<float>(), g.N, basis->K, g.N1, g.N2, *Cd, ctx->adjT.as<int32_t>(),
                       ctx->adjS.as<int32_t>(), n, ctx->adjRho.as<float2>(), ctx->stream));
  return RB_OK;
}

}  // namespace

extern "C" rb_status rb_rho_at(rb_ctx ctx, rb_basis basis, const float* strain, const rb_trigger* S, int64_t n,
                               const float* C, float* rho) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(basis != nullptr && basis->ctx == ctx, RB_ERR_ARG, "basis is NULL or from another context");
  RB_CHECK(n >= 0, RB_ERR_ARG, "n must be >= 0");
  if (n == 0) return RB_OK;
  RB_CHECK(S != nullptr && rho != nullptr, RB_ERR_ARG, "NULL argument");
  FftGeom g;
  RB_TRY(geom_for(ctx, basis->bank, &g));
  std::vector<int32_t> tm, sp;
  const float2* Cd;
  RB_TRY(adjoint_forward(ctx, basis, strain, S, n, C, g, tm, sp, &Cd));
  RB_TRY(copy_out(ctx, rho, ctx->adjRho.p, (size_t)n * sizeof(float2)));
  RB_HIP(hipStreamSynchronize(ctx->stream));
  return RB_OK;
}

extern "C" rb_status rb_backward(rb_ctx ctx, rb_basis basis, const float* strain, const rb_trigger* S,
                                 const float* seed, int64_t n, const float* C, float* grad_C, float* grad_strain,
                                 double* loss) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(basis != nullptr && basis->ctx == ctx, RB_ERR_ARG, "basis is NULL or from another context");
  RB_CHECK(n >= 0, RB_ERR_ARG, "n must be >= 0");
  RB_CHECK(n == 0 || S != nullptr, RB_ERR_ARG, "S is NULL");
  rb_bank bank = basis->bank;
  const int T = basis->T, K = basis->K;     // rows of C / grad_C: the basis's templates
  FftGeom g;
  RB_TRY(geom_for(ctx, bank, &g));
  const int64_t N = g.N;
  hipStream_t st = ctx->stream;
  std::vector<int32_t> tm, sp;
  const float2* Cd = nullptr;
  RB_TRY(adjoint_forward(ctx, basis, strain, S, n, C, g, tm, sp, &Cd));
  std::vector<float> gh((size_t)n, 1.f);
  const float* gd = nullptr;
  if (seed) {
    if (is_device_ptr(seed)) {
      RB_HIP(hipMemcpyAsync(gh.data(), seed, (size_t)n * 4, hipMemcpyDeviceToHost, st));
      RB_HIP(hipStreamSynchronize(st));
    } else {
      std::memcpy(gh.data(), seed, (size_t)n * 4);
    }
    RB_TRY(upload(ctx, ctx->adjG, gh.data(), (size_t)n * 4));
    gd = ctx->adjG.as<float>();
  }
  if (loss) {
    std::vector<float2> rh((size_t)n);
    if (n) RB_HIP(hipMemcpyAsync(rh.data(), ctx->adjRho.p, (size_t)n * sizeof(float2), hipMemcpyDeviceToHost, st));
    RB_HIP(hipStreamSynchronize(st));
    double L = 0.0;
    for (int64_t i = 0; i < n; ++i) L += (double)gh[i] * ((double)rh[i].x * rh[i].x + (double)rh[i].y * rh[i].y);
    *loss = L;
  }
  if (grad_C) {
    const size_t bytes = (size_t)T * K * sizeof(float2);
    RB_TRY(ctx->adjGC.ensure(bytes));
    RB_TRY(fill32(ctx, ctx->adjGC.p, 0u, (int64_t)(bytes / 4)));
    std::vector<int32_t> order, seg;
    group_by(tm, order, seg);
    RB_TRY(upload(ctx, ctx->adjOrd, order.data(), order.size() * 4));
    RB_TRY(upload(ctx, ctx->adjSeg, seg.data(), seg.size() * 4));
    RB_HIP(launch_grad_c(ctx->z32.as<float>(), N, K, g.N1, g.N2, ctx->adjOrd.as<int32_t>(), ctx->adjSeg.as<int32_t>(),
                         (int)seg.size() - 1, ctx->adjT.as<int32_t>(), ctx->adjS.as<int32_t>(),
                         ctx->adjRho.as<float2>(), gd, ctx->adjGC.as<float2>(), st));
    RB_TRY(copy_out(ctx, grad_C, ctx->adjGC.p, bytes));
    RB_HIP(hipStreamSynchronize(st));   // order/seg host vectors die here
  }
  if (grad_strain) {
    FftTables tw;
    RB_TRY(get_tables(ctx, g, tw));
    RB_TRY(ctx->adjA.ensure((size_t)K * N * sizeof(float2)));
    RB_TRY(ctx->adjAhat.ensure((size_t)K * N * sizeof(float2)));
    RB_TRY(fill32(ctx, ctx->adjA.p, 0u, (int64_t)K * N * 2));
    std::vector<int32_t> order, seg;
    group_by(sp, order, seg);
    RB_TRY(upload(ctx, ctx->adjOrd, order.data(), order.size() * 4));
    RB_TRY(upload(ctx, ctx->adjSeg, seg.data(), seg.size() * 4));
    RB_HIP(launch_scatter_a(K, N, ctx->adjOrd.as<int32_t>(), ctx->adjSeg.as<int32_t>(), (int)seg.size() - 1,
                            ctx->adjT.as<int32_t>(), ctx->adjS.as<int32_t>(), ctx->adjRho.as<float2>(), gd, Cd,
                            ctx->adjA.as<float2>(), st));
    // Ahat_k[f] = sum_n A_k[n] e^{+2 pi i f n / N}, natural frequency order
    const int B = batch_vectors(N, K);
    RB_TRY(ctx->work.ensure((size_t)B * N * 8));
    PassArgs a = base_args(bank, g, tw);
    a.sign = +1;
    a.src = ctx->adjA.as<float2>();
    a.work = ctx->work.as<float2>();
    a.cout = ctx->adjAhat.as<float2>();
    for (int v0 = 0; v0 < K; v0 += B) {
      a.vec_base = v0;
      a.nvec = std::min(B, K - v0);
      RB_HIP(launch_pass1(a, IN_DENSE, st));
      RB_HIP(launch_pass2(a, OUT_NATURAL, st));
    }
    // B[f] on the band, then dL/ds = 2 Re FFT_-(B)
    RB_TRY(ctx->adjB.ensure((size_t)N * sizeof(float2)));
    RB_TRY(fill32(ctx, ctx->adjB.p, 0u, N * 2));
    RB_HIP(launch_bsum(ctx->adjAhat.as<float2>(), basis->P.as<float2>(), bank->wd.as<double>(), K, N, bank->kb,
                       bank->nbs, bank->k_lo, bank->k_hi, ctx->adjB.as<float2>(), st));
    PassArgs b = base_args(bank, g, tw);
    b.sign = -1;
    b.nvec = 1;
    b.src = ctx->adjB.as<float2>();
    b.work = ctx->work.as<float2>();
    b.cout = ctx->adjAhat.as<float2>();     // reuse: first N entries
    RB_HIP(launch_pass1(b, IN_DENSE, st));
    RB_HIP(launch_pass2(b, OUT_NATURAL, st));
    float* gs = grad_strain;
    DevBuf tmp;
    const bool dev = is_device_ptr(grad_strain);
    if (!dev) {
      RB_TRY(tmp.ensure((size_t)N * 4));
      gs = tmp.as<float>();
    }
    RB_HIP(launch_real2(ctx->adjAhat.as<float2>(), N, gs, st));
    if (!dev) RB_HIP(hipMemcpyAsync(grad_strain, gs, (size_t)N * 4, hipMemcpyDeviceToHost, st));
    RB_HIP(hipStreamSynchronize(st));
  }
  RB_HIP(hipStreamSynchronize(st));
  return RB_OK;
}

extern "C" rb_status rb_refine(rb_ctx ctx, rb_basis basis, const float* strain, const rb_trigger* S, int64_t n,
                               int32_t neighbours, int32_t iters, float* c_out, int32_t* nbr_out, float* p_out) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(basis != nullptr && basis->ctx == ctx, RB_ERR_ARG, "basis is NULL or from another context");
  RB_CHECK(n >= 0, RB_ERR_ARG, "n must be >= 0");
  if (n == 0) return RB_OK;
  RB_CHECK(S != nullptr && c_out != nullptr, RB_ERR_ARG, "NULL argument");
  const int T = basis->T, K = basis->K;
  RB_CHECK(neighbours >= 0 && neighbours <= 32 && neighbours <= T - 1, RB_ERR_ARG,
           "neighbours must lie in [0, min(32, templates of the basis - 1)]");
  RB_CHECK(iters >= 0 && iters <= 100000, RB_ERR_ARG, "iters must lie in [0, 100000]");
  RB_CHECK(K <= refine_max_rank(), RB_ERR_UNSUPPORTED,
           "refinement supports ranks up to " + std::to_string(refine_max_rank()));
  FftGeom g;
  RB_TRY(geom_for(ctx, basis->bank, &g));
  FftTables tw;
  RB_TRY(get_tables(ctx, g, tw));
  std::vector<int32_t> tm, sp;
  RB_TRY(host_triggers(ctx, S, n, basis->t0, T, g.N, tm, sp));
  const float* s;
  RB_TRY(strain_device(ctx, strain, g.N, &s));
  RB_TRY(step_spectrum(ctx, basis->bank, g, tw, s));
  RB_TRY(step_basis_outputs(ctx, basis, g, tw, true));
  RB_TRY(upload(ctx, ctx->adjT, tm.data(), tm.size() * 4));
  RB_TRY(upload(ctx, ctx->adjS, sp.data(), sp.size() * 4));
  const int m = neighbours;
  const int64_t chunk = 512;                      // triggers per launch pair (bounds the scratch)
  const int64_t nc = std::min<int64_t>(n, chunk);
  RB_TRY(ctx->refOv.ensure((size_t)nc * T * sizeof(double)));
  RB_TRY(ctx->refQ.ensure((size_t)nc * (m + 1) * K * sizeof(double2)));
  RB_TRY(ctx->refC.ensure((size_t)n * K * sizeof(float2)));
  RB_TRY(ctx->refN.ensure(std::max<size_t>(16, (size_t)n * m * 4)));
  RB_TRY(ctx->refP.ensure((size_t)n * 2 * sizeof(float)));
  for (int64_t i0 = 0; i0 < n; i0 += chunk) {
    const int cnt = (int)std::min<int64_t>(chunk, n - i0);
    RB_HIP(launch_refine(ctx->z32.as<float>(), g.N, g.N1, g.N2, K, T, basis->t0, basis->C32.as<float2>(),
                         ctx->adjT.as<int32_t>() + i0, ctx->adjS.as<int32_t>() + i0, cnt, m, iters,
                         ctx->refOv.as<double>(), ctx->refQ.as<double2>(), ctx->refC.as<float2>() + i0 * K,
                         ctx->refN.as<int32_t>() + i0 * m, ctx->refP.as<float>() + 2 * i0, ctx->stream));
  }
  RB_TRY(copy_out(ctx, c_out, ctx->refC.p, (size_t)n * K * sizeof(float2)));
  if (nbr_out && m > 0) RB_TRY(copy_out(ctx, nbr_out, ctx->refN.p, (size_t)n * m * 4));
  if (p_out) RB_TRY(copy_out(ctx, p_out, ctx->refP.p, (size_t)n * 2 * sizeof(float)));
  RB_HIP(hipStreamSynchronize(ctx->stream));
  return RB_OK;
}

// ====================================================================== batch
namespace {

// Enqueues the whole search of one item with device-side counts only (no
// host synchronisation), so that it can be captured into a graph.  Results:
// sm[0..2] stage-1 summary, sm[3] non-finite flag, sm[4..6] stage-2 summary,
// triggers in out (cap_item entries, written only if they all fit).
rb_status enqueue_item(rb_ctx ctx, const rb_batch_item& it, const rb_filter_opts* opts, int64_t* sm,
                       rb_trigger* out, int64_t cap_item) {
  rb_bank bank = it.bank;
  const int T = bank->T;
  FftGeom g;
  RB_TRY(geom_for(ctx, bank, &g));
  FftTables tw;
  RB_TRY(get_tables(ctx, g, tw));
  const float* s = it.strain;
  RB_TRY(fill32(ctx, sm, 0u, 16));
  RB_HIP(launch_check_finite(s, g.N, sm + 3, ctx->stream));
  RB_TRY(step_spectrum(ctx, bank, g, tw, s));
  RB_TRY(fill32(ctx, ctx->counters.p, 0u, 4));
  RB_TRY(fill32(ctx, ctx->cnt1.p, 0u, T));
  const float thr1sq = (float)(opts->thr1 * opts->thr1);
  const int w = opts->bin_w >= 2 ? opts->bin_w : 1;
  if (w > 1) {   // binned first stage: bins appended after the snapshot of their counter, per basis
    const FftGeom gb = binned_geom(g, w);
    RB_TRY(fill32(ctx, ctx->counters.as<unsigned long long>() + 2, 0u, 2));
    RB_TRY(fill32(ctx, ctx->cntB.p, 0u, T));
    RB_TRY(ctx->snap.ensure((size_t)it.nbases * 8));
    for (int32_t m = 0; m < it.nbases; ++m) {
      RB_TRY(step_basis_outputs_binned(ctx, it.bases[m], gb, tw, w, (opts->flags & RB_OPT_FP16_INTERMEDIATE) != 0));
      unsigned long long* snap = ctx->snap.as<unsigned long long>() + m;
      RB_HIP(launch_copy_u64(ctx->counters.as<unsigned long long>() + 2, snap, ctx->stream));
      RB_TRY(stage1_gemm(ctx, it.bases[m], gb, (float)(opts->thr_bin * opts->thr_bin), nullptr, w));
      RB_TRY(step_fine(ctx, it.bases[m], gb, w, thr1sq, snap));
    }
    RB_HIP(launch_copy_u64(ctx->counters.as<unsigned long long>() + 2, reinterpret_cast<unsigned long long*>(sm + 7),
                           ctx->stream));
  } else {
    for (int32_t m = 0; m < it.nbases; ++m) {
      RB_TRY(step_basis_outputs(ctx, it.bases[m], g, tw, false, (opts->flags & RB_OPT_FP16_INTERMEDIATE) != 0));
      RB_TRY(stage1_gemm(ctx, it.bases[m], g, thr1sq, nullptr));
    }
  }
  RB_HIP(launch_scan_counts(ctx->cnt1.as<int32_t>(), T, ctx->off1.as<int32_t>(), ctx->fill1.as<int32_t>(),
                            ctx->list1.as<int32_t>(), sm, ctx->stream));
  RB_TRY(fill32(ctx, ctx->cnt2.p, 0u, T));
  RB_TRY(fill32(ctx, ctx->tmax.p, 0u, 2 * (int64_t)T));
  // the low word of sm[1] (little-endian int64, < 2^31) is the stage-1 template count
  const int32_t* nsel = reinterpret_cast<const int32_t*>(sm + 1);
  if (opts->stage2 == RB_STAGE2_RECON) {   // the candidates' own reconstruction is final above thr2
    float* inv = nullptr;
    bool scaled = false;
    for (int32_t m = 0; m < it.nbases; ++m) scaled |= w == 1 && it.bases[m]->dtype != RB_F32;
    if (scaled) {
      RB_TRY(ctx->tinv.ensure((size_t)T * 4));
      for (int32_t m = 0; m < it.nbases; ++m)
        RB_HIP(hipMemcpyAsync(ctx->tinv.as<float>() + it.bases[m]->t0, it.bases[m]->row_inv.p,
                              (size_t)it.bases[m]->T * 4, hipMemcpyDeviceToDevice, ctx->stream));
      inv = ctx->tinv.as<float>();
    }
    RB_TRY(fill32(ctx, ctx->counters.as<unsigned long long>() + 1, 0u, 2));
    RB_HIP(launch_select_final(ctx->trig1.as<TrigRec>(), ctx->counters.as<unsigned long long>(),
                               trig_capacity(ctx->trig1), inv, (float)(opts->thr2 * opts->thr2),
                               ctx->trig2.as<TrigRec>(), trig_capacity(ctx->trig2),
                               ctx->counters.as<unsigned long long>() + 1, ctx->cnt2.as<int32_t>(), nullptr,
                               trig_capacity(ctx->trig1), ctx->stream));
  } else if (opts->stage2 == RB_STAGE2_SPARSE) {
    // group the stage-1 records by template (skipped, like the stage itself, when they overflowed)
    const int64_t cap1 = trig_capacity(ctx->trig1);
    RB_HIP(launch_scatter_triggers(ctx->trig1.as<TrigRec>(), cap1, sm, ctx->off1.as<int32_t>(),
                                   ctx->fill1.as<int32_t>(), ctx->recs1.as<TrigRec>(), ctx->stream));
    // counts are on the device here: a fixed split of every template's crossings over 4 workgroups
    RB_HIP(launch_sparse_exact(sparse_args(ctx, bank, g, tw, opts->thr2, nsel, sm, cap1), T, 4, ctx->stream));
  } else {
    RB_TRY(step_mf(ctx, bank, g, tw, ctx->list1.as<int32_t>(), T, (float)(opts->thr2 * opts->thr2), nsel));
  }
  RB_HIP(launch_scan_counts(ctx->cnt2.as<int32_t>(), T, ctx->off2.as<int32_t>(), ctx->fill2.as<int32_t>(),
                            ctx->list2.as<int32_t>(), sm + 4, ctx->stream));
  const int64_t cap2 = trig_capacity(ctx->trig2);
  RB_HIP(launch_scatter_triggers(ctx->trig2.as<TrigRec>(), cap2, sm + 4, ctx->off2.as<int32_t>(),
                                 ctx->fill2.as<int32_t>(), ctx->recs.as<TrigRec>(), ctx->stream));
  RB_HIP(launch_segment_sort(ctx->recs.as<TrigRec>(), ctx->tmp.as<TrigRec>(), ctx->off2.as<int32_t>(),
                             ctx->cnt2.as<int32_t>(), ctx->list2.as<int32_t>(), T, out, sm + 4, cap_item,
                             ctx->stream));
  return RB_OK;
}

rb_status enqueue_all(rb_ctx ctx, int32_t n, const rb_batch_item* items, const rb_filter_opts* opts,
                      int64_t cap_item) {
  for (int32_t i = 0; i < n; ++i)
    RB_TRY(enqueue_item(ctx, items[i], opts, ctx->bsum.as<int64_t>() + 8 * (size_t)i,
                        ctx->bout.as<rb_trigger>() + (size_t)i * cap_item, cap_item));
  return RB_OK;
}

std::string batch_key(int32_t n, const rb_batch_item* items, const rb_filter_opts* opts, int64_t cap_item,
                      rb_ctx ctx) {
  std::string k;
  auto add = [&](const void* p, size_t b) { k.append(static_cast<const char*>(p), b); };
  add(&n, sizeof(n));
  add(opts, sizeof(*opts));
  add(&cap_item, sizeof(cap_item));
  for (int32_t i = 0; i < n; ++i) {
    add(&items[i].strain, sizeof(void*));
    add(&items[i].bank, sizeof(void*));
    add(&items[i].nbases, sizeof(int32_t));
    for (int32_t m = 0; m < items[i].nbases; ++m) add(&items[i].bases[m], sizeof(void*));
  }
  const void* bufs[] = {ctx->work.p, ctx->work64.p, ctx->dspec.p, ctx->z.p, ctx->trig1.p, ctx->trig2.p,
                        ctx->recs.p, ctx->tmp.p, ctx->bsum.p, ctx->bout.p, ctx->cnt1.p, ctx->cnt2.p,
                        ctx->recs1.p, ctx->zfine.p, ctx->zpart.p, ctx->trigB.p, ctx->cntB.p, ctx->snap.p,
                        ctx->tinv.p, ctx->hscale.p};
  add(bufs, sizeof(bufs));
  return k;
}

}  // namespace

extern "C" rb_status rb_filter_batch(rb_ctx ctx, int32_t nitems, const rb_batch_item* items,
                                     const rb_filter_opts* opts, int32_t use_graph, rb_trigger* out,
                                     int64_t cap_item, int64_t* n_out, rb_stats* stats) {
  RB_TRY(validate_ctx(ctx));
  RB_CHECK(nitems >= 1 && items != nullptr && opts != nullptr && n_out != nullptr, RB_ERR_ARG, "NULL argument");
  RB_CHECK(cap_item >= 0 && (out != nullptr || cap_item == 0), RB_ERR_ARG, "bad output buffer");
  RB_CHECK(std::isfinite(opts->thr1) && opts->thr1 > 0, RB_ERR_ARG, "thr1 must be > 0");
  RB_CHECK(std::isfinite(opts->thr2) && opts->thr2 >= opts->thr1, RB_ERR_ARG, "thr2 must be >= thr1");
  RB_CHECK(opts->stage2 != RB_STAGE2_AUTO, RB_ERR_UNSUPPORTED, "the batch search takes FULL, SPARSE or RECON");
  RB_CHECK(opts->bin_source == 0, RB_ERR_UNSUPPORTED, "the batch search takes bin_source 0");
  RB_CHECK(opts->stage2 == RB_STAGE2_FULL || opts->stage2 == RB_STAGE2_SPARSE || opts->stage2 == RB_STAGE2_RECON,
           RB_ERR_ARG, "bad stage2 mode");
  RB_CHECK((opts->flags & ~RB_OPT_FP16_INTERMEDIATE) == 0, RB_ERR_ARG, "unknown opts flag");
  {
    const int w = opts->bin_w >= 2 ? opts->bin_w : 1;
    RB_CHECK(opts->bin_w >= 0 && opts->bin_w <= 64 && (w & (w - 1)) == 0, RB_ERR_ARG,
             "bin_w must be 0, 1 or a power of two <= 64");
    RB_CHECK(w == 1 || (std::isfinite(opts->thr_bin) && opts->thr_bin > 0), RB_ERR_ARG, "thr_bin must be > 0");
    for (int32_t i = 0; i < nitems; ++i)
      RB_CHECK(items[i].bank == nullptr || items[i].bank->grid.N / w >= 256, RB_ERR_ARG, "N / bin_w must be >= 256");
  }
  int Tmax = 0;
  for (int32_t i = 0; i < nitems; ++i) {
    const rb_batch_item& it = items[i];
    RB_CHECK(it.bank != nullptr && it.bank->ctx == ctx, RB_ERR_ARG, "item bank is NULL or from another context");
    RB_TRY(check_partition(ctx, it.bases, it.nbases, it.bank));
    RB_CHECK(it.strain != nullptr && is_device_ptr(it.strain), RB_ERR_ARG,
             "item " + std::to_string(i) + ": strain must be a device pointer");
    Tmax = std::max(Tmax, it.bank->T);
  }
  RB_TRY(ensure_trigger_scratch(ctx, Tmax));
  ctx->want_peaks = false;   // the batch returns triggers only
  RB_TRY(ctx->bsum.ensure((size_t)nitems * 8 * 8));
  RB_TRY(ctx->bout.ensure(std::max<size_t>(16, (size_t)nitems * cap_item * sizeof(rb_trigger))));
  const size_t cap2 = (size_t)trig_capacity(ctx->trig2);
  RB_TRY(ctx->recs.ensure(cap2 * sizeof(TrigRec)));
  RB_TRY(ctx->tmp.ensure(cap2 * sizeof(TrigRec)));
  RB_TRY(ctx->recs1.ensure((size_t)trig_capacity(ctx->trig1) * sizeof(TrigRec)));
  std::vector<int64_t> sm((size_t)nitems * 8);
  const bool tm = stats != nullptr;
  // Each attempt counts every level whose input fitted, so overflows that
  // cascade (bins -> stage-1 records -> stage-2 records) settle within one
  // attempt per level; the loop ends only on an attempt with nothing to grow.
  bool settled = false;
  for (int attempt = 0; attempt < 6 && !settled; ++attempt) {
    if (tm) RB_TRY(event(ctx, 0));
    if (use_graph) {
      std::string key = batch_key(nitems, items, opts, cap_item, ctx);
      if (ctx->gkey != key || !ctx->gexec) {
        // eager pass: sizes every buffer and fills every cache outside the capture
        RB_TRY(enqueue_all(ctx, nitems, items, opts, cap_item));
        RB_HIP(hipStreamSynchronize(ctx->stream));
        key = batch_key(nitems, items, opts, cap_item, ctx);
        if (!ctx->gstream) RB_HIP(hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking));
        if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
        ctx->gexec = nullptr;
        hipStream_t user = ctx->stream;
        ctx->stream = ctx->gstream;
        hipGraph_t graph = nullptr;
        rb_status rs = RB_OK;
        if (hipStreamBeginCapture(ctx->gstream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
          ctx->stream = user;
          set_error("hipStreamBeginCapture failed");
          return RB_ERR_DEVICE;
        }
        rs = enqueue_all(ctx, nitems, items, opts, cap_item);
        const hipError_t ec = hipStreamEndCapture(ctx->gstream, &graph);
        ctx->stream = user;
        if (rs != RB_OK) {
          if (graph) (void)hipGraphDestroy(graph);
          return rs;
        }
        RB_CHECK(ec == hipSuccess && graph != nullptr, RB_ERR_DEVICE, "graph capture failed");
        const hipError_t ei = hipGraphInstantiate(&ctx->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        RB_CHECK(ei == hipSuccess, RB_ERR_DEVICE, "hipGraphInstantiate failed");
        ctx->gkey = key;
      }
      // order the replay after the caller's stream and the caller's stream after it
      RB_TRY(event(ctx, 1));
      RB_HIP(hipStreamWaitEvent(ctx->gstream, ctx->evs[1], 0));
      RB_HIP(hipGraphLaunch(ctx->gexec, ctx->gstream));
      RB_HIP(hipEventRecord(ctx->evs[1], ctx->gstream));
      RB_HIP(hipStreamWaitEvent(ctx->stream, ctx->evs[1], 0));
    } else {
      RB_TRY(enqueue_all(ctx, nitems, items, opts, cap_item));
    }
    if (tm) RB_TRY(event(ctx, 2));
    RB_HIP(hipMemcpyAsync(sm.data(), ctx->bsum.p, sm.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    RB_HIP(hipStreamSynchronize(ctx->stream));
    bool grow = false;
    for (int32_t i = 0; i < nitems; ++i) {
      const int64_t* q = &sm[8 * (size_t)i];
      RB_CHECK(q[3] == 0, RB_ERR_NUMERIC, "item " + std::to_string(i) + ": strain contains non-finite values");
      if (q[0] > trig_capacity(ctx->trig1)) {
        const size_t c = (size_t)(q[0] + q[0] / 4);
        RB_TRY(ctx->trig1.ensure(c * sizeof(TrigRec)));
        RB_TRY(ctx->recs1.ensure(c * sizeof(TrigRec)));
        grow = true;
      }
      if (opts->bin_w >= 2 && q[7] > trig_capacity(ctx->trigB)) {
        RB_TRY(ctx->trigB.ensure((size_t)(q[7] + q[7] / 4) * sizeof(TrigRec)));
        grow = true;
      }
      if (q[4] > trig_capacity(ctx->trig2)) {
        const size_t c = (size_t)(q[4] + q[4] / 4);
        RB_TRY(ctx->trig2.ensure(c * sizeof(TrigRec)));
        RB_TRY(ctx->recs.ensure(c * sizeof(TrigRec)));
        RB_TRY(ctx->tmp.ensure(c * sizeof(TrigRec)));
        grow = true;
      }
    }
    if (!grow) {
      settled = true;
    } else {
      ctx->gkey.clear();   // buffers moved: re-record
    }
  }
  RB_CHECK(settled, RB_ERR_CAPACITY, "internal trigger buffers still overflowed after six attempts");
  bool over = false;
  for (int32_t i = 0; i < nitems; ++i) {
    n_out[i] = sm[8 * (size_t)i + 4];
    if (n_out[i] > cap_item) over = true;
  }
  if (!over) {
    for (int32_t i = 0; i < nitems; ++i)
      RB_TRY(copy_out(ctx, out + (size_t)i * cap_item, ctx->bout.as<rb_trigger>() + (size_t)i * cap_item,
                      (size_t)n_out[i] * sizeof(rb_trigger)));
  }
  RB_HIP(hipStreamSynchronize(ctx->stream));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->min_energy = 1.0;
    for (int32_t i = 0; i < nitems; ++i) {
      for (int32_t m = 0; m < items[i].nbases; ++m)
        stats->min_energy = std::min(stats->min_energy, items[i].bases[m]->min_energy);
      stats->n_stage1 += sm[8 * (size_t)i];
      stats->n_refiltered += (int32_t)sm[8 * (size_t)i + 1];
      if (opts->bin_w >= 2) stats->n_bins += sm[8 * (size_t)i + 7];
    }
    stats->ms[6] = elapsed(ctx, 0, 2);
  }
  if (over) {
    set_error("per-item trigger capacity " + std::to_string(cap_item) + " exceeded");
    return RB_ERR_CAPACITY;
  }
  return RB_OK;
}
