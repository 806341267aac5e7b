// Trigger bookkeeping: per-template counts -> offsets and the list of
// templates that crossed (the first-stage selection of Sec. III.C), scatter of
// the unordered trigger records into per-template segments, a per-segment
// sort by sample (deterministic (tmpl, sample) order), per-template peaks and
// clustered peaks.
#include "../../include/rbmf.h"
#include "internal.h"

namespace rbmf {

namespace {

constexpr int SCAN_T = 1024;
constexpr int SEG_LDS = 4096;      // records sorted in LDS per pass

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Block-wide exclusive scan of one value per thread (SCAN_T threads).
__device__ __forceinline__ int block_excl_scan(int x, int* sh, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = x;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  if (lane == 63) sh[w] = incl;
  __syncthreads();
  if (w == 0) {
    int v = lane < SCAN_T / 64 ? sh[lane] : 0;
    int vi = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(vi, off);
      if (lane >= off) vi += y;
    }
    if (lane < SCAN_T / 64) sh[32 + lane] = vi - v;
    if (lane == SCAN_T / 64 - 1) sh[31] = vi;
  }
  __syncthreads();
  const int r = sh[32 + w] + incl - x;
  total = sh[31];
  __syncthreads();
  return r;
}

// counts[T] -> offsets (exclusive), fill = 0, list of templates with count > 0,
// summary = {total, nlist, max count}.
__global__ __launch_bounds__(SCAN_T) void k_scan_counts(const int32_t* counts, int T, int32_t* offsets,
                                                        int32_t* fill, int32_t* list, int64_t* summary) {
  __shared__ int sh[64];
  __shared__ int smax[SCAN_T / 64];
  int64_t carry = 0;
  int lcarry = 0;
  int mx = 0;
  for (int base = 0; base < T; base += SCAN_T) {
    const int i = base + threadIdx.x;
    const int c = i < T ? counts[i] : 0;
    mx = c > mx ? c : mx;
    int tot, ltot;
    const int ex = block_excl_scan(c, sh, tot);
    const int lex = block_excl_scan(c > 0 ? 1 : 0, sh, ltot);
    if (i < T) {
      offsets[i] = (int32_t)(carry + ex);
      fill[i] = 0;
      if (c > 0) list[lcarry + lex] = i;
    }
    carry += tot;
    lcarry += ltot;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const int o = __shfl_xor(mx, off);
    mx = o > mx ? o : mx;
  }
  if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    int m = 0;
    for (int w = 0; w < SCAN_T / 64; ++w) m = smax[w] > m ? smax[w] : m;
    summary[0] = carry;
    summary[1] = lcarry;
    summary[2] = m;
  }
}

// Workgroup offsets of the sparse second stage: template list[i] takes
// ceil(counts[list[i]] / per) workgroups, goff = their exclusive prefix sums.
__global__ __launch_bounds__(SCAN_T) void k_group_offsets(const int32_t* list, int n, const int32_t* counts, int per,
                                                          int32_t* goff) {
  __shared__ int sh[64];
  int carry = 0;
  for (int base = 0; base < n; base += SCAN_T) {
    const int i = base + threadIdx.x;
    const int g = i < n ? (counts[list[i]] + per - 1) / per : 0;
    int tot;
    const int ex = block_excl_scan(g, sh, tot);
    if (i < n) goff[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) goff[n] = carry;
}

// n_dev (optional): device record count; nothing is scattered when it exceeds
// n (records were dropped at capacity; the caller reports it).
__global__ void k_scatter(const TrigRec* in, int64_t n, const int64_t* n_dev, const int32_t* offsets,
                          int32_t* fill, TrigRec* out) {
  if (n_dev != nullptr) {
    if (*n_dev > n) return;
    n = *n_dev;
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const TrigRec r = in[i];
    const int pos = offsets[r.tmpl] + atomicAdd(&fill[r.tmpl], 1);
    out[pos] = r;
  }
}

__device__ __forceinline__ rb_trigger to_trigger(const TrigRec& r) {
  rb_trigger t;
  t.tmpl = r.tmpl;
  t.sample = r.sample;
  t.snr = sqrtf(r.re * r.re + r.im * r.im);
  t.phase = atan2f(r.im, r.re);
  return t;
}

// Bitonic sort of (sample, index) pairs held in LDS; n2 is a power of two.
__device__ void lds_bitonic(int2* s, int n2) {
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += blockDim.x) {
        const int p = i ^ j;
        if (p > i) {
          const int2 a = s[i], b = s[p];
          const bool up = (i & k) == 0;
          if ((a.x > b.x) == up) {
            s[i] = b;
            s[p] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

// One workgroup per listed template.  Segments up to SEG_LDS records are
// sorted in LDS; longer ones are sorted in runs of SEG_LDS and merged in
// global memory (ping-pong between recs and tmp, merge by rank: keys are
// distinct samples).
// summary_dev (optional, graph mode): {total, nlist, ...} on the device; the
// grid then covers every template, workgroups beyond nlist exit, and nothing
// is written when total exceeds out_cap.
__global__ __launch_bounds__(1024) void k_segment_sort(TrigRec* recs, TrigRec* tmp, const int32_t* offsets,
                                                       const int32_t* counts, const int32_t* list,
                                                       rb_trigger* out, const int64_t* summary_dev,
                                                       int64_t out_cap) {
  __shared__ int2 s[SEG_LDS];
  if (summary_dev != nullptr && (blockIdx.x >= summary_dev[1] || summary_dev[0] > out_cap)) return;
  const int j = list[blockIdx.x];
  const int off = offsets[j];
  const int c = counts[j];
  TrigRec* src = recs + off;
  TrigRec* alt = tmp + off;
  // sort runs
  for (int r0 = 0; r0 < c; r0 += SEG_LDS) {
    const int m = min(SEG_LDS, c - r0);
    int n2 = 1;
    while (n2 < m) n2 <<= 1;
    for (int i = threadIdx.x; i < n2; i += blockDim.x)
      s[i] = i < m ? make_int2(src[r0 + i].sample, r0 + i) : make_int2(0x7fffffff, -1);
    __syncthreads();
    lds_bitonic(s, n2);
    if (c <= SEG_LDS) {
      for (int i = threadIdx.x; i < m; i += blockDim.x) out[off + i] = to_trigger(src[s[i].y]);
      return;
    }
    for (int i = threadIdx.x; i < m; i += blockDim.x) alt[r0 + i] = src[s[i].y];
    __syncthreads();
  }
  // merge passes: runs of width w in `alt` -> `src`, alternating
  TrigRec* a = alt;
  TrigRec* b = src;
  for (int w = SEG_LDS; w < c; w <<= 1) {
    for (int i = threadIdx.x; i < c; i += blockDim.x) {
      const int run = i / w;
      const int pair = run >> 1;
      const int lo = pair * 2 * w;
      const int mid = min(lo + w, c);
      const int hi = min(lo + 2 * w, c);
      const int key = a[i].sample;
      int rank;
      if (i < mid) {   // left run: count right-run keys < key
        int l = mid, h = hi;
        while (l < h) {
          const int md = (l + h) >> 1;
          if (a[md].sample < key) l = md + 1; else h = md;
        }
        rank = (i - lo) + (l - mid);
      } else {         // right run: count left-run keys < key
        int l = lo, h = mid;
        while (l < h) {
          const int md = (l + h) >> 1;
          if (a[md].sample < key) l = md + 1; else h = md;
        }
        rank = (i - mid) + (l - lo);
      }
      b[lo + rank] = a[i];
    }
    __syncthreads();
    TrigRec* t = a;
    a = b;
    b = t;
  }
  for (int i = threadIdx.x; i < c; i += blockDim.x) out[off + i] = to_trigger(a[i]);
}

// tmax keys are never zero once a template has been evaluated (the low word
// holds ~n), so key == 0 marks "not evaluated by this call".
__global__ void k_peaks(const unsigned long long* tmax, int T, rb_peak* out) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < T; j += gridDim.x * blockDim.x) {
    rb_peak p;
    const unsigned long long key = tmax[j];
    if (key == 0ull) {
      p.snr = -1.f;
      p.sample = -1;
    } else {
      p.snr = sqrtf(__uint_as_float((uint32_t)(key >> 32)));
      p.sample = (int32_t)(0xffffffffu - (uint32_t)(key & 0xffffffffu));
    }
    out[j] = p;
  }
}

__global__ void k_cluster(const rb_trigger* t, int64_t n, int W, int64_t N, uint8_t* is_peak) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int j = t[i].tmpl;
    const int64_t s = t[i].sample;
    const float v = t[i].snr;
    // segment [b, e) of template j
    int64_t l = 0, h = i;
    while (l < h) {
      const int64_t m = (l + h) >> 1;
      if (t[m].tmpl < j) l = m + 1; else h = m;
    }
    const int64_t b = l;
    l = i + 1;
    h = n;
    while (l < h) {
      const int64_t m = (l + h) >> 1;
      if (t[m].tmpl <= j) l = m + 1; else h = m;
    }
    const int64_t e = l;
    bool peak = true;
    auto beats = [&](int64_t k) {
      const float u = t[k].snr;
      return u > v || (u == v && t[k].sample < s);
    };
    for (int64_t k = i - 1; k >= b && peak && s - t[k].sample <= W; --k) if (beats(k)) peak = false;
    for (int64_t k = i + 1; k < e && peak && t[k].sample - s <= W; ++k) if (beats(k)) peak = false;
    if (peak && s - W < 0)      // wrap: samples near the end of the segment
      for (int64_t k = e - 1; k > i && peak && t[k].sample >= s - W + N; --k) if (beats(k)) peak = false;
    if (peak && s + W >= N)     // wrap: samples near the start
      for (int64_t k = b; k < i && peak && t[k].sample <= s + W - N; ++k) if (beats(k)) peak = false;
    is_peak[i] = peak ? 1 : 0;
  }
}

// Splits a template list by first-stage crossing count: counts >= thresh to
// `heavy`, the rest to `light`; n_out[0] / n_out[1] (zeroed by the caller)
// receive the two lengths.  The order inside each list is arbitrary.
__global__ void k_split_list(const int32_t* list, int64_t n, const int32_t* counts, int thresh, int32_t* heavy,
                             int32_t* light, int32_t* n_out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int j = list[i];
    if (counts[j] >= thresh)
      heavy[atomicAdd(&n_out[0], 1)] = j;
    else
      light[atomicAdd(&n_out[1], 1)] = j;
  }
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)g), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_split_list(const int32_t* list, int64_t n, const int32_t* counts, int thresh, int32_t* heavy,
                             int32_t* light, int32_t* n_out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t g = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_split_list, dim3((unsigned)g), dim3(256), 0, s, list, n, counts, thresh, heavy, light, n_out);
  return hipGetLastError();
}

// Overlap-save stitching: keeps the triggers (sorted by template, sample) of
// one segment whose stream sample (sample + shift) lies in [lo, hi), shifted,
// appended in order after the *n_out already written (one workgroup, chunks
// of SCAN_T with a block scan, so the order is preserved).
__global__ __launch_bounds__(SCAN_T) void k_window(const rb_trigger* in, int64_t n, int64_t shift, int64_t lo,
                                                   int64_t hi, rb_trigger* out, int64_t cap, int64_t* n_out) {
  __shared__ int sh[64];
  int64_t base = *n_out;
  for (int64_t c0 = 0; c0 < n; c0 += SCAN_T) {
    const int64_t i = c0 + threadIdx.x;
    rb_trigger t;
    int keep = 0;
    if (i < n) {
      t = in[i];
      const int64_t g = (int64_t)t.sample + shift;
      keep = (g >= lo && g < hi) ? 1 : 0;
      t.sample = (int32_t)g;
    }
    int tot;
    const int ex = block_excl_scan(keep, sh, tot);
    if (keep && base + ex < cap) out[base + ex] = t;
    base += tot;
  }
  if (threadIdx.x == 0) *n_out = base;
}

hipError_t launch_window(const void* in, int64_t n, int64_t shift, int64_t lo, int64_t hi, void* out, int64_t cap,
                         int64_t* n_out, hipStream_t s) {
  hipLaunchKernelGGL(k_window, dim3(1), dim3(SCAN_T), 0, s, static_cast<const rb_trigger*>(in), n, shift, lo, hi,
                     static_cast<rb_trigger*>(out), cap, n_out);
  return hipGetLastError();
}

hipError_t launch_group_offsets(const int32_t* list, int n, const int32_t* counts, int per, int32_t* goff,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_group_offsets, dim3(1), dim3(SCAN_T), 0, s, list, n, counts, per, goff);
  return hipGetLastError();
}

hipError_t launch_scan_counts(const int32_t* counts, int T, int32_t* offsets, int32_t* fill,
                              int32_t* list, int64_t* summary, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(SCAN_T), 0, s, counts, T, offsets, fill, list, summary);
  return hipGetLastError();
}

hipError_t launch_scatter_triggers(const TrigRec* in, int64_t n, const int64_t* n_dev, const int32_t* offsets,
                                   int32_t* fill, TrigRec* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)g), dim3(256), 0, s, in, n, n_dev, offsets, fill, out);
  return hipGetLastError();
}

hipError_t launch_segment_sort(TrigRec* recs, TrigRec* tmp, const int32_t* offsets, const int32_t* counts,
                               const int32_t* list, int nlist, void* out, const int64_t* summary_dev,
                               int64_t out_cap, hipStream_t s) {
  if (nlist <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_segment_sort, dim3(nlist), dim3(1024), 0, s, recs, tmp, offsets, counts, list,
                     static_cast<rb_trigger*>(out), summary_dev, out_cap);
  return hipGetLastError();
}

hipError_t launch_peaks_from_max(const unsigned long long* tmax, int T, void* out_peaks, hipStream_t s) {
  hipLaunchKernelGGL(k_peaks, dim3((T + 255) / 256), dim3(256), 0, s, tmax, T,
                     static_cast<rb_peak*>(out_peaks));
  return hipGetLastError();
}

hipError_t launch_cluster_peaks(const void* trig, int64_t n, int W, int64_t N, uint8_t* is_peak,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_cluster, dim3((unsigned)g), dim3(256), 0, s, static_cast<const rb_trigger*>(trig),
                     n, W, N, is_peak);
  return hipGetLastError();
}

}  // namespace rbmf
