// Discord time detection over the k sketched profiles (paper Algorithm 2) and
// the ordered list of non-overlapping discords (Sections IV-B and IV-C).
//
//   combine:  A[i] = max over groups of P[g][i] with the first group kept on
//             ties (Algorithm 2 replaces its best only on a strictly larger
//             score); non-finite scores (no admissible neighbour) are dropped.
//   select:   one 256-thread block per series runs all K greedy passes: each
//             pass takes the first maximum of A among windows not masked by
//             earlier picks; a pick masks |i - i*| < halfwidth.  Maxima per
//             block of windows (computed with A) make a pass a reduction over
//             the blocks plus a re-scan of the few blocks the new mask touches.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <climits>
#include <mutex>
#include <string>
#include <vector>

#include "skmp_common.hpp"

namespace skmp {

// Windows per block maximum: a power of two >= 256, chosen per call so that
// every series has at most SEL_LDS_BLOCKS blocks (they live in LDS during
// the selection).
constexpr int DISC_BLK_MIN_SHIFT = 8;
constexpr int SEL_THREADS = 256;
constexpr int SEL_WAVES = SEL_THREADS / 64;
constexpr int MAX_TOPK = 256;
constexpr int SEL_LDS_BLOCKS = 4096;
constexpr int RESCAN_BATCH = 4;  // (1 << DISC_BLK_MIN_SHIFT) / 64: a whole minimum-size block per lane

struct DiscSeries {
  int64_t col;
  int64_t n_sub;     // 0 if the series is shorter than m
  int64_t blk_base;  // first block maximum of this series
  int32_t nblk;
  int32_t pad_;
};

struct DiscState {
  const DiscSeries* ser;
  int n_series;
  int top_k;
  int halfwidth;
  int shift;  // log2 of the windows per block
  int64_t total_blocks;
  double* A;
  int32_t* G;
  double* bval;   // per block: max of A over the block (-inf if none)
  int32_t* bidx;  // its first window (index within the series), -1 if none
  int8_t* bgrp;   // the group of that window
  int64_t* idx;   // outputs
  int32_t* group;
  double* score;
  int32_t* n_found;
};

__device__ __forceinline__ bool better(double v, int64_t i, double bv, int64_t bi) {
  return v > bv || (v == bv && i < bi);
}

__device__ __forceinline__ void wave_best(double& v, int& i) {
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_down(v, off);
    const int oi = __shfl_down(i, off);
    if (better(ov, oi, v, i)) {
      v = ov;
      i = oi;
    }
  }
}

// the same, carrying a payload that follows the winner
__device__ __forceinline__ void wave_best(double& v, int& i, int& pay) {
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_down(v, off);
    const int oi = __shfl_down(i, off);
    const int op = __shfl_down(pay, off);
    if (better(ov, oi, v, i)) {
      v = ov;
      i = oi;
      pay = op;
    }
  }
}

__device__ __forceinline__ int find_block_series(const DiscSeries* ser, int n, int64_t b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ser[mid].blk_base <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// A[i] = max over groups of P[g][i], first group on ties, non-finite scores
// dropped; one 256-thread block per block of 2^shift windows, which also
// writes that block's maximum (first window on ties).
__global__ __launch_bounds__(256) void combine_kernel(const double* __restrict__ P, int64_t ldp, int k, DiscState st) {
  __shared__ double wv[4];
  __shared__ int wi[4];
  const int64_t b = blockIdx.x;
  const int s = find_block_series(st.ser, st.n_series, b);
  const DiscSeries sr = st.ser[s];
  const int64_t first = (b - sr.blk_base) << st.shift;
  const int64_t last = min(first + ((int64_t)1 << st.shift), sr.n_sub);
  double bv = -INFINITY;
  int bi = INT_MAX;
  for (int64_t i = first + threadIdx.x; i < last; i += 256) {
    const int64_t t = sr.col + i;
    double best = -INFINITY;
    int32_t bg = -1;
    for (int g = 0; g < k; ++g) {
      const double v = P[(int64_t)g * ldp + t];
      if (isfinite(v) && v > best) {
        best = v;
        bg = g;
      }
    }
    st.A[t] = best;
    st.G[t] = bg;
    if (best > -INFINITY && better(best, i, bv, bi)) {
      bv = best;
      bi = (int)i;
    }
  }
  wave_best(bv, bi);
  if ((threadIdx.x & 63) == 0) {
    wv[threadIdx.x >> 6] = bv;
    wi[threadIdx.x >> 6] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < 4; ++q)
      if (better(wv[q], wi[q], bv, bi)) {
        bv = wv[q];
        bi = wi[q];
      }
    st.bval[b] = bv;
    st.bidx[b] = bv > -INFINITY ? bi : -1;
    st.bgrp[b] = bv > -INFINITY ? (int8_t)st.G[sr.col + bi] : (int8_t)-1;
  }
}

// One 256-thread block per series runs the K greedy passes.  The block maxima
// sit in LDS; a pass takes the best block (its maximum is the best unmasked
// window: ties resolve to the smallest window, as blocks are in window order),
// records it, and re-scans only the blocks that the new mask |i - i*| < h
// touches, skipping windows masked by any pick so far.
__global__ __launch_bounds__(SEL_THREADS) void select_kernel(DiscState st) {
  extern __shared__ __attribute__((aligned(16))) unsigned char sel_lds[];
  double* sv = reinterpret_cast<double*>(sel_lds);
  int* si = reinterpret_cast<int*>(sv + SEL_LDS_BLOCKS);
  int8_t* sg = reinterpret_cast<int8_t*>(si + SEL_LDS_BLOCKS);
  __shared__ int64_t picks[MAX_TOPK];
  __shared__ double wv[SEL_WAVES];
  __shared__ int wi[SEL_WAVES], wb[SEL_WAVES];
  __shared__ double pv;
  __shared__ int pi;
  const int s = blockIdx.x;
  const DiscSeries sr = st.ser[s];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = sr.nblk;
  const int64_t h = st.halfwidth;
  const int B = 1 << st.shift;
  for (int b = tid; b < nb; b += SEL_THREADS) {
    sv[b] = st.bval[sr.blk_base + b];
    si[b] = st.bidx[sr.blk_base + b];
    sg[b] = st.bgrp[sr.blk_base + b];
  }
  __syncthreads();
  int found = 0;
  for (int pass = 0; pass < st.top_k; ++pass) {
    // best block
    double v = -INFINITY;
    int bi = INT_MAX, bb = -1;
    for (int b = tid; b < nb; b += SEL_THREADS)
      if (sv[b] > -INFINITY && better(sv[b], si[b], v, bi)) {
        v = sv[b];
        bi = si[b];
        bb = b;
      }
    wave_best(v, bi, bb);
    if (lane == 0) {
      wv[wave] = v;
      wi[wave] = bi;
      wb[wave] = bb;
    }
    __syncthreads();
    if (wave == 0) {
      // second level: the wave maxima, reduced by wave 0
      v = lane < SEL_WAVES ? wv[lane] : -INFINITY;
      bi = lane < SEL_WAVES ? wi[lane] : INT_MAX;
      bb = lane < SEL_WAVES ? wb[lane] : -1;
      wave_best(v, bi, bb);
    }
    if (tid == 0) {
      pv = v;
      pi = bi;
      const int64_t o = (int64_t)s * st.top_k + pass;
      if (v > -INFINITY) {
        st.idx[o] = bi;
        st.group[o] = sg[bb];
        st.score[o] = v;
        picks[pass] = bi;
      }
    }
    __syncthreads();
    const double best = pv;
    const int64_t ip = pi;
    if (!(best > -INFINITY)) break;
    found = pass + 1;
    if (pass + 1 == st.top_k) break;
    // re-scan the blocks the new mask touches: wave w takes block r0 + w
    const int b_lo = (int)(max<int64_t>(0, ip - h + 1) >> st.shift);
    const int b_hi = (int)(min<int64_t>(sr.n_sub - 1, ip + h - 1) >> st.shift);
    for (int r0 = b_lo; r0 <= b_hi; r0 += SEL_WAVES) {
      const int b = r0 + wave;
      if (b <= b_hi) {
        const int64_t w0 = (int64_t)b << st.shift;
        const int64_t w1 = min(w0 + B, sr.n_sub);
        double x = -INFINITY;
        int xi = INT_MAX, xg = -1;
        // all RESCAN_BATCH loads of a lane are issued before any is used, so a
        // pass waits for one memory round trip instead of one per load
        for (int64_t i0 = w0 + lane; i0 < w1; i0 += 64 * RESCAN_BATCH) {
          double a[RESCAN_BATCH];
          int ga[RESCAN_BATCH];
#pragma unroll
          for (int u = 0; u < RESCAN_BATCH; ++u) {
            const int64_t i = i0 + 64 * u;
            a[u] = i < w1 ? st.A[sr.col + i] : -INFINITY;
            ga[u] = i < w1 ? st.G[sr.col + i] : -1;
          }
#pragma unroll
          for (int u = 0; u < RESCAN_BATCH; ++u) {
            const int64_t i = i0 + 64 * u;
            if (!(a[u] > -INFINITY) || !better(a[u], i, x, xi)) continue;
            bool masked = false;
            for (int q = 0; q <= pass; ++q) {
              const int64_t p = picks[q];
              masked |= (i - p < h) && (p - i < h);
            }
            if (!masked) {
              x = a[u];
              xi = (int)i;
              xg = ga[u];
            }
          }
        }
        wave_best(x, xi, xg);
        if (lane == 0) {
          sv[b] = x;
          si[b] = x > -INFINITY ? xi : -1;
          sg[b] = (int8_t)(x > -INFINITY ? xg : -1);
        }
      }
    }
    __syncthreads();
  }
  // entries past the last pick
  for (int p = found + tid; p < st.top_k; p += SEL_THREADS) {
    const int64_t o = (int64_t)s * st.top_k + p;
    st.idx[o] = -1;
    st.group[o] = -1;
    st.score[o] = __longlong_as_double(0x7FF8000000000000ll);
  }
  if (tid == 0) st.n_found[s] = found;
}

// Block size (log2) and per-series block ranges; ds (n_series entries) may be
// null when only the block count is wanted.
static int disc_plan(int64_t n_series, const int64_t* offsets, int32_t m, DiscSeries* ds, int64_t& blocks) {
  int64_t max_nsub = 0;
  for (int64_t s = 0; s < n_series; ++s) {
    const int64_t n = offsets[s + 1] - offsets[s];
    max_nsub = std::max<int64_t>(max_nsub, n >= m ? n - m + 1 : 0);
  }
  int shift = DISC_BLK_MIN_SHIFT;
  while ((max_nsub + (1ll << shift) - 1) >> shift > SEL_LDS_BLOCKS) ++shift;
  blocks = 0;
  for (int64_t s = 0; s < n_series; ++s) {
    const int64_t n = offsets[s + 1] - offsets[s];
    const int64_t n_sub = n >= m ? n - m + 1 : 0;
    const int32_t nblk = (int32_t)((n_sub + (1ll << shift) - 1) >> shift);
    if (ds) {
      ds[s].col = offsets[s];
      ds[s].n_sub = n_sub;
      ds[s].blk_base = blocks;
      ds[s].nblk = nblk;
      ds[s].pad_ = 0;
    }
    blocks += nblk;
  }
  return shift;
}

// ------------------------------------------- allocation-free variant's scratch
// top_discords_noalloc keeps its intermediate arrays (series table, A, G and
// the block maxima) in one file-scope device array instead of a workspace.
// Limits: at most NA_MAX_SERIES series and NA_MAX_SAMPLES samples in total.
// The series table reaches the device as a kernel argument (no host table, no
// pinned staging), so the call allocates nothing.
constexpr int NA_MAX_SERIES = 64;
constexpr int64_t NA_MAX_SAMPLES = int64_t(1) << 21;
// blocks <= sum over series of ceil(n_sub / 256) <= N / 256 + n_series
constexpr int64_t NA_MAX_BLOCKS = (NA_MAX_SAMPLES >> DISC_BLK_MIN_SHIFT) + NA_MAX_SERIES;
constexpr size_t na_round(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t NA_OFF_A = na_round(sizeof(DiscSeries) * NA_MAX_SERIES);
constexpr size_t NA_OFF_G = NA_OFF_A + na_round(sizeof(double) * NA_MAX_SAMPLES);
constexpr size_t NA_OFF_BVAL = NA_OFF_G + na_round(sizeof(int32_t) * NA_MAX_SAMPLES);
constexpr size_t NA_OFF_BIDX = NA_OFF_BVAL + na_round(sizeof(double) * NA_MAX_BLOCKS);
constexpr size_t NA_OFF_BGRP = NA_OFF_BIDX + na_round(sizeof(int32_t) * NA_MAX_BLOCKS);
constexpr size_t NA_SCRATCH_BYTES = NA_OFF_BGRP + na_round(sizeof(int8_t) * NA_MAX_BLOCKS);

static __device__ __align__(256) unsigned char scratch[NA_SCRATCH_BYTES];

struct DiscTable {
  DiscSeries s[NA_MAX_SERIES];
};

__global__ __launch_bounds__(64) void disc_table_kernel(DiscTable tab, int n_series, DiscSeries* dst) {
  for (int s = threadIdx.x; s < n_series; s += 64) dst[s] = tab.s[s];
}

// Device address of ``scratch`` on the current device, looked up once per
// device (each device holds its own copy of the array).
static int noalloc_scratch(unsigned char** out) {
  constexpr int MAX_DEV = 64;
  static std::mutex mu;
  static unsigned char* addr[MAX_DEV] = {};
  int dev = 0;
  SKMP_CHECK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEV) {
    set_error("device index out of range for the allocation-free scratch table");
    return SKMP_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    SKMP_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    addr[dev] = static_cast<unsigned char*>(p);
  }
  *out = addr[dev];
  return SKMP_OK;
}

}  // namespace skmp

using namespace skmp;

extern "C" size_t top_discords_workspace(int64_t n_series, const int64_t* offsets, int32_t k, int32_t m) {
  (void)k;
  if (n_series < 1 || !offsets || m < 1) return 0;
  int64_t blocks;
  disc_plan(n_series, offsets, m, nullptr, blocks);
  Carve cv(nullptr, 0);
  cv.take<DiscSeries>(n_series);
  cv.take<double>(offsets[n_series]);
  cv.take<int32_t>(offsets[n_series]);
  cv.take<double>(blocks);
  cv.take<int32_t>(blocks);
  cv.take<int8_t>(blocks);
  return cv.used + 256;
}

// Argument checks shared by both entry points.
static int disc_validate(const double* P, int64_t ldp, int64_t n_series, const int64_t* offsets, int32_t k, int32_t m,
                         int32_t top_k, int32_t halfwidth, const int64_t* idx, const int32_t* group,
                         const double* score, const int32_t* n_found) {
  SKMP_REQUIRE(P && offsets && idx && group && score && n_found, "null pointer argument");
  SKMP_REQUIRE(n_series >= 1 && n_series < (1 << 30), "n_series out of range");
  SKMP_REQUIRE(k >= 1 && k <= MAX_GROUPS, "k must lie in [1, 128]");
  SKMP_REQUIRE(m >= 1, "m must be >= 1");
  SKMP_REQUIRE(top_k >= 1 && top_k <= MAX_TOPK, "top_k must lie in [1, 256]");
  SKMP_REQUIRE(halfwidth >= 0, "halfwidth must be >= 0");
  SKMP_REQUIRE(offsets[0] == 0, "offsets[0] must be 0");
  for (int64_t s = 0; s < n_series; ++s) SKMP_REQUIRE(offsets[s + 1] >= offsets[s], "offsets must be non-decreasing");
  for (int64_t s = 0; s < n_series; ++s)
    SKMP_REQUIRE(offsets[s + 1] - offsets[s] < (int64_t)INT_MAX, "series too long");
  SKMP_REQUIRE(ldp >= offsets[n_series], "ldp must be >= the total number of samples");
  return SKMP_OK;
}

// combine + select on arrays already placed (st.ser filled or about to be, in
// stream order).
static int disc_launch(const double* P, int64_t ldp, int32_t k, int64_t n_series, int64_t blocks, const DiscState& st,
                       hipStream_t stream_) {
  if (blocks > 0)
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)blocks), dim3(256), 0, stream_, P, ldp, k, st);
  const size_t lds = (size_t)SEL_LDS_BLOCKS * (sizeof(double) + sizeof(int) + sizeof(int8_t));
  hipLaunchKernelGGL(select_kernel, dim3((unsigned)n_series), dim3(SEL_THREADS), lds, stream_, st);
  SKMP_CHECK_HIP(hipGetLastError());
  return SKMP_OK;
}

extern "C" int top_discords(const double* P, int64_t ldp, int64_t n_series, const int64_t* offsets, int32_t k,
                            int32_t m, int32_t top_k, int32_t halfwidth, int64_t* idx, int32_t* group, double* score,
                            int32_t* n_found, void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  if (int rc = disc_validate(P, ldp, n_series, offsets, k, m, top_k, halfwidth, idx, group, score, n_found)) return rc;
  const int64_t N = offsets[n_series];
  std::vector<DiscSeries> ds(n_series);
  int64_t blocks;
  const int shift = disc_plan(n_series, offsets, m, ds.data(), blocks);
  Carve cv(workspace, ws_bytes);
  DiscSeries* ser = cv.take<DiscSeries>(n_series);
  DiscState st;
  st.ser = ser;
  st.n_series = (int)n_series;
  st.top_k = top_k;
  st.halfwidth = halfwidth > 0 ? halfwidth : m;
  st.shift = shift;
  st.total_blocks = blocks;
  st.A = cv.take<double>(N);
  st.G = cv.take<int32_t>(N);
  st.bval = cv.take<double>(blocks);
  st.bidx = cv.take<int32_t>(blocks);
  st.bgrp = cv.take<int8_t>(blocks);
  st.idx = idx;
  st.group = group;
  st.score = score;
  st.n_found = n_found;
  if (!workspace || !cv.fits()) {
    set_error("workspace too small: need " + std::to_string(cv.used) + " bytes");
    return SKMP_ENOMEM;
  }
  hipStream_t stream_ = static_cast<hipStream_t>(stream);
  if (int rc = upload_async(ser, ds.data(), sizeof(DiscSeries) * n_series, stream_)) return rc;
  StageTimer tm(SKMP_TIMER_DISCORDS, stream_);
  return disc_launch(P, ldp, k, n_series, blocks, st, stream_);
}

extern "C" int top_discords_noalloc(const double* P, int64_t ldp, int64_t n_series, const int64_t* offsets, int32_t k,
                                    int32_t m, int32_t top_k, int32_t halfwidth, int64_t* idx, int32_t* group,
                                    double* score, int32_t* n_found, void* stream) {
  clear_error();
  if (int rc = disc_validate(P, ldp, n_series, offsets, k, m, top_k, halfwidth, idx, group, score, n_found)) return rc;
  SKMP_REQUIRE(n_series <= NA_MAX_SERIES, "top_discords_noalloc: more than 64 series");
  const int64_t N = offsets[n_series];
  SKMP_REQUIRE(N <= NA_MAX_SAMPLES, "top_discords_noalloc: more than 2^21 samples in total");
  DiscTable tab;
  int64_t blocks;
  const int shift = disc_plan(n_series, offsets, m, tab.s, blocks);
  unsigned char* base = nullptr;
  if (int rc = noalloc_scratch(&base)) return rc;
  DiscState st;
  st.ser = reinterpret_cast<DiscSeries*>(base);
  st.n_series = (int)n_series;
  st.top_k = top_k;
  st.halfwidth = halfwidth > 0 ? halfwidth : m;
  st.shift = shift;
  st.total_blocks = blocks;
  st.A = reinterpret_cast<double*>(base + NA_OFF_A);
  st.G = reinterpret_cast<int32_t*>(base + NA_OFF_G);
  st.bval = reinterpret_cast<double*>(base + NA_OFF_BVAL);
  st.bidx = reinterpret_cast<int32_t*>(base + NA_OFF_BIDX);
  st.bgrp = reinterpret_cast<int8_t*>(base + NA_OFF_BGRP);
  st.idx = idx;
  st.group = group;
  st.score = score;
  st.n_found = n_found;
  hipStream_t stream_ = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(disc_table_kernel, dim3(1), dim3(64), 0, stream_, tab, (int)n_series,
                     reinterpret_cast<DiscSeries*>(base));
  return disc_launch(P, ldp, k, n_series, blocks, st, stream_);
}
