// Discord time detection over the k sketched profiles (paper Algorithm 2) and
// the ordered list of non-overlapping discords (Sections IV-B and IV-C).
//
//   combine:  A[i] = max over groups of P[g][i] with the first group kept on
//             ties (Algorithm 2 replaces its best only on a strictly larger
//             score); non-finite scores (no admissible neighbour) are dropped.
//   select:   one 1024-thread block per series runs all K greedy passes: each
//             pass takes the first maximum of A among windows not masked by
//             earlier picks (kept in LDS); a pick masks |i - i*| < halfwidth.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "skmp_common.hpp"

namespace skmp {

constexpr int DISC_CHUNK = 1 << 16;
constexpr int DISC_THREADS = 256;

struct DiscSeries {
  int64_t col;
  int64_t n_sub;       // 0 if the series is shorter than m
  int64_t chunk_base;  // first chunk of this series
};

struct DiscState {
  const DiscSeries* ser;
  int n_series;
  int top_k;
  int halfwidth;
  double* A;
  int32_t* G;
  double* cand_val;     // per chunk
  int64_t* cand_idx;
  int64_t* idx;         // outputs
  int32_t* group;
  double* score;
  int32_t* n_found;
};

__device__ __forceinline__ bool better(double v, int64_t i, double bv, int64_t bi) {
  return v > bv || (v == bv && i < bi);
}

__global__ __launch_bounds__(256) void combine_kernel(const double* __restrict__ P, int64_t ldp, int k,
                                                      const DiscSeries* __restrict__ ser, int n_series, int64_t N,
                                                      double* __restrict__ A, int32_t* __restrict__ G) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  int lo = 0, hi = n_series - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (ser[mid].col <= t) lo = mid; else hi = mid - 1;
  }
  const int64_t i = t - ser[lo].col;
  double best = -INFINITY;
  int32_t bg = -1;
  if (i < ser[lo].n_sub) {
    for (int g = 0; g < k; ++g) {
      const double v = P[(int64_t)g * ldp + t];
      if (isfinite(v) && v > best) {
        best = v;
        bg = g;
      }
    }
  }
  A[t] = best;
  G[t] = bg;
}

constexpr int SEL_THREADS = 1024;
constexpr int MAX_TOPK = 256;

__global__ __launch_bounds__(SEL_THREADS) void select_kernel(DiscState st) {
  __shared__ int64_t picks[MAX_TOPK];
  __shared__ double wv[SEL_THREADS / 64];
  __shared__ int64_t wi[SEL_THREADS / 64];
  const int s = blockIdx.x;
  const DiscSeries sr = st.ser[s];
  const double* A = st.A + sr.col;
  const int64_t h = st.halfwidth;
  int found = 0;
  for (int pass = 0; pass < st.top_k; ++pass) {
    double v = -INFINITY;
    int64_t bi = INT64_MAX;
    for (int64_t i = threadIdx.x; i < sr.n_sub; i += SEL_THREADS) {
      const double x = A[i];
      if (!(x > -INFINITY) || !better(x, i, v, bi)) continue;
      bool masked = false;
      for (int q = 0; q < pass; ++q) {
        const int64_t p = picks[q];
        masked |= (i - p < h) && (p - i < h);
      }
      if (!masked) {
        v = x;
        bi = i;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_down(v, off);
      const int64_t oi = __shfl_down(bi, off);
      if (better(ov, oi, v, bi)) {
        v = ov;
        bi = oi;
      }
    }
    if ((threadIdx.x & 63) == 0) {
      wv[threadIdx.x >> 6] = v;
      wi[threadIdx.x >> 6] = bi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 1; q < SEL_THREADS / 64; ++q)
        if (better(wv[q], wi[q], v, bi)) {
          v = wv[q];
          bi = wi[q];
        }
      const int64_t o = (int64_t)s * st.top_k + pass;
      if (v > -INFINITY) {
        st.idx[o] = bi;
        st.group[o] = st.G[sr.col + bi];
        st.score[o] = v;
        picks[pass] = bi;
      } else {
        picks[pass] = INT64_MIN / 2;  // nothing left: masks nothing
      }
      wv[0] = v;
    }
    __syncthreads();
    if (!(wv[0] > -INFINITY)) break;
    found = pass + 1;
    __syncthreads();
  }
  if (threadIdx.x == 0) st.n_found[s] = found;
}

__global__ void init_outputs(DiscState st) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)st.n_series * st.top_k;
  if (t < total) {
    st.idx[t] = -1;
    st.group[t] = -1;
    st.score[t] = __longlong_as_double(0x7FF8000000000000ll);
  }
  if (t < st.n_series) st.n_found[t] = 0;
}

static void disc_plan(int64_t n_series, const int64_t* offsets, int32_t m, std::vector<DiscSeries>& ds,
                      int64_t& chunks) {
  ds.resize(n_series);
  chunks = 0;
  for (int64_t s = 0; s < n_series; ++s) {
    const int64_t n = offsets[s + 1] - offsets[s];
    ds[s].col = offsets[s];
    ds[s].n_sub = n >= m ? n - m + 1 : 0;
    ds[s].chunk_base = chunks;
    chunks += std::max<int64_t>(1, (ds[s].n_sub + DISC_CHUNK - 1) / DISC_CHUNK);
  }
}

}  // namespace skmp

using namespace skmp;

extern "C" size_t top_discords_workspace(int64_t n_series, const int64_t* offsets, int32_t k, int32_t m) {
  (void)k;
  if (n_series < 1 || !offsets || m < 1) return 0;
  std::vector<DiscSeries> ds;
  int64_t chunks;
  disc_plan(n_series, offsets, m, ds, chunks);
  Carve cv(nullptr, 0);
  cv.take<DiscSeries>(n_series);
  cv.take<double>(offsets[n_series]);
  cv.take<int32_t>(offsets[n_series]);
  cv.take<double>(chunks);
  cv.take<int64_t>(chunks);
  return cv.used + 256;
}

extern "C" int top_discords(const double* P, int64_t ldp, int64_t n_series, const int64_t* offsets, int32_t k,
                            int32_t m, int32_t top_k, int32_t halfwidth, int64_t* idx, int32_t* group, double* score,
                            int32_t* n_found, void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  SKMP_REQUIRE(P && offsets && idx && group && score && n_found, "null pointer argument");
  SKMP_REQUIRE(n_series >= 1 && n_series < (1 << 30), "n_series out of range");
  SKMP_REQUIRE(k >= 1 && k <= 64, "k must lie in [1, 64]");
  SKMP_REQUIRE(m >= 1, "m must be >= 1");
  SKMP_REQUIRE(top_k >= 1 && top_k <= MAX_TOPK, "top_k must lie in [1, 256]");
  SKMP_REQUIRE(halfwidth >= 0, "halfwidth must be >= 0");
  SKMP_REQUIRE(offsets[0] == 0, "offsets[0] must be 0");
  for (int64_t s = 0; s < n_series; ++s) SKMP_REQUIRE(offsets[s + 1] >= offsets[s], "offsets must be non-decreasing");
  const int64_t N = offsets[n_series];
  SKMP_REQUIRE(ldp >= N, "ldp must be >= the total number of samples");
  std::vector<DiscSeries> ds;
  int64_t chunks;
  disc_plan(n_series, offsets, m, ds, chunks);
  Carve cv(workspace, ws_bytes);
  DiscSeries* ser = cv.take<DiscSeries>(n_series);
  DiscState st;
  st.ser = ser;
  st.n_series = (int)n_series;
  st.top_k = top_k;
  st.halfwidth = halfwidth > 0 ? halfwidth : m;
  st.A = cv.take<double>(N);
  st.G = cv.take<int32_t>(N);
  st.cand_val = cv.take<double>(chunks);
  st.cand_idx = cv.take<int64_t>(chunks);
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
  const int64_t outs = std::max<int64_t>(n_series * top_k, n_series);
  hipLaunchKernelGGL(init_outputs, dim3((unsigned)((outs + 255) / 256)), dim3(256), 0, stream_, st);
  if (N > 0)
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, stream_, P, ldp, k, ser,
                       (int)n_series, N, st.A, st.G);
  hipLaunchKernelGGL(select_kernel, dim3((unsigned)n_series), dim3(SEL_THREADS), 0, stream_, st);
  SKMP_CHECK_HIP(hipGetLastError());
  return SKMP_OK;
}
