// Normalise + sketch (paper Section III-A, Algorithm 1) and the add/delete
// dimension update (Section III-C).
//
// Two streaming passes over T, both coalesced along time:
//   dimstats:  per (series, dimension) mean and population sigma.  Each block
//              reduces one 64K-sample chunk with a shifted sum (shift = the
//              chunk's first value); chunk partials (n, mean, M2) are merged in
//              order with Chan's pairwise update.
//   project:   a wave owns 64 V consecutive time columns, walks the
//              dimensions of its slice, normalises each value and accumulates
//              k sketch rows in FP64:
//              R[g][t] = sum_j S[g][j] * (T[j][t] - mu_j) / sigma_j.
// The coefficient matrix S is a pure function of (kind, k, seed, dimension
// id), so an update regenerates exactly the columns it needs.  Count and sum
// coefficients (integer hashing) are drawn on the device straight into the
// projection's table; Gaussian ones on the host (glibc libm) and copied.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "skmp_common.hpp"

namespace skmp {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

// ------------------------------------------------------- coefficient draw
static inline uint64_t splitmix64_output(uint64_t state, uint64_t i) {
  uint64_t z = state + i * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static constexpr uint64_t P61 = (1ull << 61) - 1;

static inline uint64_t mulmod61(uint64_t a, uint64_t x) {
  unsigned __int128 p = (unsigned __int128)a * x;
  uint64_t lo = (uint64_t)(p & P61), hi = (uint64_t)(p >> 61);
  uint64_t s = lo + hi;  // 2^61 = 1 (mod p)
  s = (s & P61) + (s >> 61);
  if (s >= P61) s -= P61;
  return s;
}

// Carter-Wegman parameters of the count sketch's hash pair: (a, b) for the
// bucket h, (a2, b2) for the sign s, from SplitMix64(seed) outputs 1..4.
static void count_params(uint64_t seed, uint64_t* a, uint64_t* b, uint64_t* a2, uint64_t* b2) {
  *a = 1 + splitmix64_output(seed, 1) % (P61 - 1);
  *b = splitmix64_output(seed, 2) % P61;
  *a2 = 1 + splitmix64_output(seed, 3) % (P61 - 1);
  *b2 = splitmix64_output(seed, 4) % P61;
}

static int check_ids(const int64_t* ids, int64_t d) {
  for (int64_t j = 0; j < d; ++j) {
    int64_t id = ids ? ids[j] : j;
    SKMP_REQUIRE(id >= 0 && (uint64_t)id < P61, "dimension ids must lie in [0, 2^61 - 1)");
  }
  return SKMP_OK;
}

int launch_sketch_coeffs_host(int32_t kind, int32_t k, uint64_t seed, const int64_t* ids, int64_t d, double* S) {
  SKMP_REQUIRE(k >= 1 && k <= MAX_GROUPS, "k must lie in [1, 128]");
  // the Gaussian draws are keyed by id * 64 + g: at most 64 groups
  SKMP_REQUIRE(kind != SKMP_GAUSS || k <= 64, "the Gaussian sketch has at most 64 groups");
  SKMP_REQUIRE(d >= 1, "d must be >= 1");
  SKMP_REQUIRE(S != nullptr, "S is NULL");
  SKMP_REQUIRE(kind == SKMP_SUM || kind == SKMP_COUNT || kind == SKMP_GAUSS, "unknown sketch kind");
  SKMP_REQUIRE(kind != SKMP_SUM || k == 1, "the sum sketch has k = 1");
  if (int rc = check_ids(ids, d)) return rc;
  std::memset(S, 0, sizeof(double) * (size_t)k * (size_t)d);
  if (kind == SKMP_SUM) {
    for (int64_t j = 0; j < d; ++j) S[j] = 1.0;
    return SKMP_OK;
  }
  if (kind == SKMP_COUNT) {
    uint64_t a, b, a2, b2;
    count_params(seed, &a, &b, &a2, &b2);
    for (int64_t j = 0; j < d; ++j) {
      uint64_t id = (uint64_t)(ids ? ids[j] : j);
      uint64_t hv = mulmod61(a, id) + b;
      if (hv >= P61) hv -= P61;
      uint64_t sv = mulmod61(a2, id) + b2;
      if (sv >= P61) sv -= P61;
      int g = (int)(hv % (uint64_t)k);
      S[(int64_t)g * d + j] = (sv & 1) ? -1.0 : 1.0;
    }
    return SKMP_OK;
  }
  const double two_pi = 2.0 * M_PI;
  for (int64_t j = 0; j < d; ++j) {
    uint64_t id = (uint64_t)(ids ? ids[j] : j);
    for (int g = 0; g < k; ++g) {
      uint64_t c = 2 * (id * 64 + (uint64_t)g);
      uint64_t o1 = splitmix64_output(seed, c + 1), o2 = splitmix64_output(seed, c + 2);
      double u1 = (double)((o1 >> 11) + 1) * 0x1.0p-53;
      double u2 = (double)(o2 >> 11) * 0x1.0p-53;
      S[(int64_t)g * d + j] = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
    }
  }
  return SKMP_OK;
}

// ------------------------------------------------------------- kernels
constexpr int STAT_CHUNK = 1 << 13;
constexpr int STAT_THREADS = 256;

__global__ void fill_u32(unsigned int* p, unsigned int v, int64_t count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// (a x) mod (2^61 - 1) from the 128-bit product: a x = hi 2^64 + lo and
// 2^64 = 8 (mod 2^61 - 1); fully reduced, so it equals the host's value.
__device__ __forceinline__ uint64_t mulmod61_dev(uint64_t a, uint64_t x) {
  const uint64_t lo = a * x, hi = __umul64hi(a, x);
  uint64_t s = (lo & P61) + (lo >> 61) + (hi << 3);
  s = (s & P61) + (s >> 61);
  if (s >= P61) s -= P61;
  return s;
}

// Count or sum sketch coefficients straight into the projection's transposed
// table St[j][g] (kb groups per row, zero past k): the hash pair of the host
// generator (Section III-A), evaluated per dimension, so no table crosses PCIe.
// Only groups [g0, g0 + kb) are written (a sketch of more than 64 groups is
// projected in blocks of 64).
__global__ void count_coeffs_kernel(double* __restrict__ St, int64_t d, int kb, int k, int kind,
                                    const int64_t* __restrict__ ids, uint64_t a, uint64_t b, uint64_t a2,
                                    uint64_t b2, int g0) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  double* row = St + j * kb;
  for (int g = 0; g < kb; ++g) row[g] = 0.0;
  if (kind == SKMP_SUM) {
    row[0] = 1.0;
    return;
  }
  const uint64_t id = ids ? (uint64_t)ids[j] : (uint64_t)j;
  uint64_t hv = mulmod61_dev(a, id) + b;
  if (hv >= P61) hv -= P61;
  uint64_t sv = mulmod61_dev(a2, id) + b2;
  if (sv >= P61) sv -= P61;
  const int g = (int)(hv % (uint64_t)k) - g0;
  if (g >= 0 && g < kb) row[g] = (sv & 1) ? -1.0 : 1.0;
}

struct StatPartial {
  double n, mean, m2, maxabs;
  double bad;  // non-finite values in the chunk
};

template <typename TIn>
__global__ __launch_bounds__(STAT_THREADS) void dimstats_partial(const TIn* __restrict__ T, int64_t ldt, int64_t d,
                                                                 const int64_t* __restrict__ offsets,
                                                                 const int64_t* __restrict__ cprefix, int n_series,
                                                                 StatPartial* __restrict__ part,
                                                                 unsigned int* __restrict__ nonfinite) {
  const int64_t total_chunks = cprefix[n_series];
  const int64_t bid = blockIdx.x;
  const int64_t j = bid / total_chunks;
  const int64_t c = bid - j * total_chunks;
  // series of chunk c
  int lo = 0, hi = n_series - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (cprefix[mid] <= c) lo = mid; else hi = mid - 1;
  }
  const int s = lo;
  const int64_t a = offsets[s] + (c - cprefix[s]) * (int64_t)STAT_CHUNK;
  const int64_t b = min(a + (int64_t)STAT_CHUNK, offsets[s + 1]);
  const TIn* row = T + j * ldt;
  const double shift = (double)row[a];
  double s1 = 0.0, s2 = 0.0, mx = 0.0;
  unsigned int bad = 0;
#pragma unroll 8
  for (int64_t t = a + threadIdx.x; t < b; t += STAT_THREADS) {
    double x = (double)row[t];
    bad += isfinite(x) ? 0u : 1u;
    double e = x - shift;
    s1 += e;
    s2 = fma(e, e, s2);
    mx = fmax(mx, fabs(x));
  }
  __shared__ double sh1[STAT_THREADS / 64], sh2[STAT_THREADS / 64], shm[STAT_THREADS / 64];
  __shared__ unsigned int shb[STAT_THREADS / 64];
  for (int off = 32; off > 0; off >>= 1) {
    s1 += __shfl_down(s1, off);
    s2 += __shfl_down(s2, off);
    mx = fmax(mx, __shfl_down(mx, off));
    bad += __shfl_down(bad, off);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh1[w] = s1;
    sh2[w] = s2;
    shm[w] = mx;
    shb[w] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t1 = 0.0, t2 = 0.0, tm = 0.0;
    unsigned int tb = 0;
    for (int q = 0; q < STAT_THREADS / 64; ++q) {
      t1 += sh1[q];
      t2 += sh2[q];
      tm = fmax(tm, shm[q]);
      tb += shb[q];
    }
    double cnt = (double)(b - a);
    StatPartial p;
    p.n = cnt;
    p.mean = shift + t1 / cnt;
    p.m2 = fmax(t2 - t1 * (t1 / cnt), 0.0);
    p.maxabs = tm;
    p.bad = (double)tb;
    part[bid] = p;
    if (tb && nonfinite) atomicAdd(nonfinite, tb);
  }
}

__global__ void dimstats_finalize(const StatPartial* __restrict__ part, const int64_t* __restrict__ cprefix,
                                  int n_series, int64_t d, double* __restrict__ stats) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // (s, j)
  if (idx >= (int64_t)n_series * d) return;
  const int s = (int)(idx / d);
  const int64_t j = idx - (int64_t)s * d;
  const int64_t total_chunks = cprefix[n_series];
  double n = 0.0, mean = 0.0, m2 = 0.0, mx = 0.0, bad = 0.0;
  for (int64_t c = cprefix[s]; c < cprefix[s + 1]; ++c) {
    StatPartial p = part[j * total_chunks + c];
    double nn = n + p.n;
    double delta = p.mean - mean;
    mean += delta * (p.n / nn);
    m2 += p.m2 + delta * delta * (n * p.n / nn);
    n = nn;
    mx = fmax(mx, p.maxabs);
    bad += p.bad;
  }
  double sd = sqrt(m2 / n);
  // a dimension whose sigma is negligible against its magnitude is constant
  if (sd <= FLAT_REL * mx) sd = 0.0;
  if (bad > 0.0) {
    // a dimension holding NaN or Inf has no statistics: (NaN, NaN) marks it,
    // and its NaN coefficient makes the series' sketch NaN (never a silent 0)
    mean = __longlong_as_double(0x7FF8000000000000ll);
    sd = mean;
  }
  stats[idx * 2 + 0] = mean;
  stats[idx * 2 + 1] = sd;
}

// R[g][t] (mode 0: =, +1: +=, -1: -=) sum_j S[g][j] (T[j][t] - mu_j) / sigma_j
// (Algorithm 1; sigma_j = 0 marks a constant dimension, which contributes 0).
//
// A wave owns a tile of 64 V consecutive columns (V per lane, one 8- or
// 16-byte load per row) and walks the rows of its slice of the dimensions
// (SL waves per block split d; their partial sums meet in LDS in a fixed
// order, so results are reproducible bit for bit).  PROJ_PF rows are loaded
// before any is used.  The coefficients are stored transposed and padded to
// KB groups (St[j][g], zero past k), so one row's coefficients are one
// contiguous uniform read (scalar loads, SGPR operands of the FMAs) and the
// inner loops carry no guards.  (mu, 1/sigma) per (series, dimension) comes
// from coef.  A block walks tiles_per_block consecutive tiles; the series of a
// tile is found by a wave-wide 64-ary search and kept while the tiles stay
// inside it.  Tiles that straddle a series boundary or the end of the data
// take a per-column path.
constexpr int PROJ_PF = 8;
constexpr int PROJ_LDS_BYTES = 48 * 1024;

// The series s with offsets[s] <= c < offsets[s + 1], by all 64 lanes of a
// wave (c uniform, 0 <= c < offsets[n_series]): every round probes 64 evenly
// spaced entries and keeps the span between the last probe <= c and the next.
__device__ __forceinline__ int series_of(const int64_t* __restrict__ offsets, int n_series, int64_t c, int lane) {
  int lo = 0, hi = n_series - 1;
  while (hi > lo) {
    const int step = (hi - lo + 64) / 64;
    const int p = lo + lane * step;
    const bool le = p <= hi && offsets[p] <= c;
    const unsigned long long b = __ballot(le);  // a prefix of the lanes (offsets increase); lane 0 always
    const int L = 64 - __clzll(b);
    lo = lo + (L - 1) * step;
    hi = min(hi, lo + step - 1);
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// Per-lane binary search (columns of a tile that straddles a series boundary).
__device__ __forceinline__ int series_of_lane(const int64_t* __restrict__ offsets, int n_series, int64_t c) {
  int lo = 0, hi = n_series - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (offsets[mid] <= c) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename TIn, int V>
__device__ __forceinline__ void load_cols(const TIn* __restrict__ p, TIn (&x)[V]) {
  static_assert(V == 1 || sizeof(TIn) * V == 8 || sizeof(TIn) * V == 16, "8- or 16-byte column groups");
  if constexpr (V == 1) {
    x[0] = p[0];
  } else if constexpr (sizeof(TIn) * V == 8) {
    const float2 q = *reinterpret_cast<const float2*>(p);
    x[0] = q.x;
    x[1] = q.y;
  } else if constexpr (sizeof(TIn) == 4) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    x[0] = q.x;
    x[1] = q.y;
    x[2] = q.z;
    x[3] = q.w;
  } else {
    const double2 q = *reinterpret_cast<const double2*>(p);
    x[0] = q.x;
    x[1] = q.y;
  }
}

// Rows [j0, j1) of a full tile inside one series: cu = that series' coef row (uniform).
template <typename TIn, int KB, int V>
__device__ __forceinline__ void rows_uniform(const TIn* __restrict__ T, int64_t ldt, int j0, int j1, int64_t t,
                                             const double* __restrict__ cu, const double* __restrict__ St,
                                             double (&acc)[KB][V]) {
  int j = j0;
  for (; j + PROJ_PF <= j1; j += PROJ_PF) {
    TIn x[PROJ_PF][V];
#pragma unroll
    for (int u = 0; u < PROJ_PF; ++u) load_cols<TIn, V>(T + (int64_t)(j + u) * ldt + t, x[u]);
#pragma unroll
    for (int u = 0; u < PROJ_PF; ++u) {
      const double mu = cu[2 * (j + u)], is = cu[2 * (j + u) + 1];
      const double* __restrict__ sr = St + (int64_t)(j + u) * KB;
      double xb[V];
#pragma unroll
      for (int v = 0; v < V; ++v) xb[v] = ((double)x[u][v] - mu) * is;
#pragma unroll
      for (int g = 0; g < KB; ++g) {
        const double c = sr[g];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[g][v] = fma(c, xb[v], acc[g][v]);
      }
    }
  }
  for (; j < j1; ++j) {
    TIn x[V];
    load_cols<TIn, V>(T + (int64_t)j * ldt + t, x);
    const double mu = cu[2 * j], is = cu[2 * j + 1];
    const double* __restrict__ sr = St + (int64_t)j * KB;
#pragma unroll
    for (int g = 0; g < KB; ++g) {
      const double c = sr[g];
#pragma unroll
      for (int v = 0; v < V; ++v) acc[g][v] = fma(c, ((double)x[v] - mu) * is, acc[g][v]);
    }
  }
}

// Rows [j0, j1) for columns t + v that may lie past N or in different series.
template <typename TIn, int KB, int V>
__device__ __forceinline__ void rows_general(const TIn* __restrict__ T, int64_t ldt, int64_t d, int j0, int j1,
                                             int64_t t, int64_t N, const int64_t* __restrict__ offsets,
                                             int n_series, const double* __restrict__ coef,
                                             const double* __restrict__ St, double (&acc)[KB][V]) {
  const double* cp[V];
  bool ok[V];
  int64_t cc[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    ok[v] = t + v < N;
    cc[v] = ok[v] ? t + v : N - 1;
    cp[v] = coef + (int64_t)series_of_lane(offsets, n_series, cc[v]) * d * 2;
  }
  for (int j = j0; j < j1; ++j) {
    const double* __restrict__ sr = St + (int64_t)j * KB;
    double xb[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double x = (double)T[(int64_t)j * ldt + cc[v]];
      xb[v] = ok[v] ? (x - cp[v][2 * j]) * cp[v][2 * j + 1] : 0.0;
    }
#pragma unroll
    for (int g = 0; g < KB; ++g) {
      const double c = sr[g];
#pragma unroll
      for (int v = 0; v < V; ++v) acc[g][v] = fma(c, xb[v], acc[g][v]);
    }
  }
}

template <typename TIn, int KB, int V>
__global__ __launch_bounds__(256) void project_kernel(const TIn* __restrict__ T, int64_t ldt, int64_t d, int64_t N,
                                                      const int64_t* __restrict__ offsets, int n_series,
                                                      const double* __restrict__ coef, const double* __restrict__ St,
                                                      int k, double* __restrict__ R, int64_t ldr, int mode,
                                                      int64_t tiles_per_block, double* __restrict__ dpart,
                                                      const int64_t* __restrict__ oshift) {
  extern __shared__ double part[];  // (SL - 1) x KB x V x 64
  constexpr int TW = 64 * V;
  const int lane = threadIdx.x & 63;
  const int SL = blockDim.x >> 6;
  const int sl = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // the wave's slice of the dimensions
  // the block's chunk of the dimensions (gridDim.y chunks; one unless d is
  // large against the number of column tiles), split among its SL waves
  const int64_t D0 = d * blockIdx.y / gridDim.y, D1 = d * (blockIdx.y + 1) / gridDim.y;
  const int j0 = (int)(D0 + (D1 - D0) * sl / SL), j1 = (int)(D0 + (D1 - D0) * (sl + 1) / SL);
  const int64_t n_tiles = (N + TW - 1) / TW;
  const int64_t tile0 = (int64_t)blockIdx.x * tiles_per_block;
  const int64_t tile1 = min(tile0 + tiles_per_block, n_tiles);
  int s = 0;
  int64_t s_end = -1;  // first column after series s (uniform)
  for (int64_t tile = tile0; tile < tile1; ++tile) {
    const int64_t c0 = tile * TW;
    if (c0 >= s_end) {
      s = series_of(offsets, n_series, c0, lane);
      s_end = offsets[s + 1];
    }
    const int64_t t = c0 + (int64_t)lane * V;
    const bool full = c0 + TW <= s_end;  // a full tile inside series s (s_end <= N)
    double acc[KB][V];
#pragma unroll
    for (int g = 0; g < KB; ++g)
#pragma unroll
      for (int v = 0; v < V; ++v) acc[g][v] = 0.0;
    if (full)
      rows_uniform<TIn, KB, V>(T, ldt, j0, j1, t, coef + (int64_t)s * d * 2, St, acc);
    else
      rows_general<TIn, KB, V>(T, ldt, d, j0, j1, t, N, offsets, n_series, coef, St, acc);
    if (SL > 1) {
      if (sl > 0) {
#pragma unroll
        for (int g = 0; g < KB; ++g)
#pragma unroll
          for (int v = 0; v < V; ++v) part[(((sl - 1) * KB + g) * V + v) * 64 + lane] = acc[g][v];
      }
      __syncthreads();
      if (sl == 0) {
        for (int q = 0; q < SL - 1; ++q)
#pragma unroll
          for (int g = 0; g < KB; ++g)
#pragma unroll
            for (int v = 0; v < V; ++v) acc[g][v] += part[((q * KB + g) * V + v) * 64 + lane];
      }
      __syncthreads();  // part is rewritten by the next tile
    }
    if (sl == 0) {
      // output columns: t + v, moved by the series' shift when one is given
      int64_t oc[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        oc[v] = t + v;
        if (oshift && t + v < N) oc[v] += full ? oshift[s] : oshift[series_of_lane(offsets, n_series, t + v)];
      }
#pragma unroll
      for (int g = 0; g < KB; ++g) {
        if (g < k) {
#pragma unroll
          for (int v = 0; v < V; ++v) {
            if (t + v < N) {
              if (gridDim.y > 1) {  // one chunk's partial sum; project_sum adds the chunks
                dpart[((int64_t)blockIdx.y * KB + g) * N + t + v] = acc[g][v];
              } else {
                double* dst = R + (int64_t)g * ldr + oc[v];
                if (mode == 0) *dst = acc[g][v];
                else if (mode > 0) *dst += acc[g][v];
                else *dst -= acc[g][v];
              }
            }
          }
        }
      }
    }
  }
}

// R[g][t] (=, +=, -=) the sum of the chunks' partial sums, in chunk order.
__global__ void project_sum(const double* __restrict__ dpart, int n_chunks, int kb, int k, int64_t N,
                            double* __restrict__ R, int64_t ldr, int mode, const int64_t* __restrict__ offsets,
                            int n_series, const int64_t* __restrict__ oshift) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)k * N) return;
  const int g = (int)(i / N);
  const int64_t t = i - (int64_t)g * N;
  double acc = 0.0;
  for (int c = 0; c < n_chunks; ++c) acc += dpart[((int64_t)c * kb + g) * N + t];
  double* dst = R + (int64_t)g * ldr + t + (oshift ? oshift[series_of_lane(offsets, n_series, t)] : 0);
  if (mode == 0) *dst = acc;
  else if (mode > 0) *dst += acc;
  else *dst -= acc;
}

__global__ void prep_coef(const double* __restrict__ stats, int64_t pairs, double* __restrict__ coef) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pairs) return;
  const double sd = stats[2 * i + 1];
  coef[2 * i] = stats[2 * i];
  // sigma = 0: a constant dimension, contributes 0; sigma = NaN (non-finite
  // input, or NaN statistics passed in): NaN, so the sketch shows it
  coef[2 * i + 1] = sd > 0.0 ? 1.0 / sd : (sd == 0.0 ? 0.0 : __longlong_as_double(0x7FF8000000000000ll));
}

// Sketch rows padded to the kernel's group count: 1, 4, 8, 16, 32 or 64.
static int proj_kb(int k) { return k <= 1 ? 1 : k <= 4 ? 4 : k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : 64; }

// S [k][d] (row-major) -> St [d][KB], zero for g >= k.
static std::vector<double> transpose_coeffs(const std::vector<double>& S, int k, int64_t d) {
  const int kb = proj_kb(k);
  std::vector<double> St((size_t)d * kb, 0.0);
  for (int g = 0; g < k; ++g)
    for (int64_t j = 0; j < d; ++j) St[(size_t)j * kb + g] = S[(size_t)g * d + j];
  return St;
}

// Columns per lane: 16-byte loads while the lane's accumulators (KB x V
// doubles) stay within 32 doubles; 1 when T's rows are not aligned for them.
template <typename TIn>
static int proj_vec(int kb, const void* T, int64_t ldt) {
  int v = sizeof(TIn) == 8 ? (kb <= 16 ? 2 : 1) : (kb <= 8 ? 4 : kb <= 16 ? 2 : 1);
  while (v > 1 && ((reinterpret_cast<uintptr_t>(T) % (v * sizeof(TIn))) != 0 || ldt % v != 0)) v /= 2;
  return v;
}

// Waves per block (slices of the dimensions) while the column tiles alone leave
// the chip under-filled (4096 waves): each slice at least PROJ_PF rows, the
// partial sums within the LDS budget.
static int proj_slices(int64_t n_tiles, int64_t d, int kb, int v) {
  int SL = 1;
  while (SL < 4 && n_tiles * SL < 4096 && d >= 2 * SL * PROJ_PF &&
         (size_t)(2 * SL - 1) * kb * v * 64 * sizeof(double) <= PROJ_LDS_BYTES)
    SL *= 2;
  return SL;
}

// Chunks of the dimensions across blocks when tiles x slices still leave the
// chip under-filled and there are many dimensions (each chunk >= 32 rows per slice).
static int64_t proj_chunks(int64_t n_tiles, int SL, int64_t d) {
  if (n_tiles * SL >= 4096 || d < 2 * SL * 64) return 1;
  const int64_t c = (4096 + n_tiles * SL - 1) / (n_tiles * SL);
  return std::max<int64_t>(1, std::min<int64_t>(c, d / (SL * 32)));
}

// Workspace doubles for the chunks' partial sums (the most any column-group width needs).
static size_t proj_part_elems(int64_t d, int64_t N, int k) {
  const int kb = proj_kb(k);
  size_t best = 0;
  for (int v : {1, 2, 4}) {
    if ((kb > 16 && v > 1) || (kb == 16 && v > 2)) continue;  // widths proj_vec never picks for this kb
    const int64_t n_tiles = (N + 64 * v - 1) / (64 * v);
    const int64_t nc = proj_chunks(n_tiles, proj_slices(n_tiles, d, kb, v), d);
    if (nc > 1) best = std::max(best, (size_t)nc * kb * (size_t)N);
  }
  return best;
}

template <typename TIn, int KB, int V>
static void launch_project_v(const TIn* T, int64_t ldt, int64_t d, int64_t N, const int64_t* offsets, int n_series,
                             const double* coef, const double* St, int k, double* R, int64_t ldr, int mode,
                             double* dpart, size_t dpart_elems, const int64_t* oshift, hipStream_t st) {
  constexpr int TW = 64 * V;
  const int64_t n_tiles = (N + TW - 1) / TW;
  const int SL = proj_slices(n_tiles, d, KB, V);
  int64_t nc = proj_chunks(n_tiles, SL, d);
  nc = std::min<int64_t>(nc, dpart ? (int64_t)(dpart_elems / ((size_t)KB * (size_t)N)) : 1);
  nc = std::max<int64_t>(nc, 1);
  // at most two blocks per resident slot (8192 waves); more tiles go to each block
  const int64_t max_blocks = std::max<int64_t>(1, 16384 / (SL * nc));
  const int64_t tpb = (n_tiles + max_blocks - 1) / max_blocks;
  const int64_t blocks = (n_tiles + tpb - 1) / tpb;
  const size_t lds = (size_t)(SL - 1) * KB * V * 64 * sizeof(double);
  hipLaunchKernelGGL((project_kernel<TIn, KB, V>), dim3((unsigned)blocks, (unsigned)nc), dim3(64 * SL), lds, st, T,
                     ldt, d, N, offsets, n_series, coef, St, k, R, ldr, mode, tpb, dpart, oshift);
  if (nc > 1)
    hipLaunchKernelGGL(project_sum, dim3((unsigned)(((int64_t)k * N + 255) / 256)), dim3(256), 0, st, dpart, (int)nc,
                       KB, k, N, R, ldr, mode, offsets, n_series, oshift);
}

template <typename TIn, int KB>
static void launch_project_kb(const TIn* T, int64_t ldt, int64_t d, int64_t N, const int64_t* offsets, int n_series,
                              const double* coef, const double* St, int k, double* R, int64_t ldr, int mode,
                              double* dpart, size_t dpart_elems, const int64_t* oshift, hipStream_t st) {
  const int v = proj_vec<TIn>(KB, T, ldt);
  constexpr int VMAX = sizeof(TIn) == 8 ? (KB <= 16 ? 2 : 1) : (KB <= 8 ? 4 : KB <= 16 ? 2 : 1);
  if constexpr (VMAX >= 4) {
    if (v == 4) return launch_project_v<TIn, KB, 4>(T, ldt, d, N, offsets, n_series, coef, St, k, R, ldr, mode, dpart, dpart_elems, oshift, st);
  }
  if constexpr (VMAX >= 2) {
    if (v == 2) return launch_project_v<TIn, KB, 2>(T, ldt, d, N, offsets, n_series, coef, St, k, R, ldr, mode, dpart, dpart_elems, oshift, st);
  }
  launch_project_v<TIn, KB, 1>(T, ldt, d, N, offsets, n_series, coef, St, k, R, ldr, mode, dpart, dpart_elems, oshift, st);
}

// coef: workspace of n_series * d * 2 doubles; St: transpose_coeffs(S) on the device;
// oshift (device, n_series; NULL: none): column t of series s is written to R column t + oshift[s]
template <typename TIn>
static void launch_project(const void* Tv, int64_t ldt, int64_t d, int64_t N, const int64_t* offsets, int n_series,
                           const double* stats, double* coef, const double* St, int k, double* R, int64_t ldr,
                           int mode, double* dpart, size_t dpart_elems, hipStream_t st,
                           const int64_t* oshift = nullptr) {
  const int64_t pairs = (int64_t)n_series * d;
  hipLaunchKernelGGL(prep_coef, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, st, stats, pairs, coef);
  const TIn* T = static_cast<const TIn*>(Tv);
  switch (proj_kb(k)) {
    case 1: return launch_project_kb<TIn, 1>(T, ldt, d, N, offsets, n_series, coef, St, k, R, ldr, mode, dpart, dpart_elems, oshift, st);
    case 4: return launch_project_kb<TIn, 4>(T, ldt, d, N, offsets, n_series, coef, St, k, R, ldr, mode, dpart, dpart_elems, oshift, st);
    case 8: return launch_project_kb<TIn, 8>(T, ldt, d, N, offsets, n_series, coef, St, k, R, ldr, mode, dpart, dpart_elems, oshift, st);
    case 16: return launch_project_kb<TIn, 16>(T, ldt, d, N, offsets, n_series, coef, St, k, R, ldr, mode, dpart, dpart_elems, oshift, st);
    case 32: return launch_project_kb<TIn, 32>(T, ldt, d, N, offsets, n_series, coef, St, k, R, ldr, mode, dpart, dpart_elems, oshift, st);
    default: return launch_project_kb<TIn, 64>(T, ldt, d, N, offsets, n_series, coef, St, k, R, ldr, mode, dpart, dpart_elems, oshift, st);
  }
}

// Per-dimension statistics of the columns [offsets[s], offsets[s+1]) of every series.
struct StatsBuffers {
  int64_t* offsets_dev;  // n_series + 1 (a table of the call's blob)
  int64_t* cprefix_dev;  // n_series + 1 (a table of the call's blob)
  StatPartial* part;
  unsigned int* nonfinite;
};

// The small host tables of one call (series offsets, chunk prefix, sketch
// coefficients) sit next to each other in the workspace and go to the device
// with one copy.  With a null workspace base it only sizes the region.
class TableBlob {
 public:
  explicit TableBlob(Carve& cv) : cv_(cv), begin_(cv.used) {}
  template <typename T>
  T* put(const T* src, size_t count) {
    const size_t off = (cv_.used + 255) & ~size_t(255);
    T* dst = cv_.take<T>(count);
    parts_.push_back({off, src, count * sizeof(T)});
    return dst;
  }
  int upload(hipStream_t st) const {
    const size_t end = parts_.empty() ? begin_ : parts_.back().off + parts_.back().bytes;
    std::vector<unsigned char> host(end - begin_, 0);
    for (const Part& p : parts_)
      if (p.bytes) std::memcpy(host.data() + (p.off - begin_), p.src, p.bytes);
    return host.empty() ? SKMP_OK : upload_async(cv_.base + begin_, host.data(), host.size(), st);
  }

 private:
  struct Part {
    size_t off;
    const void* src;
    size_t bytes;
  };
  Carve& cv_;
  size_t begin_;
  std::vector<Part> parts_;
};

static size_t stats_workspace(int64_t d, int64_t total_chunks, Carve& cv, StatsBuffers* out) {
  StatPartial* part = cv.take<StatPartial>((size_t)d * (size_t)total_chunks);
  unsigned int* nonfinite = cv.take<unsigned int>(64);
  if (out) {
    out->part = part;
    out->nonfinite = nonfinite;
  }
  return cv.used;
}

// Enqueues the statistics pass; the offsets and chunk-prefix tables of b must
// already be on their way (the call's table blob).
static int run_dimstats(const void* T, int32_t dtype, int64_t ldt, int64_t d, int64_t n_series,
                        const std::vector<int64_t>& cpre, const StatsBuffers& b, double* stats_out, bool check,
                        hipStream_t st) {
  if (check && stream_capturing(st)) {
    set_error("the non-finite input check reads its result back on the host and cannot run under graph capture");
    return SKMP_EINVAL;
  }
  if (check) hipLaunchKernelGGL(fill_u32, dim3(1), dim3(64), 0, st, b.nonfinite, 0u, (int64_t)1);
  const int64_t total_chunks = cpre[n_series];
  dim3 grid((unsigned)(d * total_chunks)), block(STAT_THREADS);
  if (dtype == SKMP_F64)
    hipLaunchKernelGGL(dimstats_partial<double>, grid, block, 0, st, static_cast<const double*>(T), ldt, d,
                       b.offsets_dev, b.cprefix_dev, (int)n_series, b.part, check ? b.nonfinite : nullptr);
  else
    hipLaunchKernelGGL(dimstats_partial<float>, grid, block, 0, st, static_cast<const float*>(T), ldt, d,
                       b.offsets_dev, b.cprefix_dev, (int)n_series, b.part, check ? b.nonfinite : nullptr);
  const int64_t pairs = n_series * d;
  hipLaunchKernelGGL(dimstats_finalize, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, st, b.part,
                     b.cprefix_dev, (int)n_series, d, stats_out);
  SKMP_CHECK_HIP(hipGetLastError());
  if (check) {
    unsigned int bad = 0;
    SKMP_CHECK_HIP(hipMemcpyAsync(&bad, b.nonfinite, sizeof(bad), hipMemcpyDeviceToHost, st));
    SKMP_CHECK_HIP(hipStreamSynchronize(st));
    if (bad) {
      set_error("input contains " + std::to_string(bad) + " non-finite values");
      return SKMP_ENONFINITE;
    }
  }
  return SKMP_OK;
}

// Point updates (Section III-C): raising sample t of dimension j of series s
// by delta raises R^(g)_t by S_gj * delta / sigma_sj (sigma = 0: a constant
// dimension, no change).  The host sorts the updates by column, keeping their
// order within a column; thread (segment, g) applies one column's updates in
// that order, so the result is that of applying them one by one.
struct PointUpd {
  int64_t col;    // column of R
  int64_t stat;   // row of the (series, dimension) statistics table
  double delta;   // change of the raw sample
  int64_t crow;   // row of the coefficient table (k values)
};

__global__ void point_update_kernel(double* __restrict__ R, int64_t ldr, int k, int64_t n_seg,
                                    const int64_t* __restrict__ seg, const PointUpd* __restrict__ upd,
                                    const double* __restrict__ coef, const double* __restrict__ stats) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_seg * k) return;
  const int64_t sgm = i / k;
  const int g = (int)(i - sgm * k);
  const int64_t u0 = seg[sgm], u1 = seg[sgm + 1];
  double* dst = R + (int64_t)g * ldr + upd[u0].col;
  double r = *dst;
  for (int64_t u = u0; u < u1; ++u) {
    const PointUpd p = upd[u];
    const double sd = stats[2 * p.stat + 1];
    const double c = coef[p.crow * k + g];
    if (sd > 0.0 && c != 0.0) r += c * (p.delta / sd);
  }
  *dst = r;
}

static std::vector<int64_t> chunk_prefix(int64_t n_series, const int64_t* offsets) {
  std::vector<int64_t> cpre(n_series + 1, 0);
  for (int64_t s = 0; s < n_series; ++s) {
    int64_t L = offsets[s + 1] - offsets[s];
    cpre[s + 1] = cpre[s] + (L + STAT_CHUNK - 1) / STAT_CHUNK;
  }
  return cpre;
}

}  // namespace skmp

using namespace skmp;

extern "C" const char* skmp_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* skmp_version(void) { return "sketchmp 0.1 (gfx950)"; }

extern "C" int sketch_coeffs(int32_t kind, int32_t k, uint64_t seed, const int64_t* dim_ids, int64_t d,
                             double* S_host) {
  clear_error();
  return launch_sketch_coeffs_host(kind, k, seed, dim_ids, d, S_host);
}

// ceil(sqrt(d)) in integers (no rounding of a floating square root), capped at 128
extern "C" int32_t sketch_default_k(int64_t d) {
  clear_error();
  if (d < 1) {
    set_error("d must be >= 1");
    return SKMP_EINVAL;
  }
  int64_t s = 1;
  while (s < MAX_GROUPS && s * s < d) ++s;
  return (int32_t)s;
}

extern "C" size_t sketch_build_workspace(int64_t d, int64_t n_series, const int64_t* offsets, int32_t k) {
  if (d < 1 || n_series < 1 || !offsets || k < 1) return 0;
  std::vector<int64_t> cpre = chunk_prefix(n_series, offsets);
  Carve cv(nullptr, 0);
  TableBlob tb(cv);
  tb.put<int64_t>(nullptr, n_series + 1);
  tb.put<int64_t>(nullptr, n_series + 1);
  const int kc = std::min<int>(k, 64);  // groups per projection pass
  tb.put<double>(nullptr, (size_t)proj_kb(kc) * (size_t)d);
  cv.take<int64_t>((size_t)d);  // dimension ids when the coefficients are drawn on the device
  cv.take<double>((size_t)n_series * (size_t)d * 2);
  cv.take<double>(proj_part_elems(d, offsets[n_series], kc));
  stats_workspace(d, cpre[n_series], cv, nullptr);
  return cv.used + 256;
}

extern "C" int sketch_build(const void* T, int32_t dtype, int64_t d, int64_t ldt, int64_t n_series,
                            const int64_t* offsets, const int64_t* dim_ids, int32_t k, int32_t kind, uint64_t seed,
                            uint32_t flags, double* R, int64_t ldr, double* dim_stats, void* workspace,
                            size_t ws_bytes, void* stream) {
  clear_error();
  SKMP_REQUIRE(T && R && dim_stats && offsets, "null pointer argument");
  SKMP_REQUIRE(dtype == SKMP_F64 || dtype == SKMP_F32, "dtype must be SKMP_F64 or SKMP_F32");
  SKMP_REQUIRE(d >= 1, "d must be >= 1");
  SKMP_REQUIRE(n_series >= 1, "n_series must be >= 1");
  SKMP_REQUIRE(offsets[0] == 0, "offsets[0] must be 0");
  for (int64_t s = 0; s < n_series; ++s)
    SKMP_REQUIRE(offsets[s + 1] > offsets[s], "every series needs at least one sample (offsets strictly increasing)");
  const int64_t N = offsets[n_series];
  SKMP_REQUIRE(ldt >= N && ldr >= N, "row strides must be >= the total number of samples");
  SKMP_REQUIRE(k >= 1 && k <= MAX_GROUPS, "k must lie in [1, 128]");
  // count and sum coefficients are drawn on the device (integer hashing only);
  // Gaussian ones on the host (glibc libm), shipped as a table
  const bool device_coeffs = (kind == SKMP_COUNT || kind == SKMP_SUM);
  SKMP_REQUIRE(kind == SKMP_SUM || kind == SKMP_COUNT || kind == SKMP_GAUSS, "unknown sketch kind");
  SKMP_REQUIRE(kind != SKMP_SUM || k == 1, "the sum sketch has k = 1");
  SKMP_REQUIRE(kind != SKMP_GAUSS || k <= 64, "the Gaussian sketch has at most 64 groups");
  int rc = SKMP_OK;
  std::vector<double> St;
  if (device_coeffs) {
    if ((rc = check_ids(dim_ids, d))) return rc;
  } else {
    std::vector<double> S((size_t)k * (size_t)d);
    if ((rc = launch_sketch_coeffs_host(kind, k, seed, dim_ids, d, S.data()))) return rc;
    St = transpose_coeffs(S, k, d);
  }
  std::vector<int64_t> cpre = chunk_prefix(n_series, offsets);
  Carve cv(workspace, ws_bytes);
  TableBlob tb(cv);
  StatsBuffers sb;
  sb.offsets_dev = tb.put(offsets, n_series + 1);
  sb.cprefix_dev = tb.put(cpre.data(), n_series + 1);
  // more than 64 groups (count sketch): projected in passes of 64 groups
  const int kc = std::min<int>(k, 64);
  const int kb = proj_kb(kc);
  double* S_dev = device_coeffs ? cv.take<double>((size_t)kb * (size_t)d) : tb.put(St.data(), St.size());
  const int64_t* ids_dev = (device_coeffs && dim_ids) ? tb.put(dim_ids, (size_t)d) : nullptr;
  double* coef = cv.take<double>((size_t)n_series * (size_t)d * 2);
  const size_t dpart_elems = proj_part_elems(d, N, kc);
  double* dpart = cv.take<double>(dpart_elems);
  stats_workspace(d, cpre[n_series], cv, &sb);
  if (!workspace || !cv.fits()) {
    set_error("workspace too small: need " + std::to_string(cv.used) + " bytes");
    return SKMP_ENOMEM;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc2 = tb.upload(st)) return rc2;
  StageTimer tm(SKMP_TIMER_SKETCH, st);
  rc = run_dimstats(T, dtype, ldt, d, n_series, cpre, sb, dim_stats, (flags & SKMP_FLAG_CHECK_FINITE) != 0, st);
  if (rc) return rc;
  for (int g0 = 0; g0 < k; g0 += 64) {
    const int kk = std::min(64, k - g0);
    if (device_coeffs) {
      uint64_t a = 0, b = 0, a2 = 0, b2 = 0;
      count_params(seed, &a, &b, &a2, &b2);
      hipLaunchKernelGGL(count_coeffs_kernel, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, st, S_dev, d,
                         proj_kb(kk), k, kind, ids_dev, a, b, a2, b2, g0);
    }
    double* Rg = R + (int64_t)g0 * ldr;
    if (dtype == SKMP_F64)
      launch_project<double>(T, ldt, d, N, sb.offsets_dev, (int)n_series, dim_stats, coef, S_dev, kk, Rg, ldr, 0,
                             dpart, dpart_elems, st);
    else
      launch_project<float>(T, ldt, d, N, sb.offsets_dev, (int)n_series, dim_stats, coef, S_dev, kk, Rg, ldr, 0,
                            dpart, dpart_elems, st);
  }
  SKMP_CHECK_HIP(hipGetLastError());
  return SKMP_OK;
}

extern "C" size_t sketch_update_workspace(int64_t n, int64_t d_add, int64_t d_rem, int32_t k) {
  if (n < 1 || k < 1 || d_add < 0 || d_rem < 0) return 0;
  int64_t offs[2] = {0, n};
  std::vector<int64_t> cpre = chunk_prefix(1, offs);
  Carve cv(nullptr, 0);
  TableBlob tb(cv);
  tb.put<int64_t>(nullptr, 2);
  tb.put<int64_t>(nullptr, 2);
  tb.put<double>(nullptr, (size_t)proj_kb(k) * (size_t)std::max<int64_t>(d_add, 1));
  tb.put<double>(nullptr, (size_t)proj_kb(k) * (size_t)std::max<int64_t>(d_rem, 1));
  cv.take<double>((size_t)std::max<int64_t>(std::max<int64_t>(d_add, d_rem), 1) * 2);
  cv.take<double>(proj_part_elems(std::max<int64_t>(std::max<int64_t>(d_add, d_rem), 1), n, k));
  stats_workspace(std::max<int64_t>(d_add, 1), cpre[1], cv, nullptr);
  return cv.used + 256;
}

extern "C" int sketch_update_dims(double* R, int64_t ldr, int64_t n, int32_t k, int32_t kind, uint64_t seed,
                                  int32_t dtype, int64_t ldt, const void* T_add, int64_t d_add,
                                  const int64_t* add_ids, double* add_stats, const void* T_rem, int64_t d_rem,
                                  const int64_t* rem_ids, const double* rem_stats, uint32_t flags,
                                  uint64_t* changed_groups, void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  SKMP_REQUIRE(R != nullptr, "R is NULL");
  SKMP_REQUIRE(k >= 1 && k <= 64, "k must lie in [1, 64]");
  SKMP_REQUIRE(n >= 1 && ldr >= n && ldt >= n, "bad length or strides");
  SKMP_REQUIRE(dtype == SKMP_F64 || dtype == SKMP_F32, "dtype must be SKMP_F64 or SKMP_F32");
  SKMP_REQUIRE(d_add >= 0 && d_rem >= 0, "negative dimension count");
  SKMP_REQUIRE(d_add == 0 || (T_add && add_ids && add_stats), "added dimensions need T_add, add_ids and add_stats");
  SKMP_REQUIRE(d_rem == 0 || (T_rem && rem_ids && rem_stats), "removed dimensions need T_rem, rem_ids and rem_stats");
  for (int64_t a = 0; a < d_add; ++a)
    for (int64_t b = 0; b < d_rem; ++b)
      SKMP_REQUIRE(add_ids[a] != rem_ids[b], "a dimension id is both added and removed");
  for (int64_t a = 0; a < d_add; ++a)
    for (int64_t b = a + 1; b < d_add; ++b) SKMP_REQUIRE(add_ids[a] != add_ids[b], "duplicate added dimension id");
  for (int64_t a = 0; a < d_rem; ++a)
    for (int64_t b = a + 1; b < d_rem; ++b) SKMP_REQUIRE(rem_ids[a] != rem_ids[b], "duplicate removed dimension id");
  std::vector<double> Sa((size_t)k * (size_t)std::max<int64_t>(d_add, 1)),
      Sr((size_t)k * (size_t)std::max<int64_t>(d_rem, 1));
  int rc;
  if (d_add) {
    rc = launch_sketch_coeffs_host(kind, k, seed, add_ids, d_add, Sa.data());
    if (rc) return rc;
  }
  if (d_rem) {
    rc = launch_sketch_coeffs_host(kind, k, seed, rem_ids, d_rem, Sr.data());
    if (rc) return rc;
  }
  if (!d_add && !d_rem) {
    if (changed_groups) *changed_groups = 0;
    return SKMP_OK;
  }
  int64_t offs[2] = {0, n};
  std::vector<int64_t> cpre = chunk_prefix(1, offs);
  Carve cv(workspace, ws_bytes);
  TableBlob tb(cv);
  StatsBuffers sb;
  sb.offsets_dev = tb.put(offs, 2);
  sb.cprefix_dev = tb.put(cpre.data(), 2);
  const std::vector<double> Sat = transpose_coeffs(Sa, k, std::max<int64_t>(d_add, 1));
  const std::vector<double> Srt = transpose_coeffs(Sr, k, std::max<int64_t>(d_rem, 1));
  double* Sa_dev = tb.put(Sat.data(), Sat.size());
  double* Sr_dev = tb.put(Srt.data(), Srt.size());
  double* coef = cv.take<double>((size_t)std::max<int64_t>(std::max<int64_t>(d_add, d_rem), 1) * 2);
  const size_t dpart_elems = proj_part_elems(std::max<int64_t>(std::max<int64_t>(d_add, d_rem), 1), n, k);
  double* dpart = cv.take<double>(dpart_elems);
  stats_workspace(std::max<int64_t>(d_add, 1), cpre[1], cv, &sb);
  if (!workspace || !cv.fits()) {
    set_error("workspace too small: need " + std::to_string(cv.used) + " bytes");
    return SKMP_ENOMEM;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc2 = tb.upload(st)) return rc2;
  uint64_t mask = 0;
  if (d_add) {
    rc = run_dimstats(T_add, dtype, ldt, d_add, 1, cpre, sb, add_stats, (flags & SKMP_FLAG_CHECK_FINITE) != 0, st);
    if (rc) return rc;
    if (dtype == SKMP_F64)
      launch_project<double>(T_add, ldt, d_add, n, sb.offsets_dev, 1, add_stats, coef, Sa_dev, k, R, ldr, +1,
                             dpart, dpart_elems, st);
    else
      launch_project<float>(T_add, ldt, d_add, n, sb.offsets_dev, 1, add_stats, coef, Sa_dev, k, R, ldr, +1,
                            dpart, dpart_elems, st);
    for (int g = 0; g < k; ++g)
      for (int64_t j = 0; j < d_add; ++j)
        if (Sa[(size_t)g * d_add + j] != 0.0) mask |= 1ull << g;
  }
  if (d_rem) {
    if (dtype == SKMP_F64)
      launch_project<double>(T_rem, ldt, d_rem, n, sb.offsets_dev, 1, rem_stats, coef, Sr_dev, k, R, ldr, -1,
                             dpart, dpart_elems, st);
    else
      launch_project<float>(T_rem, ldt, d_rem, n, sb.offsets_dev, 1, rem_stats, coef, Sr_dev, k, R, ldr, -1,
                            dpart, dpart_elems, st);
    for (int g = 0; g < k; ++g)
      for (int64_t j = 0; j < d_rem; ++j)
        if (Sr[(size_t)g * d_rem + j] != 0.0) mask |= 1ull << g;
  }
  SKMP_CHECK_HIP(hipGetLastError());
  if (changed_groups) *changed_groups = mask;
  return SKMP_OK;
}

// ------------------------------------------------------------- streaming
extern "C" size_t sketch_append_workspace(int64_t d, int64_t n_series, const int64_t* new_offsets, int32_t k) {
  if (d < 1 || n_series < 1 || !new_offsets || k < 1) return 0;
  const int64_t N = new_offsets[n_series];
  if (N < 0) return 0;
  std::vector<int64_t> cpre = chunk_prefix(n_series, new_offsets);
  Carve cv(nullptr, 0);
  TableBlob tb(cv);
  tb.put<int64_t>(nullptr, n_series + 1);
  tb.put<int64_t>(nullptr, n_series + 1);
  tb.put<int64_t>(nullptr, n_series);
  tb.put<double>(nullptr, (size_t)proj_kb(k) * (size_t)d);
  cv.take<int64_t>((size_t)d);
  cv.take<double>((size_t)n_series * (size_t)d * 2);  // coefficients of the normalisation
  cv.take<double>((size_t)n_series * (size_t)d * 2);  // statistics of the finiteness check
  cv.take<double>(proj_part_elems(d, std::max<int64_t>(N, 1), k));
  stats_workspace(d, std::max<int64_t>(cpre[n_series], 1), cv, nullptr);
  return cv.used + 256;
}

extern "C" int sketch_append(const void* T_new, int32_t dtype, int64_t d, int64_t ldt, int64_t n_series,
                             const int64_t* new_offsets, const int64_t* dst_cols, const int64_t* dim_ids, int32_t k,
                             int32_t kind, uint64_t seed, const double* dim_stats, uint32_t flags, double* R,
                             int64_t ldr, void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  SKMP_REQUIRE(T_new && R && dim_stats && new_offsets && dst_cols, "null pointer argument");
  SKMP_REQUIRE(dtype == SKMP_F64 || dtype == SKMP_F32, "dtype must be SKMP_F64 or SKMP_F32");
  SKMP_REQUIRE(d >= 1, "d must be >= 1");
  SKMP_REQUIRE(n_series >= 1 && n_series < (1 << 30), "n_series out of range");
  SKMP_REQUIRE(new_offsets[0] == 0, "new_offsets[0] must be 0");
  for (int64_t s = 0; s < n_series; ++s)
    SKMP_REQUIRE(new_offsets[s + 1] >= new_offsets[s], "new_offsets must be non-decreasing");
  const int64_t N = new_offsets[n_series];
  SKMP_REQUIRE(ldt >= N, "ldt must be >= the number of new samples");
  for (int64_t s = 0; s < n_series; ++s) {
    const int64_t cnt = new_offsets[s + 1] - new_offsets[s];
    SKMP_REQUIRE(dst_cols[s] >= 0 && dst_cols[s] + cnt <= ldr, "a series' new columns run past ldr");
    SKMP_REQUIRE(s == 0 || dst_cols[s] >= dst_cols[s - 1] + (new_offsets[s] - new_offsets[s - 1]),
                 "destination columns must be ascending and disjoint");
  }
  SKMP_REQUIRE(k >= 1 && k <= 64, "k must lie in [1, 64]");
  SKMP_REQUIRE(kind == SKMP_SUM || kind == SKMP_COUNT || kind == SKMP_GAUSS, "unknown sketch kind");
  SKMP_REQUIRE(kind != SKMP_SUM || k == 1, "the sum sketch has k = 1");
  if (N == 0) return SKMP_OK;
  const bool device_coeffs = (kind == SKMP_COUNT || kind == SKMP_SUM);
  int rc = SKMP_OK;
  std::vector<double> St;
  if (device_coeffs) {
    if ((rc = check_ids(dim_ids, d))) return rc;
  } else {
    std::vector<double> S((size_t)k * (size_t)d);
    if ((rc = launch_sketch_coeffs_host(kind, k, seed, dim_ids, d, S.data()))) return rc;
    St = transpose_coeffs(S, k, d);
  }
  std::vector<int64_t> cpre = chunk_prefix(n_series, new_offsets);
  std::vector<int64_t> shift((size_t)n_series);
  for (int64_t s = 0; s < n_series; ++s) shift[s] = dst_cols[s] - new_offsets[s];
  Carve cv(workspace, ws_bytes);
  TableBlob tb(cv);
  StatsBuffers sb;
  sb.offsets_dev = tb.put(new_offsets, n_series + 1);
  sb.cprefix_dev = tb.put(cpre.data(), n_series + 1);
  const int64_t* shift_dev = tb.put(shift.data(), (size_t)n_series);
  const int kb = proj_kb(k);
  double* S_dev = device_coeffs ? cv.take<double>((size_t)kb * (size_t)d) : tb.put(St.data(), St.size());
  const int64_t* ids_dev = (device_coeffs && dim_ids) ? tb.put(dim_ids, (size_t)d) : nullptr;
  double* coef = cv.take<double>((size_t)n_series * (size_t)d * 2);
  double* check_stats = cv.take<double>((size_t)n_series * (size_t)d * 2);
  const size_t dpart_elems = proj_part_elems(d, N, k);
  double* dpart = cv.take<double>(dpart_elems);
  stats_workspace(d, std::max<int64_t>(cpre[n_series], 1), cv, &sb);
  if (!workspace || !cv.fits()) {
    set_error("workspace too small: need " + std::to_string(cv.used) + " bytes");
    return SKMP_ENOMEM;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc2 = tb.upload(st)) return rc2;
  StageTimer tm(SKMP_TIMER_SKETCH, st);
  if (device_coeffs) {
    uint64_t a = 0, b = 0, a2 = 0, b2 = 0;
    count_params(seed, &a, &b, &a2, &b2);
    hipLaunchKernelGGL(count_coeffs_kernel, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, st, S_dev, d, kb, k,
                       kind, ids_dev, a, b, a2, b2, 0);
  }
  if (flags & SKMP_FLAG_CHECK_FINITE) {
    // the statistics pass doubles as the finiteness check; its values are not used
    rc = run_dimstats(T_new, dtype, ldt, d, n_series, cpre, sb, check_stats, true, st);
    if (rc) return rc;
  }
  if (dtype == SKMP_F64)
    launch_project<double>(T_new, ldt, d, N, sb.offsets_dev, (int)n_series, dim_stats, coef, S_dev, k, R, ldr, 0,
                           dpart, dpart_elems, st, shift_dev);
  else
    launch_project<float>(T_new, ldt, d, N, sb.offsets_dev, (int)n_series, dim_stats, coef, S_dev, k, R, ldr, 0,
                          dpart, dpart_elems, st, shift_dev);
  SKMP_CHECK_HIP(hipGetLastError());
  return SKMP_OK;
}

extern "C" size_t sketch_point_update_workspace(int64_t n_upd, int32_t k) {
  if (n_upd < 1 || k < 1 || k > 64) return 0;
  Carve cv(nullptr, 0);
  TableBlob tb(cv);
  tb.put<int64_t>(nullptr, (size_t)n_upd + 1);
  tb.put<PointUpd>(nullptr, (size_t)n_upd);
  tb.put<double>(nullptr, (size_t)n_upd * (size_t)k);
  return cv.used + 256;
}

extern "C" int sketch_point_update(double* R, int64_t ldr, int64_t n_cols, int32_t k, int32_t kind, uint64_t seed,
                                   int64_t d, const int64_t* dim_ids, int64_t n_series, const double* dim_stats,
                                   int64_t n_upd, const int64_t* upd_series, const int64_t* upd_dim,
                                   const int64_t* upd_col, const double* upd_delta, uint64_t* changed_groups,
                                   void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  if (changed_groups) *changed_groups = 0;
  SKMP_REQUIRE(R && dim_stats, "null pointer argument");
  SKMP_REQUIRE(k >= 1 && k <= 64, "k must lie in [1, 64]");
  SKMP_REQUIRE(kind == SKMP_SUM || kind == SKMP_COUNT || kind == SKMP_GAUSS, "unknown sketch kind");
  SKMP_REQUIRE(kind != SKMP_SUM || k == 1, "the sum sketch has k = 1");
  SKMP_REQUIRE(d >= 1 && n_series >= 1, "d and n_series must be >= 1");
  SKMP_REQUIRE(n_cols >= 1 && ldr >= n_cols, "bad column count or stride");
  SKMP_REQUIRE(n_upd >= 0, "negative update count");
  if (n_upd == 0) return SKMP_OK;
  SKMP_REQUIRE(upd_dim && upd_col && upd_delta, "null update array");
  if (int rc = check_ids(dim_ids, d)) return rc;
  for (int64_t u = 0; u < n_upd; ++u) {
    SKMP_REQUIRE(upd_dim[u] >= 0 && upd_dim[u] < d, "update dimension out of range");
    SKMP_REQUIRE(upd_col[u] >= 0 && upd_col[u] < n_cols, "update column out of range");
    SKMP_REQUIRE(!upd_series || (upd_series[u] >= 0 && upd_series[u] < n_series), "update series out of range");
    SKMP_REQUIRE(std::isfinite(upd_delta[u]), "update deltas must be finite");
  }
  // coefficient rows of the dimensions the updates touch
  std::vector<int64_t> dims(upd_dim, upd_dim + n_upd);
  std::sort(dims.begin(), dims.end());
  dims.erase(std::unique(dims.begin(), dims.end()), dims.end());
  std::vector<int64_t> ids(dims.size());
  for (size_t q = 0; q < dims.size(); ++q) ids[q] = dim_ids ? dim_ids[dims[q]] : dims[q];
  const int64_t nd = (int64_t)dims.size();
  std::vector<double> S((size_t)k * (size_t)nd);
  if (int rc = launch_sketch_coeffs_host(kind, k, seed, ids.data(), nd, S.data())) return rc;
  std::vector<double> coef((size_t)nd * (size_t)k);  // row q: the k coefficients of dims[q]
  uint64_t mask = 0;
  for (int64_t q = 0; q < nd; ++q)
    for (int g = 0; g < k; ++g) {
      coef[(size_t)q * k + g] = S[(size_t)g * nd + q];
      if (S[(size_t)g * nd + q] != 0.0) mask |= 1ull << g;
    }
  // updates sorted by column, stable, and the column segments
  std::vector<int64_t> order((size_t)n_upd);
  for (int64_t u = 0; u < n_upd; ++u) order[u] = u;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return upd_col[a] < upd_col[b]; });
  std::vector<PointUpd> upd((size_t)n_upd);
  std::vector<int64_t> seg;
  seg.reserve((size_t)n_upd + 1);
  for (int64_t q = 0; q < n_upd; ++q) {
    const int64_t u = order[q];
    const int64_t s = upd_series ? upd_series[u] : 0;
    const int64_t crow = std::lower_bound(dims.begin(), dims.end(), upd_dim[u]) - dims.begin();
    upd[q] = PointUpd{upd_col[u], s * d + upd_dim[u], upd_delta[u], crow};
    if (q == 0 || upd_col[u] != upd[q - 1].col) seg.push_back(q);
  }
  seg.push_back(n_upd);
  const int64_t n_seg = (int64_t)seg.size() - 1;
  Carve cv(workspace, ws_bytes);
  TableBlob tb(cv);
  const int64_t* seg_dev = tb.put(seg.data(), seg.size());
  const PointUpd* upd_dev = tb.put(upd.data(), upd.size());
  const double* coef_dev = tb.put(coef.data(), coef.size());
  if (!workspace || !cv.fits()) {
    set_error("workspace too small: need " + std::to_string(cv.used) + " bytes");
    return SKMP_ENOMEM;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc2 = tb.upload(st)) return rc2;
  const int64_t threads = n_seg * k;
  hipLaunchKernelGGL(point_update_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, R, ldr, k, n_seg,
                     seg_dev, upd_dev, coef_dev, dim_stats);
  SKMP_CHECK_HIP(hipGetLastError());
  if (changed_groups) *changed_groups = mask;
  return SKMP_OK;
}
