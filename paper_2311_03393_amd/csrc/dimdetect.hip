// Discord dimension detection (Algorithm 3): for every dimension j of the
// discord's group, the z-normalised distance (Def. 3) from the test
// subsequence starting at i* in dimension j to its nearest subsequence of the
// train series in dimension j -- the AB-join of that one subsequence (Def. 6);
// with the train series itself as the test series (the self-join setting),
// subsequences within excl of i* are trivial matches -- and the first
// dimension with the strictly largest score.
//
// The dimensions are read raw.  The z-normalised distance does not change
// under Algorithm 1's per-dimension normalisation, which only decides two
// things the kernels reproduce: a constant dimension (sigma_j = 0 in the
// sketch statistics) normalises to zeros, so all its subsequences are flat;
// and a subsequence of the normalised dimension is flat when its sigma is
// <= 1e-10 max|Tbar_j|, i.e. sigma(window of T_j) <= 1e-10 max|T_j - mu_j|.
//
//   dd_scale:  max|T_j - mu_j| of every selected dimension of both series;
//   dd_dist:   one block per (dimension, 1024 train subsequences): the test
//              subsequence and the block's samples in LDS; each thread takes
//              four consecutive subsequences: means and sigmas (two passes),
//              then the distances from explicit differences of the normalised
//              windows, all FP64; the block's nearest (smallest index on ties)
//              goes to the workspace;
//   dd_reduce: the nearest over a dimension's blocks -> score, neighbour;
//   dd_pick:   the first dimension with the strictly largest score above 0.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <climits>
#include <string>
#include <vector>

#include "skmp_common.hpp"

namespace skmp {

constexpr int DD_THREADS = 256;
constexpr double DD_FLAT_REL = 1e-10;

struct DDState {
  const void* Ttr;  // train series, dims x n_tr (row stride ld_tr), FP64 or FP32
  const void* Tte;  // test series (== Ttr in the self-join setting)
  int64_t ld_tr, ld_te;
  int64_t n_tr, n_te;
  const double* st_tr;  // (mu, sigma) per dimension of the train series
  const double* st_te;
  const int64_t* dims;  // selected dimension rows, n_dims
  int32_t n_dims;
  int32_t f32;          // input dtype is FP32
  int32_t m;
  int32_t excl;         // > 0: self-join setting, |t - i*| < excl excluded
  int64_t i_star;
  int64_t nblk;         // blocks of DD_SPAN train subsequences per dimension
  unsigned long long* scale;  // 2 x n_dims: max|T_j - mu_j| bits (train, test)
  double2* part;        // n_dims x nblk: (distance, index) of each block's nearest
  double* scores;
  int64_t* nn;
  int32_t* best;
};

__device__ __forceinline__ double sample(const void* T, bool f32, int64_t idx) {
  return f32 ? (double)static_cast<const float*>(T)[idx] : static_cast<const double*>(T)[idx];
}

// max |T_j - mu_j| over both series: grid (n_dims, chunks), grid-stride over the
// longer series; one 64-bit atomic max per block and series (non-negative
// doubles order like their bit patterns).
__global__ __launch_bounds__(DD_THREADS) void dd_scale(DDState s) {
  __shared__ double red[2][DD_THREADS / 64];
  const int p = blockIdx.x;
  const int64_t row = s.dims[p];
  const double mu_tr = s.st_tr[2 * row], mu_te = s.st_te[2 * row];
  double a = 0.0, b = 0.0;
  const int64_t n = max(s.n_tr, s.n_te);
  for (int64_t t = (int64_t)blockIdx.y * DD_THREADS + threadIdx.x; t < n; t += (int64_t)gridDim.y * DD_THREADS) {
    if (t < s.n_tr) a = fmax(a, fabs(sample(s.Ttr, s.f32, row * s.ld_tr + t) - mu_tr));
    if (t < s.n_te) b = fmax(b, fabs(sample(s.Tte, s.f32, row * s.ld_te + t) - mu_te));
  }
  for (int off = 32; off > 0; off >>= 1) {
    a = fmax(a, __shfl_down(a, off));
    b = fmax(b, __shfl_down(b, off));
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < DD_THREADS / 64; ++w) {
      a = fmax(a, red[0][w]);
      b = fmax(b, red[1][w]);
    }
    atomicMax(s.scale + p, (unsigned long long)__double_as_longlong(a));
    atomicMax(s.scale + s.n_dims + p, (unsigned long long)__double_as_longlong(b));
  }
}

// (distance, index) order: smaller distance, then smaller index
__device__ __forceinline__ bool closer(double d, double i, double bd, double bi) {
  return d < bd || (d == bd && i < bi);
}

__device__ __forceinline__ void block_nearest(double& d, double& i, double* sd, double* si) {
  for (int off = 32; off > 0; off >>= 1) {
    const double od = __shfl_down(d, off), oi = __shfl_down(i, off);
    if (closer(od, oi, d, i)) {
      d = od;
      i = oi;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    sd[threadIdx.x >> 6] = d;
    si[threadIdx.x >> 6] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < DD_THREADS / 64; ++w)
      if (closer(sd[w], si[w], d, i)) {
        d = sd[w];
        i = si[w];
      }
  }
}

// Each thread takes DD_R consecutive train subsequences (windows r = 0 ..
// DD_R - 1 starting at w + r): in each pass over the samples every LDS read
// of w[k'] serves all the windows containing position k' (window r holds
// positions r .. r + m - 1), with one partial sum per window.  The reads per
// subsequence drop DD_R-fold; LDS bandwidth bounded the one-subsequence form.
constexpr int DD_R = 4;
constexpr int DD_SPAN = DD_THREADS * DD_R;  // train subsequences per block

template <typename F>
__device__ __forceinline__ void over_windows(const double* w, int m, F f) {
#pragma unroll
  for (int kp = 0; kp < DD_R - 1; ++kp) {  // positions before every window has started
    const double x = w[kp];
#pragma unroll
    for (int r = 0; r <= kp; ++r) f(x, kp, r);
  }
  for (int kp = DD_R - 1; kp < m; ++kp) {  // positions inside every window
    const double x = w[kp];
#pragma unroll
    for (int r = 0; r < DD_R; ++r) f(x, kp, r);
  }
#pragma unroll
  for (int e = 0; e < DD_R - 1; ++e) {  // positions after the first windows have ended
    const int kp = m + e;
    const double x = w[kp];
#pragma unroll
    for (int r = e + 1; r < DD_R; ++r) f(x, kp, r);
  }
}

__global__ __launch_bounds__(DD_THREADS) void dd_dist(DDState s) {
  extern __shared__ double dd_lds[];  // query m, then samples DD_SPAN + m - 1
  __shared__ double qstat[2];         // query mean, 1/sigma (0 when flat)
  __shared__ double sd[DD_THREADS / 64], si[DD_THREADS / 64];
  const int p = blockIdx.y;
  const int m = s.m;
  const int64_t row = s.dims[p];
  double* q = dd_lds;
  double* seg = dd_lds + m;
  const int64_t t0 = (int64_t)blockIdx.x * DD_SPAN;
  const int64_t n_sub = s.n_tr - m + 1;
  for (int k = threadIdx.x; k < m; k += DD_THREADS) q[k] = sample(s.Tte, s.f32, row * s.ld_te + s.i_star + k);
  for (int k = threadIdx.x; k < DD_SPAN + m - 1; k += DD_THREADS) {
    const int64_t t = t0 + k;
    seg[k] = t < s.n_tr ? sample(s.Ttr, s.f32, row * s.ld_tr + t) : 0.0;
  }
  __syncthreads();
  const bool const_tr = s.st_tr[2 * row + 1] == 0.0;
  if (threadIdx.x < 64) {  // the test subsequence's moments, by wave 0
    double a = 0.0;
    for (int k = threadIdx.x; k < m; k += 64) a += q[k];
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
    const double mq = a / m;
    double v = 0.0;
    for (int k = threadIdx.x; k < m; k += 64) {
      const double e = q[k] - mq;
      v = fma(e, e, v);
    }
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const double sq = sqrt(v / m);
    const double scale_te = __longlong_as_double((long long)s.scale[s.n_dims + p]);
    const bool qflat = s.st_te[2 * row + 1] == 0.0 || sq <= DD_FLAT_REL * scale_te;
    if (threadIdx.x == 0) {
      qstat[0] = mq;
      qstat[1] = qflat ? 0.0 : 1.0 / sq;
    }
  }
  __syncthreads();
  const double mq = qstat[0], iq = qstat[1];
  for (int k = threadIdx.x; k < m; k += DD_THREADS) q[k] = (q[k] - mq) * iq;  // zero vector when flat
  __syncthreads();

  const int64_t tb = t0 + (int64_t)threadIdx.x * DD_R;  // the thread's first subsequence
  bool ok[DD_R];
  bool any = false;
#pragma unroll
  for (int r = 0; r < DD_R; ++r) {
    const int64_t t = tb + r;
    ok[r] = t < n_sub;
    if (s.excl > 0) ok[r] = ok[r] && (t - s.i_star >= s.excl || s.i_star - t >= s.excl);
    any = any || ok[r];
  }
  double best_d = INFINITY, best_i = (double)INT64_MAX;
  if (any) {
    const double* w = seg + threadIdx.x * DD_R;
    // pass 1: means
    double S[DD_R];
#pragma unroll
    for (int r = 0; r < DD_R; ++r) S[r] = 0.0;
    over_windows(w, m, [&](double x, int, int r) { S[r] += x; });
    double mw[DD_R];
#pragma unroll
    for (int r = 0; r < DD_R; ++r) mw[r] = S[r] / m;
    // pass 2: variances
    double V[DD_R];
#pragma unroll
    for (int r = 0; r < DD_R; ++r) V[r] = 0.0;
    over_windows(w, m, [&](double x, int, int r) {
      const double e = x - mw[r];
      V[r] = fma(e, e, V[r]);
    });
    const double scale_tr = __longlong_as_double((long long)s.scale[p]);
    const bool qflat = iq == 0.0;
    bool wflat[DD_R];
    double iw[DD_R];
#pragma unroll
    for (int r = 0; r < DD_R; ++r) {
      const double sw = sqrt(V[r] / m);
      wflat[r] = const_tr || sw <= DD_FLAT_REL * scale_tr;
      iw[r] = wflat[r] ? 0.0 : 1.0 / sw;
    }
    // pass 3: distances from explicit differences of the normalised windows
    double A[DD_R];
#pragma unroll
    for (int r = 0; r < DD_R; ++r) A[r] = 0.0;
    over_windows(w, m, [&](double x, int kp, int r) {
      const double e = q[kp - r] - (x - mw[r]) * iw[r];
      A[r] = fma(e, e, A[r]);
    });
#pragma unroll
    for (int r = 0; r < DD_R; ++r) {
      if (!ok[r]) continue;
      double dist;
      if (qflat && wflat[r]) dist = 0.0;
      else if (qflat || wflat[r]) dist = sqrt((double)m);
      else dist = sqrt(A[r]);
      const double ti = (double)(tb + r);
      if (closer(dist, ti, best_d, best_i)) {
        best_d = dist;
        best_i = ti;
      }
    }
  }
  block_nearest(best_d, best_i, sd, si);
  if (threadIdx.x == 0) s.part[(int64_t)p * s.nblk + blockIdx.x] = make_double2(best_d, best_i);
}

__global__ __launch_bounds__(DD_THREADS) void dd_reduce(DDState s) {
  __shared__ double sd[DD_THREADS / 64], si[DD_THREADS / 64];
  const int p = blockIdx.x;
  double d = INFINITY, i = (double)INT64_MAX;
  for (int64_t b = threadIdx.x; b < s.nblk; b += DD_THREADS) {
    const double2 e = s.part[(int64_t)p * s.nblk + b];
    if (closer(e.x, e.y, d, i)) {
      d = e.x;
      i = e.y;
    }
  }
  block_nearest(d, i, sd, si);
  if (threadIdx.x == 0) {
    s.scores[p] = d;
    s.nn[p] = isinf(d) ? -1 : (int64_t)i;
  }
}

// Algorithm 3's scan: s_bsf = 0, j* replaced only by a strictly larger score;
// that is the first position of the maximum when the maximum exceeds 0.
__global__ __launch_bounds__(64) void dd_pick(DDState s) {
  double v = -1.0;
  int at = INT_MAX;
  for (int p = threadIdx.x; p < s.n_dims; p += 64) {
    const double x = s.scores[p];
    if (x > v) {
      v = x;
      at = p;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_down(v, off);
    const int oa = __shfl_down(at, off);
    if (ov > v || (ov == v && oa < at)) {
      v = ov;
      at = oa;
    }
  }
  if (threadIdx.x == 0) *s.best = (v > 0.0) ? at : 0;
}

__global__ void dd_fill_u64(unsigned long long* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

static size_t dd_carve(Carve& cv, int32_t n_dims, int64_t nblk, int64_t** dims_dev, unsigned long long** scale,
                       double2** part) {
  *dims_dev = cv.take<int64_t>((size_t)n_dims);
  *scale = cv.take<unsigned long long>(2 * (size_t)n_dims);
  *part = cv.take<double2>((size_t)n_dims * (size_t)nblk);
  return cv.used;
}

}  // namespace skmp

using namespace skmp;

extern "C" size_t dim_detect_workspace(int64_t n_train, int32_t n_dims, int32_t m) {
  if (n_train < m || n_dims < 1 || m < 4) return 0;
  const int64_t nblk = (n_train - m + 1 + DD_SPAN - 1) / DD_SPAN;
  Carve cv(nullptr, 0);
  int64_t* a;
  unsigned long long* b;
  double2* c;
  dd_carve(cv, n_dims, nblk, &a, &b, &c);
  return cv.used + 256;
}

extern "C" int dim_detect(const void* T_train, int64_t ld_train, int64_t n_train, const double* stats_train,
                          const void* T_test, int64_t ld_test, int64_t n_test, const double* stats_test,
                          int32_t dtype, int64_t d, const int64_t* dims, int32_t n_dims, int64_t i_star, int32_t m,
                          int32_t excl, double* scores, int64_t* nn, int32_t* best, void* workspace, size_t ws_bytes,
                          void* stream) {
  clear_error();
  SKMP_REQUIRE(T_train && stats_train && T_test && stats_test && dims && scores && nn && best, "null pointer argument");
  SKMP_REQUIRE(dtype == SKMP_F64 || dtype == SKMP_F32, "dtype must be SKMP_F64 or SKMP_F32");
  SKMP_REQUIRE(m >= 4 && m <= 2048, "m must lie in [4, 2048]");
  SKMP_REQUIRE(d >= 1 && n_dims >= 1 && n_dims <= 65535, "need 1 <= n_dims <= 65535 and d >= 1");
  SKMP_REQUIRE(n_train >= m && n_test >= m, "both series need at least m samples");
  SKMP_REQUIRE(ld_train >= n_train && ld_test >= n_test, "row strides must be >= the series lengths");
  SKMP_REQUIRE(i_star >= 0 && i_star <= n_test - m, "i_star must start a subsequence of the test series");
  SKMP_REQUIRE(excl >= 0, "excl must be >= 0");
  SKMP_REQUIRE(excl == 0 || (T_test == T_train && stats_test == stats_train && ld_test == ld_train &&
                             n_test == n_train),
               "excl > 0 is the self-join setting: the test series must be the train series");
  SKMP_REQUIRE(n_train - m + 1 < ((int64_t)1 << 52), "series too long");
  for (int32_t q = 0; q < n_dims; ++q) SKMP_REQUIRE(dims[q] >= 0 && dims[q] < d, "dimension index out of range");
  const int64_t nblk = (n_train - m + 1 + DD_SPAN - 1) / DD_SPAN;
  SKMP_REQUIRE(nblk < (1ll << 31), "series too long");
  Carve cv(workspace, ws_bytes);
  int64_t* dims_dev;
  unsigned long long* scale;
  double2* part;
  dd_carve(cv, n_dims, nblk, &dims_dev, &scale, &part);
  if (!workspace || !cv.fits()) {
    set_error("workspace too small: need " + std::to_string(cv.used) + " bytes");
    return SKMP_ENOMEM;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (int rc = upload_async(dims_dev, dims, sizeof(int64_t) * (size_t)n_dims, st)) return rc;
  DDState s;
  s.Ttr = T_train;
  s.Tte = T_test;
  s.ld_tr = ld_train;
  s.ld_te = ld_test;
  s.n_tr = n_train;
  s.n_te = n_test;
  s.st_tr = stats_train;
  s.st_te = stats_test;
  s.dims = dims_dev;
  s.n_dims = n_dims;
  s.f32 = dtype == SKMP_F32;
  s.m = m;
  s.excl = excl;
  s.i_star = i_star;
  s.nblk = nblk;
  s.scale = scale;
  s.part = part;
  s.scores = scores;
  s.nn = nn;
  s.best = best;
  StageTimer tm(SKMP_TIMER_DIMDETECT, st);
  hipLaunchKernelGGL(dd_fill_u64, dim3((unsigned)((2 * (int64_t)n_dims + 255) / 256)), dim3(256), 0, st, scale,
                     2 * (int64_t)n_dims);
  const int64_t chunks = std::min<int64_t>((std::max(n_train, n_test) + DD_THREADS - 1) / DD_THREADS, 64);
  hipLaunchKernelGGL(dd_scale, dim3((unsigned)n_dims, (unsigned)chunks), dim3(DD_THREADS), 0, st, s);
  const size_t lds = sizeof(double) * (size_t)(m + DD_SPAN + m - 1);
  hipLaunchKernelGGL(dd_dist, dim3((unsigned)nblk, (unsigned)n_dims), dim3(DD_THREADS), lds, st, s);
  hipLaunchKernelGGL(dd_reduce, dim3((unsigned)n_dims), dim3(DD_THREADS), 0, st, s);
  hipLaunchKernelGGL(dd_pick, dim3(1), dim3(64), 0, st, s);
  SKMP_CHECK_HIP(hipGetLastError());
  return SKMP_OK;
}
