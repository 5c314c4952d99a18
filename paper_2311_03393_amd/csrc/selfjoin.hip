// Self-join matrix profile of the sketched series (paper Def. 3, Def. 6 and the
// self-join variant of Section III-B), FP64 diagonal kernel + shared stages.
//
// Stages (all on the caller's stream):
//   init      queue head and flat-window summaries;
//   scale     max |r| per (series, group): the flat-window threshold;
//   substats  per window x: mean, 1/(sqrt(m) sigma) (0 if flat), and the
//             difference terms df_x = (r[x+m] - r[x]) / 2,
//             dg_x = (r[x+m] - mu[x+1]) + (r[x] - mu[x]), all FP64 (plus
//             FP32 copies for the FP32 kernel); zeroes the key arrays;
//   tiles     the diagonal recurrence of the centred covariance
//             C(i+1, j+1) = C(i, j) + df_i dg_j + df_j dg_i, seeded exactly in
//             FP64, rho = C / (m sigma_i sigma_j), row and column nearest
//             neighbours as minima of 1 - rho with the partner encoded in the
//             low mantissa bits;
//   merge     pick the best row / column key, apply the flat-window rule and
//             recompute the reported distance exactly from explicit differences.
//
// Tile geometry (one wave64 per work unit):  a band holds 64*C consecutive
// diagonals, lane t owning diagonals db + t*C + q (q < C).  At step u lane t
// sits on row i = u - t, so the 64 lanes touch 64 distinct rows and, through
// the sliding window of C columns each lane keeps, 64 distinct retiring
// columns: per-step partial minima go to LDS with ds_min_u64 without
// conflicts.  Every TL steps the rows and columns that no later step of the
// unit can reach are flushed into the global key arrays with 64-bit atomic
// max; the others stay in LDS.  A work unit is one strip of S steps of one
// band of one (series, group); block b starts with unit b, a shared counter
// hands out the rest.  The FP32 kernel (below) walks the same geometry; the
// BF16x3 / FP16x3 MFMA tiles are in selfjoin_mixed.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <unistd.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "skmp_common.hpp"

namespace skmp {

// chunk (256 padded windows of one (series, group slot)) -> (s, gi, x0)
struct ChunkPos {
  int s, gi;
  int64_t x0;  // first window index (may be negative, down to -PADL)
};

__device__ __forceinline__ ChunkPos decode_chunk(const SJState& st, int64_t chunk) {
  ChunkPos c;
  c.s = find_series(st.plan, st.n_series, chunk, &SeriesPlan::chunk_base);
  const SeriesPlan& sp = st.plan[c.s];
  const int64_t per_group = (sp.lpad + 255) / 256;
  const int64_t local = chunk - sp.chunk_base;
  c.gi = (int)(local / per_group);
  c.x0 = (local - (int64_t)c.gi * per_group) * 256 - PADL;
  return c;
}

// max |r| per (series, group) for the flat-window threshold.  A block walks
// SCALE_CHUNKS consecutive chunks of 256 windows and keeps a running maximum
// per thread; whenever the (series, group) changes (and at the end) the block
// reduces it and issues one 64-bit atomic max, so an address receives a few
// atomics instead of one per wave.
constexpr int SCALE_CHUNKS = 8;

__device__ __forceinline__ void scale_flush(double v, unsigned long long* dst, double* red) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double b = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    if (b > 0.0) atomicMax(dst, (unsigned long long)__double_as_longlong(b));
  }
  __syncthreads();
}

// Start values of the per-(series, group) and per-block arrays and of the
// work counter, in one launch.
__global__ __launch_bounds__(256) void init_small(SJState st, int64_t n_sg, int64_t n_blk) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < max(n_sg, n_blk);
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i < n_sg) {
      reinterpret_cast<unsigned long long*>(st.scale)[i] = 0ull;
      st.flat_first[i] = INT_MAX;
      st.flat_last[i] = -1;
    }
    if (i < n_blk) st.flat_blk[i] = INT_MAX;
    if (i < 64) st.counter[i] = 0u;
  }
}

__global__ __launch_bounds__(256) void scale_kernel(SJState st) {
  __shared__ double red[4];
  const int64_t c0 = (int64_t)blockIdx.x * SCALE_CHUNKS;
  const int64_t c1 = min(c0 + SCALE_CHUNKS, st.total_chunks);
  // every chunk's sample first (independent loads in flight together), then
  // the running maxima in chunk order
  double v[SCALE_CHUNKS];
  int64_t key[SCALE_CHUNKS];
#pragma unroll
  for (int k = 0; k < SCALE_CHUNKS; ++k) {
    v[k] = 0.0;
    key[k] = -1;
    if (c0 + k < c1) {
      const ChunkPos c = decode_chunk(st, c0 + k);
      key[k] = (int64_t)c.s * st.groups.count + c.gi;
      const SeriesPlan& sp = st.plan[c.s];
      const int64_t t = c.x0 + threadIdx.x;
      const double* r = sp.r0 + (int64_t)st.groups.g[c.gi] * sp.ldr;
      if (t >= 0 && t < sp.n) v[k] = fabs(r[t]);
    }
  }
  double run = 0.0;
  int64_t cur = -1;
#pragma unroll
  for (int k = 0; k < SCALE_CHUNKS; ++k) {
    if (key[k] < 0) break;  // uniform
    if (key[k] != cur) {
      if (cur >= 0) scale_flush(run, reinterpret_cast<unsigned long long*>(st.scale) + cur, red);
      cur = key[k];
      run = 0.0;
    }
    run = fmax(run, v[k]);
  }
  if (cur >= 0) scale_flush(run, reinterpret_cast<unsigned long long*>(st.scale) + cur, red);
}

// Sum of m consecutive samples in four interleaved partial sums (shorter
// dependency chains); every window's sum is formed in this one order.
__device__ __forceinline__ double window_sum(const double* w, int m) {
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  int q = 0;
  for (; q + 4 <= m; q += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] += w[q + u];
  }
  for (; q < m; ++q) a[0] += w[q];
  return (a[0] + a[1]) + (a[2] + a[3]);
}

__global__ __launch_bounds__(256) void substats_kernel(SJState st) {
  extern __shared__ double sh_r[];  // 256 + m + 1 samples, then the 256 window means
  const ChunkPos c = decode_chunk(st, blockIdx.x);
  const SeriesPlan& sp = st.plan[c.s];
  const int m = st.m;
  const double* r = sp.r0 + (int64_t)st.groups.g[c.gi] * sp.ldr;
  const int span = 256 + m + 1;
  for (int q = threadIdx.x; q < span; q += 256) {
    const int64_t t = c.x0 + q;
    sh_r[q] = (t >= 0 && t < sp.n) ? r[t] : 0.0;
  }
  __syncthreads();
  const int64_t x = c.x0 + threadIdx.x;
  const double* w = sh_r + threadIdx.x;
  const double inv_m = 1.0 / m;
  // window means first: the mean of window x + 1 (needed for dg) is read from
  // its own thread, so both uses of it carry the same bits
  double* smu = sh_r + span;
  double mu = 0.0;
  if (x >= 0 && x < sp.n_sub) mu = window_sum(w, m) * inv_m;
  smu[threadIdx.x] = mu;
  __syncthreads();
  // the chunk grid rounds each group's padded range up to 256: stay inside it
  if (x >= sp.lpad - PADL) return;
  const int64_t gbase = (int64_t)c.gi * st.gstride + sp.stat_base;
  const int64_t sidx = gbase + PADL + x;
  const int64_t xp = x + PADL;
  const int64_t tidx = gbase + (xp % st.cstride) * (sp.lpad / st.cstride) + xp / st.cstride;
  st.rowkey[sidx] = 0ull;  // the tile kernels' max targets start at zero
  st.colkey[sidx] = 0ull;
  if (x < 0 || x >= sp.n_sub) {
    const double qnan = __longlong_as_double(0x7FF8000000000000ll);  // quiet NaN marks padding
    st.invn[sidx] = qnan;
    st.mu[sidx] = 0.0;
    if (st.bplanes) {
      blk_write_planes(st, 8 * gbase, sp.lpad, xp, 0.0, 0.0, 1.0);
      st.finvn[sidx] = __int_as_float(0x7FC00000);
    }
    if (!st.walk_stats) return;
    st.dfdg[sidx] = make_double2(0.0, 0.0);
    st.cdfdg[tidx] = make_double2(0.0, 0.0);
    st.cinvn[tidx] = qnan;
    if (st.fdfdg) {
      const float fnan = __int_as_float(0x7FC00000);
      st.fdfdg[sidx] = make_float2(0.f, 0.f);
      st.finvn[sidx] = fnan;
      st.fcdfdg[tidx] = make_float2(0.f, 0.f);
      st.fcinvn[tidx] = fnan;
    }
    return;
  }
  double va[4] = {0.0, 0.0, 0.0, 0.0};
  {
    int q = 0;
    for (; q + 4 <= m; q += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double e = w[q + u] - mu;
        va[u] = fma(e, e, va[u]);
      }
    }
    for (; q < m; ++q) {
      const double e = w[q] - mu;
      va[0] = fma(e, e, va[0]);
    }
  }
  const double v = (va[0] + va[1]) + (va[2] + va[3]);
  const double sd = sqrt(v * inv_m);
  const double scale = st.scale[(int64_t)c.s * st.groups.count + c.gi];
  const bool flat = sd <= FLAT_REL * scale;
  double df = 0.0, dg = 0.0;
  if (x + 1 < sp.n_sub) {
    double mu1;
    if (threadIdx.x + 1 < 256) {
      mu1 = smu[threadIdx.x + 1];
    } else {  // window x + 1 belongs to the next chunk: same sum, same order
      mu1 = window_sum(w + 1, m) * inv_m;
    }
    df = 0.5 * (w[m] - w[0]);
    dg = (w[m] - mu1) + (w[0] - mu);
  }
  const double iv = flat ? 0.0 : 1.0 / (sd * sqrt((double)m));
  st.invn[sidx] = iv;
  st.mu[sidx] = mu;
  if (st.bplanes) {
    // the blocked MFMA form's covariance carries the operands' power-of-two
    // scale squared; its FP32 norms carry 1 / scale each, so a cell's product
    // of the two norms removes it (exactly: powers of two)
    const double bs = blk_scale(scale, st.bprec);
    blk_write_planes(st, 8 * gbase, sp.lpad, xp, df, dg, bs);
    st.finvn[sidx] = (float)(iv / bs);
  }
  if (st.walk_stats) {
    st.dfdg[sidx] = make_double2(df, dg);
    st.cdfdg[tidx] = make_double2(df, dg);
    st.cinvn[tidx] = iv;
  }
  if (st.walk_stats && st.fdfdg) {
    st.fdfdg[sidx] = make_float2((float)df, (float)dg);
    st.finvn[sidx] = (float)iv;
    st.fcdfdg[tidx] = make_float2((float)df, (float)dg);
    st.fcinvn[tidx] = (float)iv;
  }
  if (flat) {
    const int64_t sg = (int64_t)c.s * st.groups.count + c.gi;
    atomicMin(st.flat_first + sg, (int32_t)x);
    atomicMax(st.flat_last + sg, (int32_t)x);
    atomicMin(st.flat_blk + (int64_t)c.gi * st.blk_stride + sp.blk_base + (x >> 8), (int32_t)x);
  }
}

// v_min_f64 without the canonicalising copy the compiler adds to IEEE fmin for
// operands it cannot prove canonical (the keys are bit-manipulated).  IEEE-mode
// min returns the non-NaN operand, which masks padded cells.
__device__ __forceinline__ double vmin(double a, double b) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// FP64 local keys: 1 - rho + 2^-40 (positive; FP64 rounding of rho is far
// below the bias) with the lane's diagonal code in the low bits, ordered by
// minimum; as positive doubles their bit patterns order like u64, so the LDS
// partials use ds_min_u64.  ~0 marks an empty partial, NaN bits (padded
// cells) lie above every real key.  Flushing converts to the global form
// 3 - key (= rho + 2, ordered by maximum).
constexpr double KEY_ONE64 = 1.0 + 9.094947017729282e-13;  // 1 + 2^-40
constexpr unsigned long long KEY_NONE64 = ~0ull;

__device__ __forceinline__ double embed(double x, uint32_t keep, uint32_t code) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const uint32_t lo = ((uint32_t)b & keep) | code;
  return __longlong_as_double((long long)((b & 0xFFFFFFFF00000000ull) | lo));
}

__device__ __forceinline__ unsigned long long kbits(double k) { return (unsigned long long)__double_as_longlong(k); }




// Exact FP64 seeds C(rr, j0 + q) = sum_x (r[rr+x] - mu[rr]) (r[j0+q+x] - mu[j0+q])
// for the C consecutive diagonals of every lane of the wave at step u: lane t
// is on row rr = max(u - t, 0) and its first diagonal starts at column
// j0 = rr + db + t C.  Rows come from (r, mu), columns from the column series
// (rc, muc): the same series in a self-join.  Written as sum_x a_x r[j0+q+x] - mu[j0+q] sum_x a_x with
// a_x = r[rr+x] - mu[rr], so the r values of the C diagonals stream through
// one sliding window.  The 64 rows span at most 64 + m samples and the 64 C
// diagonals at most 64 C + m, so chunks of MCH samples of both ranges are
// first staged in LDS with coalesced loads (stage: 64 + MCH + 64 C + MCH
// doubles); every lane then reads its windows from LDS.  Diagonals that end
// before row rr (j0 + q >= n_cols) read clamped samples and are zeroed.  Must be
// called by all 64 lanes with the same u.
// MCH is a multiple of C: 128 samples by default; 96 where the workgroups of a
// 4-wave-per-SIMD FP32 variant (16 per CU) must each fit in 10 KB of LDS.
template <int C, int WPE = 0>
constexpr int seed_chunk() { return ((WPE >= 4 && C == 16 ? 96 : 128) / C) * C; }
template <int C, int MCH = seed_chunk<C>()>
constexpr int seed_stage_len() { return 64 + MCH + 64 * C + MCH; }

// LDS of the FP32 tile kernel's workgroup: the row and column key partials
// (NROW + NCOL keys) and the exact-seed stage share one buffer, since the
// stage is only used at the start of a work unit, before the walk touches the
// keys (refill_keys empties them again).  The workgroup then needs the larger
// of the two (10.5 KB instead of 16.75 KB at C = 16; 10 KB with MCH = 96), so
// LDS does not cap the occupancy below what the register budget allows (3 or 4
// waves per SIMD).
template <typename K, int NROW, int NCOL, int C, int MCH>
constexpr int tile_lds_bytes() {
  return (int)sizeof(K) * (NROW + NCOL) > (int)sizeof(double) * seed_stage_len<C, MCH>()
             ? (int)sizeof(K) * (NROW + NCOL)
             : (int)sizeof(double) * seed_stage_len<C, MCH>();
}

template <typename K>
__device__ __forceinline__ void refill_keys(K* keys, int count, K empty, int t) {
  __syncthreads();  // every lane is done with the seed stage
  for (int x = t; x < count; x += 64) keys[x] = empty;
  __syncthreads();
}

template <int C, int MCH = seed_chunk<C>()>
__device__ __forceinline__ void exact_seeds(double* stage, const double* __restrict__ r, const double* __restrict__ mu,
                                            const double* __restrict__ rc, const double* __restrict__ muc, int u,
                                            int db, int t, int n_cols, int nlast, int nlast_c, int m,
                                            double (&acc)[C]) {
  double* srow = stage;
  double* scol = stage + 64 + MCH;
  const int rr = max(u - t, 0);
  const int j0 = rr + db + t * C;
  const int rbase = max(u - 63, 0);
  const int cbase = u + db;
  const int ro = rr - rbase;   // [0, 64)
  const int co = j0 - cbase;   // [0, 63 C]
  const double mr = mu[rr];
  double sa = 0.0;
#pragma unroll
  for (int q = 0; q < C; ++q) acc[q] = 0.0;
  constexpr int NR = (64 + MCH + 63) / 64, NCS = (64 * C + MCH + 63) / 64;
  for (int x0 = 0; x0 < m; x0 += MCH) {
    // every load of the chunk is issued before the first store (clamped
    // indices: all in bounds), so their latencies overlap
    double vr[NR], vc[NCS];
#pragma unroll
    for (int k = 0; k < NR; ++k) vr[k] = r[min(rbase + x0 + t + 64 * k, nlast)];
#pragma unroll
    for (int k = 0; k < NCS; ++k) vc[k] = rc[min(cbase + x0 + t + 64 * k, nlast_c)];
    __syncthreads();  // the previous chunk (or the caller's use of the stage) is done
#pragma unroll
    for (int k = 0; k < NR; ++k)
      if (t + 64 * k < 64 + MCH) srow[t + 64 * k] = vr[k];
#pragma unroll
    for (int k = 0; k < NCS; ++k)
      if (t + 64 * k < 64 * C + MCH) scol[t + 64 * k] = vc[k];
    __syncthreads();
    const int xe = min(MCH, m - x0);
    int xx = 0;
    for (; xx + C <= xe; xx += C) {
      double w[2 * C - 1];
#pragma unroll
      for (int k = 0; k < 2 * C - 1; ++k) w[k] = scol[co + xx + k];
#pragma unroll
      for (int dx = 0; dx < C; ++dx) {
        const double a = srow[ro + xx + dx] - mr;
        sa += a;
#pragma unroll
        for (int q = 0; q < C; ++q) acc[q] = fma(a, w[dx + q], acc[q]);
      }
    }
    for (; xx < xe; ++xx) {  // the last m mod C samples, one at a time (same summation order)
      const double a = srow[ro + xx] - mr;
      sa += a;
#pragma unroll
      for (int q = 0; q < C; ++q) acc[q] = fma(a, scol[co + xx + q], acc[q]);
    }
  }
  double mq[C];
#pragma unroll
  for (int q = 0; q < C; ++q) mq[q] = muc[min(j0 + q, n_cols - 1)];
#pragma unroll
  for (int q = 0; q < C; ++q) acc[q] = (j0 + q < n_cols) ? fma(-mq[q], sa, acc[q]) : 0.0;
}

template <int C>
struct LaneState {
  double Cq[C];
  double cdf[C], cdg[C], cinv[C];
  double colacc[C];
};

// Statistics of the row and of the newly entering column, fetched one step ahead.
struct StepLoad {
  double2 rs;    // (df, dg) of row i
  double rinv;   // invn of row i
  double2 cs;    // (df, dg) of the column entering the window
  double cinv;
};

// Buffer resources over one (series, group)'s padded statistics (element 0 is
// window -PADL).  Offsets split into a per-lane constant (voffset), a uniform
// part (soffset, scalar unit) and the step's immediate, so the per-step
// address arithmetic costs no vector instructions.
struct StatRsrc {
  __amdgpu_buffer_rsrc_t rd, ri;  // natural layout: dfdg, invn
  __amdgpu_buffer_rsrc_t cd, ci;  // de-interleaved by C - 1: cdfdg, cinvn
  int plane;                      // lpad / (C - 1)
};


template <int C>
__device__ __forceinline__ StatRsrc make_rsrc(const SJState& st, int64_t gbase, int64_t lpad, int64_t cgbase,
                                              int64_t clpad) {
  StatRsrc r;
  r.rd = __builtin_amdgcn_make_buffer_rsrc((void*)(st.dfdg + gbase), 0, (int)(lpad * 16), kBufWord3);
  r.ri = __builtin_amdgcn_make_buffer_rsrc((void*)(st.invn + gbase), 0, (int)(lpad * 8), kBufWord3);
  r.cd = __builtin_amdgcn_make_buffer_rsrc((void*)(st.cdfdg + cgbase), 0, (int)(clpad * 16), kBufWord3);
  r.ci = __builtin_amdgcn_make_buffer_rsrc((void*)(st.cinvn + cgbase), 0, (int)(clpad * 8), kBufWord3);
  r.plane = (int)(clpad / (C - 1));
  return r;
}

// Loads for the step whose rows are u - t and whose entering column is
// U + (C - 1) t (U = u + db + C - 1, uniform): rows from the natural layout at
// element u - t + PADL = (u + PADL - 63) + (63 - t); the column from plane
// (U + PADL) mod (C - 1), slot (U + PADL) div (C - 1) + t.
template <int C>
__device__ __forceinline__ StepLoad load_step(const StatRsrc& R, int u, int U, int t) {
  StepLoad l;
  const int rs_el = u + PADL - 63;        // >= 1: u >= 0
  const int vrow = 63 - t;
  l.rs = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(R.rd, vrow * 16, rs_el * 16, 0));
  l.rinv = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(R.ri, vrow * 8, rs_el * 8, 0));
  const int up = U + PADL;
  const int el = (up % (C - 1)) * R.plane + up / (C - 1);
  l.cs = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(R.cd, t * 16, el * 16, 0));
  l.cinv = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(R.ci, t * 8, el * 8, 0));
  return l;
}

// Runs ngroups * C steps.  On entry ring[k] holds the loads of step k of this
// call (k < PD); on exit it holds those of the PD steps after the last one.
// CL = false: each lane keeps a running maximum per open column and retires
// one column per step into LDS; CL = true: every cell's key goes straight to
// LDS with ds_max_u64 (fewer VALU max instructions, more LDS atomics).
template <int C, int PD, bool CL>
__device__ __forceinline__ void sj_run_groups(LaneState<C>& ls, StepLoad (&ring)[PD], const uint32_t (&code)[C],
                                              uint32_t keep, int ngroups, int u0, int db, const StatRsrc& R,
                                              unsigned long long* rowk, unsigned long long* colk, int t) {
  static_assert(C >= 2 && 64 * C <= 1024, "C diagonals per lane, local codes of at most 10 bits");
  for (int gidx = 0; gidx < ngroups; ++gidx) {
#pragma unroll
    for (int p = 0; p < C; ++p) {
      const int us = gidx * C + p;
      // prefetch PD steps ahead
      const int ua = u0 + us + PD;
      const StepLoad ahead = load_step<C>(R, ua, ua + db + C - 1, t);
      const StepLoad cur = ring[0];
#pragma unroll
      for (int k = 0; k + 1 < PD; ++k) ring[k] = ring[k + 1];
      ring[PD - 1] = ahead;
      const int sn = (p + C - 1) % C;
      ls.cdf[sn] = cur.cs.x;
      ls.cdg[sn] = cur.cs.y;
      ls.cinv[sn] = cur.cinv;
      const double2 rs = cur.rs;
      const double rinv = cur.rinv;
      double rowp = 0.0;
#pragma unroll
      for (int q = 0; q < C; ++q) {
        const int sl = (p + q) % C;
        const double a = ls.Cq[q] * ls.cinv[sl];
        double key = fma(-a, rinv, KEY_ONE64);  // 1 - rho + 2^-40
        key = embed(key, keep, code[q]);
        if (q == 0) rowp = key;
        else rowp = vmin(rowp, key);
        if (CL) {
          atomicMin(&colk[us + t * (C - 1) + q], kbits(key));
        } else {
          if (q == C - 1) ls.colacc[sl] = key;
          else ls.colacc[sl] = vmin(ls.colacc[sl], key);
        }
        ls.Cq[q] = fma(rs.x, ls.cdg[sl], ls.Cq[q]);
        ls.Cq[q] = fma(ls.cdf[sl], rs.y, ls.Cq[q]);
      }
      atomicMin(&rowk[us + 63 - t], kbits(rowp));
      if (!CL) atomicMin(&colk[us + t * (C - 1)], kbits(ls.colacc[p]));
    }
  }
}

// Flush of the LDS partials after the block of TL steps that starts at step
// u0.  rowk[x] holds row u0 - 63 + x (x < TL + 64), colk[x] column u0 + db + x
// (x < TL + 64 C).  After the block, rows x < TL and columns x < TL have all
// their cells of this unit (the one-lane skew and the band width bound the
// rows and columns a later step can touch), so they go to the global key
// arrays; unless this was the unit's last block, the other 64 rows and 64 C
// columns move down by TL and keep accumulating in the next block.  Every row
// and column of a unit is thereby flushed once.  to_global(key, delta) forms
// the global 64-bit key of a local key whose partner lies delta diagonals up.
// The local code in a key's low bits names the cell's diagonal within the
// band: QB = 0: code = LMAX - (t C + q) (lane t, its diagonal q); QB < 0:
// code = 63 - t in the low 6 bits, naming only the lane, whose C diagonals
// then all go up to the global key as the first of them (the key's partner
// is one of C consecutive ones).
template <int C, int TL, int QB = 0, typename K, typename G, typename V>
__device__ __forceinline__ void flush_block(K* rowk, K* colk, bool last, int u0, int db, int n_rows, int n_cols, int t,
                                            unsigned long long* gro, unsigned long long* gco, K empty, G to_global,
                                            V valid) {
  constexpr int NROW = TL + 64, NCOL = TL + 64 * C;
  constexpr int RPL = (NROW + 63) / 64, CPL = (NCOL + 63) / 64;
  constexpr uint32_t LMAX = (QB < 0) ? 63u : ((64 * C <= 512) ? 511u : ((64 * C <= 1024) ? 1023u : 2047u));
  auto diag = [](uint32_t code) -> int {
    if constexpr (QB < 0) {
      return (63 - (int)code) * C;  // the first of the lane's C diagonals
    } else {
      return (int)(LMAX - code);
    }
  };
  __syncthreads();
  K kr[RPL], kc[CPL];
#pragma unroll
  for (int q = 0; q < RPL; ++q) kr[q] = (t + 64 * q < NROW) ? rowk[t + 64 * q] : empty;
#pragma unroll
  for (int q = 0; q < CPL; ++q) kc[q] = (t + 64 * q < NCOL) ? colk[t + 64 * q] : empty;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int x = t + 64 * q;
    if (x < NROW) {
      if (x >= NROW - TL) rowk[x] = empty;                  // [64, NROW): cleared
      if (x >= TL) rowk[x - TL] = last ? empty : kr[q];    // [TL, NROW) -> [0, 64)
    }
  }
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int x = t + 64 * q;
    if (x < NCOL) {
      if (x >= NCOL - TL) colk[x] = empty;                  // [64 C, NCOL): cleared
      if (x >= TL) colk[x - TL] = last ? empty : kc[q];    // [TL, NCOL) -> [0, 64 C)
    }
  }
#pragma unroll
  for (int q = 0; q < RPL; ++q) {
    const int xl = t + 64 * q;
    const int x = u0 - 63 + xl;
    if (valid(kr[q]) && (last || xl < TL) && xl < NROW && x >= 0 && x < n_rows) {
      const int delta = db + diag((uint32_t)(kr[q] & LMAX));
      atomicMax(gro + x, to_global(kr[q], delta));
    }
  }
#pragma unroll
  for (int q = 0; q < CPL; ++q) {
    const int xl = t + 64 * q;
    const int j = u0 + db + xl;
    if (valid(kc[q]) && (last || xl < TL) && xl < NCOL && j < n_cols) {
      const int delta = db + diag((uint32_t)(kc[q] & LMAX));
      atomicMax(gco + j, to_global(kc[q], delta));
    }
  }
  __syncthreads();
}

template <int C, int TL, int PD, int WPE, bool CL>
__global__ __launch_bounds__(64, WPE) void sj_fp64_kernel(SJState st) {
  constexpr int NROW = TL + 64;
  constexpr int NCOL = TL + 64 * C;
  constexpr int LBITS = (64 * C <= 512) ? 9 : ((64 * C <= 1024) ? 10 : 11);
  constexpr uint32_t LMAX = (1u << LBITS) - 1;
  static_assert(TL % C == 0, "tile length must be a multiple of C");
  // separate key and seed buffers: measured faster for this kernel than the
  // shared buffer of the FP32 kernel (whose higher occupancy does not pay here)
  __shared__ unsigned long long rowk[NROW];
  __shared__ unsigned long long colk[NCOL];
  __shared__ double sseed[seed_stage_len<C>()];
  const int t = threadIdx.x;
  for (int x = t; x < NROW; x += 64) rowk[x] = KEY_NONE64;
  for (int x = t; x < NCOL; x += 64) colk[x] = KEY_NONE64;
  __syncthreads();
  const uint32_t keep = ~LMAX;
  uint32_t code[C];
#pragma unroll
  for (int q = 0; q < C; ++q) code[q] = LMAX - (uint32_t)(t * C + q);
  const unsigned long long GMAX = (1ull << st.key_bits) - 1;
  const int m = st.m;

  // work queue: the block's first unit is its own index (no contention on the
  // queue head while the grid fills the chip); each later unit is the counter's
  // value plus the grid size, taken when the previous unit is done
  auto take = [&]() -> unsigned int {
    unsigned int u = 0;
    if (t == 0) u = atomicAdd(st.counter, 1u);
    return __builtin_amdgcn_readfirstlane(__shfl(u, 0)) + gridDim.x;
  };
  for (unsigned int unit = blockIdx.x; (int64_t)unit < st.total_units; unit = take()) {
    const int s = uni(find_series(st.plan, st.n_series, (int64_t)unit, &SeriesPlan::unit_base));
    const SeriesPlan sp = load_plan(st, s);
    const int64_t local = (int64_t)unit - sp.unit_base;
    const int64_t per_group = (int64_t)sp.nb * sp.ns;
    const int gi = (int)(local / per_group);
    const int64_t rem = local - (int64_t)gi * per_group;
    const int sigma = (int)(rem / sp.nb);
    const int b = (int)(rem - (int64_t)sigma * sp.nb);
    const int n_sub = (int)sp.n_sub;    // rows: windows of this series
    const int n_cols = (int)sp.n_cols;  // columns: windows of the column series
    const int db = sp.d0 + b * 64 * C;
    // steps of the band: lane t is on row u - t, so the walk lasts until the
    // last lane has passed the last row of its longest diagonal (in a self-join
    // that is the first diagonal's n_sub - db rows; rows past n_sub are padding)
    const int Ub = min(n_sub + 63, n_cols - db);
    const int u_begin = max(0, sp.c0 - db) + sigma * st.strip;
    if (u_begin >= Ub) continue;
    const int u_end = min(u_begin + st.strip, Ub);

    const int64_t gbase = (int64_t)gi * st.gstride + sp.stat_base;    // rows
    const int64_t cgbase = (int64_t)gi * st.gstride + sp.cstat_base;  // columns
    const double2* __restrict__ cdfdg_n = st.dfdg + cgbase + PADL;
    const double* __restrict__ cinvn_n = st.invn + cgbase + PADL;
    const double* __restrict__ mu = st.mu + gbase + PADL;
    const double* __restrict__ muc = st.mu + cgbase + PADL;
    const int g = st.groups.g[gi];
    const double* __restrict__ r = sp.r0 + (int64_t)g * sp.ldr;
    const double* __restrict__ rc = sp.cr0 + (int64_t)g * sp.cldr;
    unsigned long long* gro = st.rowkey + gbase + PADL;
    unsigned long long* gco = st.colkey + cgbase + PADL;

    LaneState<C> ls;
    // exact FP64 seeds at the strip start: lane t's first row is u_begin - t
    exact_seeds<C>(sseed, r, mu, rc, muc, u_begin, db, t, n_cols, (int)sp.n - 1, (int)sp.cn - 1, m, ls.Cq);
    // column window: columns J + q (q < C-1) in slots q, J = u_begin + db + t (C-1)
    {
      const int J = u_begin + db + t * (C - 1);
#pragma unroll
      for (int q = 0; q < C - 1; ++q) {
        const double2 cs = cdfdg_n[J + q];
        ls.cdf[q] = cs.x;
        ls.cdg[q] = cs.y;
        ls.cinv[q] = cinvn_n[J + q];
        ls.colacc[q] = __longlong_as_double((long long)KEY_NONE64);
      }
    }

    const StatRsrc R = make_rsrc<C>(st, gbase, sp.lpad, cgbase, sp.clpad);
    StepLoad ring[PD];
#pragma unroll
    for (int k = 0; k < PD; ++k) ring[k] = load_step<C>(R, u_begin + k, u_begin + k + db + C - 1, t);
    for (int u0 = u_begin; u0 < u_end; u0 += TL) {
      const int ngroups = (min(TL, u_end - u0) + C - 1) / C;
      sj_run_groups<C, PD, CL>(ls, ring, code, keep, ngroups, u0, db, R, rowk, colk, t);
      const bool last = (u0 + TL >= u_end);
      if (last && !CL) {
        // retire the columns still open in the window (phase 0 after full groups)
#pragma unroll
        for (int q = 0; q < C - 1; ++q)
          atomicMin(&colk[ngroups * C + t * (C - 1) + q], kbits(ls.colacc[q]));
      }
      flush_block<C, TL>(
          rowk, colk, last, u0, db, n_sub, n_cols, t, gro, gco, KEY_NONE64,
          [GMAX](unsigned long long key, int delta) {
            const double v = 3.0 - __longlong_as_double((long long)(key & ~(unsigned long long)LMAX));
            return ((unsigned long long)__double_as_longlong(v) & ~GMAX) | (GMAX - (unsigned long long)delta);
          },
          [](unsigned long long key) { return key < 0x7FF0000000000000ull; });
    }
  }
}


// ------------------------------------------------------- FP32 tile kernel
// Same walk as the FP64 kernel with the running covariance, the window
// statistics and the keys in FP32: C(i+1, j+1) = C(i, j) + df_i dg_j + df_j dg_i
// in FP32 from an exact FP64 seed recomputed at the start of every strip
// (the strip length is the refresh period).  Keys are the bits of the FP32
// value 1 - rho + 2^-10 in (0, 2]; as positive floats they order like
// unsigned integers, so the nearest neighbour is a 32-bit integer minimum
// (v_min3_u32).  What reaches LDS has the lane's code in the low 6 bits, so
// the key keeps 17 of the 23 fraction bits: relative to its own distance,
// 1 - rho ~ 0.2 is resolved to 2^-20 (about 1e-6; rho + 2 in [1, 3] would
// resolve 2.4e-4), and near ties are decided far below the tolerance.  A key
// names the lane, not its diagonal: the merge scores the lane's C diagonals
// exactly and keeps the best (kgroup = C).  Padded cells give NaN
// keys, whose bits lie above every real key, so the minima ignore them.
// Flushing converts a key f to the global form 3 + 2^-10 - f = rho + 2 (maxima).
// The bias 2^-10 keeps the key positive while rho <= 1 + 2^-10: FP32 drift
// over a refresh period is orders of magnitude smaller, and a negative key
// (sign bit set) would read as an invalid cell.  The bias shifts every key
// alike, so it changes no ordering.
constexpr float KEY_ONE = 1.0f + 9.765625e-4f;  // 1 + 2^-10
constexpr double KEY_BACK = 3.0 + 9.765625e-4;

// Statistics of a row, fetched PD steps ahead.
struct StepLoadF {
  float2 rs;
  float rinv;
};

struct StatRsrcF {
  __amdgpu_buffer_rsrc_t rd, ri, cd, ci;
  int plane;
};

template <int C>
__device__ __forceinline__ StatRsrcF make_rsrc_f(const SJState& st, int64_t gbase, int64_t lpad, int64_t cgbase,
                                                 int64_t clpad) {
  StatRsrcF r;
  r.rd = __builtin_amdgcn_make_buffer_rsrc((void*)(st.fdfdg + gbase), 0, (int)(lpad * 8), kBufWord3);
  r.ri = __builtin_amdgcn_make_buffer_rsrc((void*)(st.finvn + gbase), 0, (int)(lpad * 4), kBufWord3);
  r.cd = __builtin_amdgcn_make_buffer_rsrc((void*)(st.fcdfdg + cgbase), 0, (int)(clpad * 8), kBufWord3);
  r.ci = __builtin_amdgcn_make_buffer_rsrc((void*)(st.fcinvn + cgbase), 0, (int)(clpad * 4), kBufWord3);
  r.plane = (int)(clpad / (C - 1));
  return r;
}

template <int C>
__device__ __forceinline__ StepLoadF load_row_f(const StatRsrcF& R, int u, int t) {
  StepLoadF l;
  const int rs_el = u + PADL - 63;
  const int vrow = 63 - t;
  l.rs = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(R.rd, vrow * 8, rs_el * 8, 0));
  l.rinv = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(R.ri, vrow * 4, rs_el * 4, 0));
  return l;
}

// Statistics of the column U (lane 0's; lane t's is U + t (C - 1)), loaded
// straight into the registers of a column slot.
template <int C>
__device__ __forceinline__ void load_col_f(const StatRsrcF& R, int U, int t, float& df, float& dg, float& inv) {
  const int up = U + PADL;
  const int el = (up % (C - 1)) * R.plane + up / (C - 1);
  const float2 cs = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(R.cd, t * 8, el * 8, 0));
  df = cs.x;
  dg = cs.y;
  inv = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(R.ci, t * 4, el * 4, 0));
}

template <int C>
struct LaneStateF {
  float Cq[C];
  float cdf[C], cdg[C], cinv[C];
  uint32_t colacc[C];
};

// A cell's key is the bare bits of its FP32 value: which of the lane's C
// diagonals it came from is not recorded.  The lane's row minimum of a step
// and a retiring column minimum (every key they combine is the lane's own)
// have their low 6 bits replaced by the lane's code 63 - t once, on their way
// to LDS; the merge later finds the partner among the lane's C diagonals.
// Truncating the low bits is monotone, so the truncated minimum is the
// minimum of the truncated keys.
// Column slots: the column of a step's diagonal 0 is used for the last time
// by that step's first cell, and the column entering at the next step (its
// diagonal C - 1, computed last) takes over its slot.  Its statistics are
// loaded right after that first cell, into the slot's own registers: about
// two steps of latency cover, and no register copies where the unrolled
// walk wraps around.
template <int C, int PD>
__device__ __forceinline__ void sjf_run_groups(LaneStateF<C>& ls, StepLoadF (&ring)[PD], uint32_t lcode,
                                               uint32_t keep, int ngroups, int u0, int db, const StatRsrcF& R,
                                               uint32_t* rowk, uint32_t* colk, int t) {
  for (int gidx = 0; gidx < ngroups; ++gidx) {
#pragma unroll
    for (int p = 0; p < C; ++p) {
      const int us = gidx * C + p;
      const StepLoadF ahead = load_row_f<C>(R, u0 + us + PD, t);
      const StepLoadF cur = ring[0];
#pragma unroll
      for (int k = 0; k + 1 < PD; ++k) ring[k] = ring[k + 1];
      ring[PD - 1] = ahead;
      uint32_t rowp = 0u;
#pragma unroll
      for (int q = 0; q < C; ++q) {
        const int sl = (p + q) % C;
        const float a = ls.Cq[q] * ls.cinv[sl];
        // 1 - rho (+ 2^-10 so FP32 rounding never makes it negative): a positive
        // float, resolved relative to itself, so close candidates stay apart
        const float kf = __builtin_fmaf(-a, cur.rinv, KEY_ONE);
        const uint32_t key = __float_as_uint(kf);  // padded cells: NaN bits, above every key
        rowp = (q == 0) ? key : min(rowp, key);
        if (q == C - 1) ls.colacc[sl] = key;
        else ls.colacc[sl] = min(ls.colacc[sl], key);
        ls.Cq[q] = __builtin_fmaf(cur.rs.x, ls.cdg[sl], ls.Cq[q]);
        ls.Cq[q] = __builtin_fmaf(ls.cdf[sl], cur.rs.y, ls.Cq[q]);
        if (q == 0) load_col_f<C>(R, u0 + us + db + C, t, ls.cdf[sl], ls.cdg[sl], ls.cinv[sl]);
      }
      atomicMin(&rowk[us + 63 - t], (rowp & keep) | lcode);
      atomicMin(&colk[us + t * (C - 1)], (ls.colacc[p] & keep) | lcode);
    }
  }
}

template <int C, int TL, int PD, int WPE>
__global__ __launch_bounds__(64, WPE) void sj_fp32_kernel(SJState st) {
  constexpr int NROW = TL + 64;
  constexpr int NCOL = TL + 64 * C;
  constexpr uint32_t LMAX = 63u;  // local code: the lane
  static_assert(TL % C == 0, "tile length must be a multiple of C");
  static_assert(C >= 2 && C <= 16, "C diagonals per lane (the merge searches at most 16)");
  constexpr int MCH = seed_chunk<C, WPE>();
  static_assert(WPE < 4 || tile_lds_bytes<uint32_t, NROW, NCOL, C, MCH>() <= 10240,
                "16 workgroups of one wave per CU share its 160 KB of LDS");
  __shared__ __align__(16) uint32_t lds[tile_lds_bytes<uint32_t, NROW, NCOL, C, MCH>() / 4];
  uint32_t* rowk = lds;
  uint32_t* colk = lds + NROW;
  double* sseed = reinterpret_cast<double*>(lds);
  const int t = threadIdx.x;
  const uint32_t keep = ~LMAX;
  const uint32_t lcode = (uint32_t)(63 - t);
  const unsigned long long GMAX = (1ull << st.key_bits) - 1;
  const int m = st.m;

  // work queue: the block's first unit is its own index (no contention on the
  // queue head while the grid fills the chip); each later unit is the counter's
  // value plus the grid size, taken when the previous unit is done
  auto take = [&]() -> unsigned int {
    unsigned int u = 0;
    if (t == 0) u = atomicAdd(st.counter, 1u);
    return __builtin_amdgcn_readfirstlane(__shfl(u, 0)) + gridDim.x;
  };
  for (unsigned int unit = blockIdx.x; (int64_t)unit < st.total_units; unit = take()) {
    const int s = uni(find_series(st.plan, st.n_series, (int64_t)unit, &SeriesPlan::unit_base));
    const SeriesPlan sp = load_plan(st, s);
    const int64_t local = (int64_t)unit - sp.unit_base;
    const int64_t per_group = (int64_t)sp.nb * sp.ns;
    const int gi = (int)(local / per_group);
    const int64_t rem = local - (int64_t)gi * per_group;
    const int sigma = (int)(rem / sp.nb);
    const int b = (int)(rem - (int64_t)sigma * sp.nb);
    const int n_sub = (int)sp.n_sub;    // rows: windows of this series
    const int n_cols = (int)sp.n_cols;  // columns: windows of the column series
    const int db = sp.d0 + b * 64 * C;
    // steps of the band: lane t is on row u - t, so the walk lasts until the
    // last lane has passed the last row of its longest diagonal (in a self-join
    // that is the first diagonal's n_sub - db rows; rows past n_sub are padding)
    const int Ub = min(n_sub + 63, n_cols - db);
    const int u_begin = max(0, sp.c0 - db) + sigma * st.strip;
    if (u_begin >= Ub) continue;
    const int u_end = min(u_begin + st.strip, Ub);
    const int64_t gbase = (int64_t)gi * st.gstride + sp.stat_base;    // rows
    const int64_t cgbase = (int64_t)gi * st.gstride + sp.cstat_base;  // columns
    const double* __restrict__ mu = st.mu + gbase + PADL;
    const double* __restrict__ muc = st.mu + cgbase + PADL;
    const int g = st.groups.g[gi];
    const double* __restrict__ r = sp.r0 + (int64_t)g * sp.ldr;
    const double* __restrict__ rc = sp.cr0 + (int64_t)g * sp.cldr;
    unsigned long long* gro = st.rowkey + gbase + PADL;
    unsigned long long* gco = st.colkey + cgbase + PADL;

    LaneStateF<C> ls;
    // a wave computing seeds (FP64, single rate) yields the issue to the waves
    // that walk (FP32 pairs dual-issue): 2 % faster on the water-treatment join
    __builtin_amdgcn_s_setprio(0);
    {  // exact FP64 seeds, rounded once to FP32
      double acc[C];
      exact_seeds<C, MCH>(sseed, r, mu, rc, muc, u_begin, db, t, n_cols, (int)sp.n - 1, (int)sp.cn - 1, m, acc);
#pragma unroll
      for (int q = 0; q < C; ++q) ls.Cq[q] = (float)acc[q];
    }
    refill_keys(lds, NROW + NCOL, 0xFFFFFFFFu, t);
    const StatRsrcF R = make_rsrc_f<C>(st, gbase, sp.lpad, cgbase, sp.clpad);
    // the first step's columns: diagonal q in slot q (C - 1 enters with it)
#pragma unroll
    for (int q = 0; q < C; ++q) {
      load_col_f<C>(R, u_begin + db + q, t, ls.cdf[q], ls.cdg[q], ls.cinv[q]);
      ls.colacc[q] = 0xFFFFFFFFu;
    }
    __builtin_amdgcn_s_setprio(1);
    StepLoadF ring[PD];
#pragma unroll
    for (int k = 0; k < PD; ++k) ring[k] = load_row_f<C>(R, u_begin + k, t);
    for (int u0 = u_begin; u0 < u_end; u0 += TL) {
      const int ngroups = (min(TL, u_end - u0) + C - 1) / C;
      sjf_run_groups<C, PD>(ls, ring, lcode, keep, ngroups, u0, db, R, rowk, colk, t);
      const bool last = (u0 + TL >= u_end);
      if (last) {
#pragma unroll
        for (int q = 0; q < C - 1; ++q)
          atomicMin(&colk[ngroups * C + t * (C - 1) + q], (ls.colacc[q] & keep) | lcode);
      }
      flush_block<C, TL, -1>(
          rowk, colk, last, u0, db, n_sub, n_cols, t, gro, gco, 0xFFFFFFFFu,
          [GMAX](uint32_t key, int delta) {
            // local keys order by 1 - rho + 2^-10 (min); the global ones by
            // 3 + 2^-10 - that = rho + 2 (max)
            const double v = KEY_BACK - (double)__uint_as_float(key & ~LMAX);
            const unsigned long long kb = (unsigned long long)__double_as_longlong(v);
            return (kb & ~GMAX) | (GMAX - (unsigned long long)delta);
          },
          [](uint32_t key) { return key < 0x7F800000u; });
    }
  }
}

// ------------------------------------------------------------------ merge
__device__ int smallest_flat_at_or_after(const SJState& st, const double* invn, const int32_t* fblk, int64_t y,
                                         int64_t last) {
  if (y > last) return -1;
  int64_t blk = y >> 8;
  // partial first block: scan elements
  const int64_t first_end = (blk + 1) << 8;
  if (fblk[blk] != INT_MAX && fblk[blk] <= last) {
    for (int64_t z = y; z < first_end && z <= last; ++z)
      if (invn[z] == 0.0) return (int)z;
  }
  for (++blk; (blk << 8) <= last; ++blk)
    if (fblk[blk] != INT_MAX) return fblk[blk];
  return -1;
}

// ------------------------------------------------- short appends, direct
// An append of at most APPEND_DIRECT new windows per series does not walk
// bands (a short walk is a chain of dependent per-step loads): every new pair
// (i, j), j >= keep, j - i >= excl, is computed directly as an exact FP64 dot
// product of the centred windows, C = sum_t (r[i+t] - mu_i)(r[j+t] - mu_j),
// one thread per row i of a 256-window chunk, the new windows' samples staged
// in LDS.  Row i's best new partner above goes to rowkey[i] (this thread is its
// only writer); new window j's best partner below is reduced over the wave and
// the block and goes to colkey[j] by atomic maximum.  Keys have the tile
// kernels' global form (rho + 2 with GMAX - delta in the low bits), so the
// merge and FP64 polish are shared.
constexpr int APPEND_DIRECT = 32;  // the kernel's limit (LDS sizing)
// Chosen for up to about 2000 / m new windows: its cost grows by ~3.4 us per
// new window per 100 samples of m (8 groups of 50,000 windows), the band walk
// of a short append costs ~85 us whatever the count (measured: break-even
// near 20 new windows at m = 100).
static inline int append_direct_max(int m) { return std::min(APPEND_DIRECT, std::max(1, 2000 / m)); }

__global__ __launch_bounds__(256) void append_direct_kernel(SJState st) {
  extern __shared__ double sh_a[];  // the chunk's rows: 256 + m - 1 samples, then the new windows' A + m - 1 (+ 3 zeros)
  __shared__ unsigned long long ckey[APPEND_DIRECT];
  const ChunkPos c = decode_chunk(st, blockIdx.x);
  const SeriesPlan& sp = st.plan[c.s];
  const int m = st.m;
  const int64_t n_sub = sp.n_sub, keep = sp.keep;
  const int A = (int)(n_sub - keep);
  // rows that can pair with a new window: x <= n_sub - 1 - excl
  if (sp.p0 == nullptr || A <= 0 || A > APPEND_DIRECT || c.x0 + 255 < 0 || c.x0 > n_sub - 1 - st.excl) return;
  const int g = st.groups.g[c.gi];
  const double* r = sp.r0 + (int64_t)g * sp.ldr;
  double* sw = sh_a;
  double* sq = sh_a + 256 + m - 1;
  for (int q = threadIdx.x; q < 256 + m - 1; q += 256) {
    const int64_t t = c.x0 + q;
    sw[q] = (t >= 0 && t < sp.n) ? r[t] : 0.0;
  }
  for (int q = threadIdx.x; q < A + m - 1 + 3; q += 256) sq[q] = (q < A + m - 1) ? r[keep + q] : 0.0;
  if (threadIdx.x < APPEND_DIRECT) ckey[threadIdx.x] = 0ull;
  __syncthreads();
  const int64_t sbase = (int64_t)c.gi * st.gstride + sp.stat_base + PADL;
  const unsigned long long GMAX = (1ull << st.key_bits) - 1;
  const int64_t x = c.x0 + threadIdx.x;
  const bool row_ok = x >= 0 && x < n_sub;
  const double mx = row_ok ? st.mu[sbase + x] : 0.0;
  const double ix = row_ok ? st.invn[sbase + x] : 0.0;
  const double* w = sw + threadIdx.x;
  double se = 0.0;  // sum_t (r[x+t] - mu_x)
  if (row_ok)
    for (int t = 0; t < m; ++t) se += w[t] - mx;
  unsigned long long rk = 0ull;
  const int lane = threadIdx.x & 63;
  // four new windows per pass: each centred row sample feeds four products
  for (int a0 = 0; a0 < A; a0 += 4) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const double* q = sq + a0;  // q[k + t]: window a0 + k (staged up to index A + m - 2; k + t past it is unused)
    if (row_ok) {
      for (int t = 0; t < m; ++t) {
        const double e = w[t] - mx;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = fma(e, q[k + t], acc[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int a = a0 + k;
      if (a >= A) break;  // uniform
      const int64_t j = keep + a;
      const int64_t delta = j - x;
      unsigned long long key = 0ull;
      if (row_ok && delta >= st.excl) {
        const double mj = st.mu[sbase + j], ij = st.invn[sbase + j];
        const double C = fma(-mj, se, acc[k]);
        const double v = fma(C * ij, ix, 2.0);  // rho + 2
        key = ((unsigned long long)__double_as_longlong(v) & ~GMAX) | (GMAX - (unsigned long long)delta);
        rk = max(rk, key);
      }
      // column j: the best partner below over the wave, then the block
      unsigned long long wk = key;
      for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = (unsigned long long)__shfl_xor((long long)wk, off);
        wk = max(wk, o);
      }
      if (lane == 0 && wk != 0ull) atomicMax(&ckey[a], wk);
    }
  }
  if (row_ok) st.rowkey[sbase + x] = rk;
  __syncthreads();
  if ((int)threadIdx.x < A && ckey[threadIdx.x] != 0ull) atomicMax(st.colkey + sbase + keep + threadIdx.x, ckey[threadIdx.x]);
}

// The partner named by a key of a tile kernel that records only a lane's
// group of G <= 16 consecutive diagonals: the candidates are p0 + dir q,
// q < G (dir = +1: row key, partners above; -1: column key, partners below).
// Each admissible candidate (a window of the column series, at least pexcl
// from x, with finite statistics, and at or after `keep` when x is an old
// window of an append) is scored by the exact FP64 correlation of the centred
// windows; a flat candidate scores the flat distance sqrt(m).  The best
// squared distance wins, ties to the smaller index; -1 if none is admissible.
// The 16 correlations are one sliding product: the partner samples pass
// through a ring of 16 registers, each sample loaded once.  Buffer loads
// (global only, so they stay in flight across the LDS reads of the window's
// own samples) read zeros past the column series' end: candidates there are
// discarded.  The 16 scored positions start at the group's first candidate
// or at 0, whichever is larger, so no offset is ever negative: the compiler
// folds parts of an index into the loads' immediate offsets, and a negative
// register offset fails the buffer's range check even where the immediate
// brings the sum back into range.
__device__ int64_t best_in_group(const double* wx, double mx, double ix, const double* rc, int64_t cn,
                                 const double* cmu, const double* cinvn, int64_t n_cols, int64_t x, int64_t p0, int dir,
                                 int G, int pexcl, int64_t keep, int m, double& d2_best) {
  const int64_t glo = dir > 0 ? p0 : p0 - (G - 1), ghi = glo + G - 1;  // the group's candidates
  const int64_t lo = glo < 0 ? 0 : glo;
  const __amdgpu_buffer_rsrc_t yr = __builtin_amdgcn_make_buffer_rsrc((void*)rc, 0, (int)(cn * 8), kBufWord3);
  auto sample = [&](int64_t i) -> double {  // i >= 0
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(yr, (int)i * 8, 0, 0));
  };
  const double shift = sample(p0 < 0 ? 0 : (p0 >= cn ? cn - 1 : p0));
  double yw[16], acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    yw[q] = sample(lo + q) - shift;
    acc[q] = 0.0;
  }
  double se = 0.0;
  // no branches inside a block of 16 samples (past m the window's samples
  // read as zero: the stage holds 16 zeros after the last window), so each
  // load has a whole block of products to arrive
  for (int s0 = 0; s0 < m; s0 += 16) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int sidx = s0 + u;
      const double e = sidx < m ? wx[sidx] - mx : 0.0;
      se += e;
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = fma(e, yw[(q + u) & 15], acc[q]);
      yw[u] = sample(lo + sidx + 16) - shift;  // slot u next holds sample lo + s + 16
    }
  }
  const __amdgpu_buffer_rsrc_t ir = __builtin_amdgcn_make_buffer_rsrc((void*)cinvn, 0, (int)(n_cols * 8), kBufWord3);
  const __amdgpu_buffer_rsrc_t mr = __builtin_amdgcn_make_buffer_rsrc((void*)cmu, 0, (int)(n_cols * 8), kBufWord3);
  int64_t arg = -1;
  double best = INFINITY;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int64_t p = lo + q;
    const double ip = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(ir, (int)p * 8, 0, 0));
    const double mp = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(mr, (int)p * 8, 0, 0));
    const bool ok = p <= ghi && p < n_cols && (p > x ? p - x : x - p) >= pexcl && !(x < keep && p < keep) &&
                    !isnan(ip);
    const double rho = (acc[q] - (mp - shift) * se) * ix * ip;
    const double d2 = ip == 0.0 ? (double)m : 2.0 * m * (1.0 - rho);
    if (ok && d2 < best) {  // ascending p: a tie keeps the smaller index
      best = d2;
      arg = p;
    }
  }
  d2_best = best;
  return arg;
}

// Squared distances (in units of m) from which the FP32 keys' group search
// result is reported directly; nearer partners get the explicit-difference
// distance, which keeps full precision down to d = 0.
constexpr double kPolishFromCorr = 0.01;

__global__ __launch_bounds__(256) void merge_kernel(SJState st) {
  // samples [x0, x0 + 256 + m - 1) of the chunk (the block's own windows),
  // then 16 zeros read by the group search past the last window's samples
  extern __shared__ double sh_w[];
  const ChunkPos c = decode_chunk(st, blockIdx.x);
  const SeriesPlan& sp = st.plan[c.s];
  if (sp.p0 == nullptr) return;  // this series' profile is not wanted
  const int64_t x = c.x0 + threadIdx.x;
  const int m = st.m;
  const int g = st.groups.g[c.gi];
  const double* r = sp.r0 + (int64_t)g * sp.ldr;
  for (int q = threadIdx.x; q < 256 + m - 1 + 16; q += 256) {
    const int64_t t = c.x0 + q;
    sh_w[q] = (q < 256 + m - 1 && t >= 0 && t < sp.n) ? r[t] : 0.0;
  }
  __syncthreads();
  if (x < 0 || x >= sp.n_sub) return;
  // partners are windows of the column series cs (this series in a self-join)
  const int pexcl = sp.pexcl;
  const int64_t n_cols = sp.n_cols;
  const SeriesPlan& cp = st.plan[sp.cs];
  const int64_t sbase = (int64_t)c.gi * st.gstride + sp.stat_base + PADL;
  const int64_t cbase = (int64_t)c.gi * st.gstride + sp.cstat_base + PADL;
  const double* invn = st.invn + sbase;
  const double* mu = st.mu + sbase;
  const double* cinvn = st.invn + cbase;
  const double* cmu = st.mu + cbase;
  const double* rc = sp.cr0 + (int64_t)g * sp.cldr;
  const unsigned long long GMAX = (1ull << st.key_bits) - 1;
  if (isnan(invn[x])) {
    // a window whose sketched samples are not finite (non-finite input): it
    // has no distance to anything; P = NaN marks it (no admissible partner
    // is +inf), and the tile kernels never paired it with another window
    sp.p0[(int64_t)g * sp.ldp + x] = __longlong_as_double(0x7FF8000000000000ll);
    sp.i0[(int64_t)g * sp.ldp + x] = -1;
    return;
  }
  const unsigned long long rk = st.rowkey[sbase + x], ck = st.colkey[sbase + x];
  int64_t partner = -1;
  int dir = 0;
  if (ck != 0ull && ck >= rk) {
    partner = x - (int64_t)(GMAX - (ck & GMAX));
    dir = -1;
  } else if (rk != 0ull) {
    partner = x + (int64_t)(GMAX - (rk & GMAX));
    dir = 1;
  }
  // an append's old window whose new candidate, judged by its key, cannot
  // beat the stored distance keeps it without a polish (nor, for grouped
  // keys, the search of the group).  Appends run in FP64 or FP32: the FP32
  // keys resolve 1 - rho to better than 1.2e-4 relative plus 1.2e-7
  // absolute, the FP64 keys far better; a flat partner is covered by the
  // flat-window rule below.
  bool worse = false;
  if (dir != 0 && x < sp.keep && invn[x] != 0.0 && (st.kgroup > 1 || cinvn[partner] != 0.0)) {
    const unsigned long long kk = dir < 0 ? ck : rk;
    const double rho = __longlong_as_double((long long)(kk & ~GMAX)) - 2.0;
    const double d2 = 2.0 * m * (1.0 - rho);
    const double po = sp.p0[(int64_t)g * sp.ldp + x];
    worse = d2 > po * po * (1.0 + 1e-3) + 2e-4 * m;
  }
  double d2_group = -1.0;  // the group search's squared distance of its choice (-1: no search)
  if (!worse && st.kgroup > 1 && dir != 0 && invn[x] != 0.0)
    partner = best_in_group(sh_w + threadIdx.x, mu[x], invn[x], rc, sp.cn, cmu, cinvn, n_cols, x, partner, dir,
                            st.kgroup, pexcl, sp.keep, m, d2_group);

  const double sqrt_m = sqrt((double)m);
  const int64_t sg = (int64_t)sp.cs * st.groups.count + c.gi;
  const int32_t ff = st.flat_first[sg], fl = st.flat_last[sg];
  const int32_t* fblk = st.flat_blk + (int64_t)c.gi * st.blk_stride + cp.blk_base;
  const bool xflat = invn[x] == 0.0;

  // smallest admissible flat partner (|j - x| >= pexcl), -1 if none
  int64_t jf = -1;
  if (ff != INT_MAX) {
    if ((int64_t)ff <= x - pexcl) jf = ff;
    else jf = smallest_flat_at_or_after(st, cinvn, fblk, x + pexcl, fl);
  }

  double best;
  int64_t arg;
  if (xflat) {
    if (jf >= 0) {
      best = 0.0;
      arg = jf;
    } else {
      arg = (x >= pexcl) ? 0 : ((x + pexcl < n_cols) ? x + pexcl : -1);
      best = (arg >= 0) ? sqrt_m : INFINITY;
    }
  } else {
    best = INFINITY;
    arg = -1;
    if (partner >= 0 && !worse) {
      if (cinvn[partner] == 0.0) {
        best = sqrt_m;
      } else if (d2_group >= kPolishFromCorr * m) {
        // the group search scored the partner by its exact FP64 centred
        // correlation: d^2 = 2 m (1 - rho) carries an absolute error of about
        // m eps (|e| / sigma) (|y| / sigma) in d^2, below 1e-10 in d this far
        // from zero, so the explicit-difference pass is not repeated
        best = sqrt(fmin(d2_group, 4.0 * m));
      } else {
        // exact distance from explicit differences of the normalised windows
        const double ax = invn[x] * sqrt_m, ap = cinvn[partner] * sqrt_m;
        const double mx = mu[x], mp = cmu[partner];
        // the window itself comes from LDS, the partner's is gathered; four
        // independent partial sums keep several gathers in flight
        const double* wx = sh_w + threadIdx.x;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        int q = 0;
        for (; q + 4 <= m; q += 4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double e = (wx[q + u] - mx) * ax - (rc[partner + q + u] - mp) * ap;
            acc[u] = fma(e, e, acc[u]);
          }
        }
        for (; q < m; ++q) {
          const double e = (wx[q] - mx) * ax - (rc[partner + q] - mp) * ap;
          acc[0] = fma(e, e, acc[0]);
        }
        best = sqrt((acc[0] + acc[1]) + (acc[2] + acc[3]));
      }
      arg = partner;
    }
    if (jf >= 0 && (sqrt_m < best || (sqrt_m == best && jf < arg))) {
      best = sqrt_m;
      arg = jf;
    }
  }
  double* pdst = sp.p0 + (int64_t)g * sp.ldp + x;
  int64_t* idst = sp.i0 + (int64_t)g * sp.ldp + x;
  if (x < sp.keep) {
    // an append: the stored entry covers every partner before the new
    // samples; the new candidate replaces it only if strictly nearer, or
    // equally near with a smaller index (flat windows: the smallest flat
    // partner, as in a join of the whole series)
    const double pold = *pdst;
    const int64_t iold = *idst;
    if (!(best < pold || (best == pold && arg >= 0 && (iold < 0 || arg < iold)))) return;
  }
  *pdst = best;
  *idst = arg;
}

// ------------------------------------------------------------------ host
struct PlanInfo {
  std::vector<SeriesPlan> sp;
  int64_t gstride = 0, total_units_per_group = 0, total_chunks_per_group = 0, blk_stride = 0;
  int64_t total_units = 0, total_chunks = 0;
  int key_bits = 0;
};

// C > 0: diagonal kernels (bands of 64 C diagonals x strips of `strip` rows);
// C = 0: MFMA tiles (row panels of MFMA_TILE rows x segments of MFMA_SEG column tiles).
// ab = false: every series is joined with itself from diagonal excl on.
// ab = true: the two series of an AB-join (0 = A, 1 = B): A's units cover the
// diagonals j - i >= 0 of A x B, B's units the diagonals >= 1 of B x A, so
// every pair is met once and there is no trivial-match zone.
// keep (diagonal kernels only; NULL: none): per series, the windows whose
// profile entries already cover every partner below that index (an append).
// Only pairs with a column at or after keep are new; a band reaches such a
// column first at step keep - db - 64 (C - 1) (lane t, diagonal q of the band
// at step u is on column u + db + t (C - 1) + q), so its walk starts there
// and the few older cells it passes again are merged harmlessly.  A series
// with keep = its window count has nothing new: no units, no merge.
static int make_plan(int64_t n_series, const int64_t* offsets, int32_t m, int32_t excl, int kact, int C, int strip,
                     PlanInfo& pl, bool validate, bool ab = false, const int64_t* keep = nullptr) {
  // de-interleave stride of the column statistics (diagonal kernels); the
  // MFMA forms read natural layouts only (8 keeps their rows 32-byte aligned)
  const int cs = C > 0 ? C - 1 : (C < 0 ? 8 : 7);
  pl.sp.assign(n_series, SeriesPlan{});
  int64_t stat = 0, chunk = 0, blk = 0, max_nsub = 1;
  for (int64_t s = 0; s < n_series; ++s) {
    SeriesPlan& p = pl.sp[s];
    p.col = offsets[s];
    p.n = offsets[s + 1] - offsets[s];
    if (validate && p.n < m) {
      set_error("series " + std::to_string(s) + " is shorter than m");
      return SKMP_EINVAL;
    }
    p.n_sub = std::max<int64_t>(p.n - m + 1, 1);
    max_nsub = std::max(max_nsub, p.n_sub);
    p.stat_base = stat;
    p.lpad = ((p.n_sub + PADL + PADR + cs - 1) / cs) * cs;
    stat += p.lpad;
    p.chunk_base = chunk;
    chunk += ((p.lpad + 255) / 256) * kact;
    p.blk_base = blk;
    blk += (p.n_sub + 255) / 256;
    p.cs = ab ? (int32_t)(1 - s) : (int32_t)s;
    p.d0 = ab ? (int32_t)s : excl;
    p.pexcl = ab ? 0 : excl;
    p.keep = (keep && C > 0) ? std::min<int64_t>(std::max<int64_t>(keep[s], 0), p.n - m + 1) : 0;
    p.c0 = p.keep > 0 ? (int32_t)std::max<int64_t>(p.keep - 64 * (int64_t)(C - 1), 0) : 0;
  }
  int64_t unit = 0;
  for (int64_t s = 0; s < n_series; ++s) {
    SeriesPlan& p = pl.sp[s];
    const SeriesPlan& q = pl.sp[p.cs];
    p.n_cols = q.n_sub;
    p.cn = q.n;
    p.cstat_base = q.stat_base;
    p.clpad = q.lpad;
    const int64_t nd = p.n_cols - p.d0;  // diagonals with pairs
    if (C > 0) {
      const int64_t D = 64 * (int64_t)C;
      // steps of the first band (no later band walks more)
      const int64_t rows = std::min<int64_t>(p.n_sub + 63, p.n_cols - p.d0) - std::max<int64_t>(p.c0 - p.d0, 0);
      const bool fresh = p.keep < p.n - m + 1;  // false: an append with no new window
      p.nb = (nd > 0 && fresh && rows > 0) ? (int32_t)((nd + D - 1) / D) : 0;
      p.ns = (nd > 0 && fresh && rows > 0) ? (int32_t)((rows + strip - 1) / strip) : 0;
    } else if (C < 0) {
      // blocked MFMA form: units of BLK_DIAGS diagonals x BLK_UNIT_ROWS rows
      const int64_t rows = std::min<int64_t>(p.n_sub, p.n_cols - p.d0);
      p.nb = (nd > 0 && rows > 0) ? (int32_t)((nd + BLK_DIAGS - 1) / BLK_DIAGS) : 0;
      p.ns = (nd > 0 && rows > 0) ? (int32_t)((rows + BLK_UNIT_ROWS - 1) / BLK_UNIT_ROWS) : 0;
    } else {
      const int64_t jt_last = (p.n_sub - 1) / MFMA_TILE;
      const int64_t nt0 = jt_last - (int64_t)excl / MFMA_TILE + 1;  // tiles of row panel 0
      p.nb = nd > 0 ? (int32_t)((p.n_sub + MFMA_TILE - 1) / MFMA_TILE) : 0;
      p.ns = nd > 0 ? (int32_t)((nt0 + MFMA_SEG - 1) / MFMA_SEG) : 0;
    }
    p.unit_base = unit;
    unit += (int64_t)p.nb * p.ns * kact;
  }
  pl.gstride = stat;
  pl.total_units = unit;
  pl.total_chunks = chunk;
  pl.blk_stride = blk;
  int bits = 1;
  while ((1ll << bits) <= max_nsub) ++bits;
  pl.key_bits = std::max(bits, 11);
  return SKMP_OK;
}

struct SJBuffers {
  SeriesPlan* plan;
  double2* dfdg;
  double* invn;
  double2* cdfdg;
  double* cinvn;
  float2* fdfdg = nullptr;
  float* finvn = nullptr;
  float2* fcdfdg = nullptr;
  float* fcinvn = nullptr;
  uint16_t* bplanes = nullptr;
  double* mu;
  unsigned long long* rowkey;
  unsigned long long* colkey;
  double* scale;
  int32_t* flat_first;
  int32_t* flat_last;
  int32_t* flat_blk;
  unsigned int* counter;
};

// blocked: the blocked MFMA form (16-bit operand planes + FP32 window norms)
static void carve_sj(Carve& cv, const PlanInfo& pl, int64_t n_series, int kact, int prec, SJBuffers& b,
                     bool blocked = false) {
  const size_t cells = (size_t)kact * (size_t)pl.gstride;
  if (prec == SKMP_FP32) {
    b.fdfdg = cv.take<float2>(cells);
    b.finvn = cv.take<float>(cells);
    b.fcdfdg = cv.take<float2>(cells);
    b.fcinvn = cv.take<float>(cells);
  }
  if (blocked) {
    b.finvn = cv.take<float>(cells);
    b.bplanes = cv.take<uint16_t>(8 * cells);
  }
  b.plan = cv.take<SeriesPlan>(n_series);
  b.dfdg = cv.take<double2>(cells);
  b.invn = cv.take<double>(cells);
  b.cdfdg = cv.take<double2>(cells);
  b.cinvn = cv.take<double>(cells);
  b.mu = cv.take<double>(cells);
  b.rowkey = cv.take<unsigned long long>(cells);
  b.colkey = cv.take<unsigned long long>(cells);
  b.scale = cv.take<double>((size_t)n_series * kact);
  b.flat_first = cv.take<int32_t>((size_t)n_series * kact);
  b.flat_last = cv.take<int32_t>((size_t)n_series * kact);
  b.flat_blk = cv.take<int32_t>((size_t)kact * (size_t)pl.blk_stride);
  b.counter = cv.take<unsigned int>(64);
}

// tile configuration of the FP64 kernel
constexpr int DEFAULT_STRIP = 2048;
// Default FP32 refresh period: at least 256 rows and at least 2.5 m (rounded up
// to 256), so the exact seeds (m FP64 FMAs per diagonal per period) stay near
// 0.4 FMA per cell whatever the window length.
static inline int default_refresh(int m) { return std::max(256, ((5 * m / 2 + 255) / 256) * 256); }

// Compiled variants of the FP64 tile kernel: diagonals per lane C, prefetch
// depth PD and the waves-per-SIMD occupancy the register allocation is held to.
struct Fp64Variant {
  const char* name;
  int C;
  const void* fn;
  void (*launch)(dim3 grid, hipStream_t st, const SJState& s);
  int group;  // diagonals a local key names (0 or 1: its own)
};

// tile length: the largest multiple of C not above 256
constexpr int tl_for(int C) { return 256 - 256 % C; }

template <int C, int PD, int WPE, bool CL>
static void launch_fp64(dim3 grid, hipStream_t st, const SJState& s) {
  hipLaunchKernelGGL((sj_fp64_kernel<C, tl_for(C), PD, WPE, CL>), grid, dim3(64), 0, st, s);
}

#define SKMP_FP64_V(C, PD, WPE, CL)                                                                 \
  {                                                                                                 \
    "c" #C "_pd" #PD "_w" #WPE "_cl" #CL, C,                                                        \
        reinterpret_cast<const void*>(&sj_fp64_kernel<C, tl_for(C), PD, WPE, CL>), &launch_fp64<C, PD, WPE, CL> \
  }
static const Fp64Variant kFp64Variants[] = {
    SKMP_FP64_V(8, 1, 2, false), SKMP_FP64_V(8, 1, 2, true),  SKMP_FP64_V(8, 2, 2, true),
    SKMP_FP64_V(10, 1, 2, true), SKMP_FP64_V(12, 1, 2, true), SKMP_FP64_V(6, 1, 3, true),
    SKMP_FP64_V(8, 1, 3, true),  SKMP_FP64_V(16, 1, 2, true), SKMP_FP64_V(8, 1, 3, false), SKMP_FP64_V(2, 1, 4, false),
    SKMP_FP64_V(4, 1, 3, false), SKMP_FP64_V(8, 2, 2, false),
};
#undef SKMP_FP64_V
constexpr int kNumFp64Variants = sizeof(kFp64Variants) / sizeof(kFp64Variants[0]);

template <int C, int PD, int WPE>
static void launch_fp32(dim3 grid, hipStream_t st, const SJState& s) {
  hipLaunchKernelGGL((sj_fp32_kernel<C, tl_for(C), PD, WPE>), grid, dim3(64), 0, st, s);
}

#define SKMP_FP32_V(C, PD, WPE)                                                                              \
  {                                                                                                          \
    "f32_c" #C "_pd" #PD "_w" #WPE, C, reinterpret_cast<const void*>(&sj_fp32_kernel<C, tl_for(C), PD, WPE>), \
        &launch_fp32<C, PD, WPE>, C                                                                          \
  }
static const Fp64Variant kFp32Variants[] = {
    SKMP_FP32_V(8, 1, 2), SKMP_FP32_V(16, 1, 2), SKMP_FP32_V(8, 1, 3), SKMP_FP32_V(12, 1, 2), SKMP_FP32_V(8, 2, 3),
    SKMP_FP32_V(16, 2, 2), SKMP_FP32_V(16, 1, 3), SKMP_FP32_V(16, 2, 3), SKMP_FP32_V(2, 2, 4),
    SKMP_FP32_V(4, 2, 4), SKMP_FP32_V(16, 2, 4),
};
#undef SKMP_FP32_V
constexpr int kNumFp32Variants = sizeof(kFp32Variants) / sizeof(kFp32Variants[0]);

// Forms of the 16-bit split-precision join (BF16x3 / FP16x3): C = 0 the
// Hankel-direct tiles (selfjoin_mixed.hip), C < 0 the blocked recurrence
// (selfjoin_blocked.hip) with -C = 10 x (tiles per band) + (waves per SIMD).
// Measured on the water-treatment join (BF16x3, refresh 256): 8 tiles at 2
// waves per SIMD (215 VGPRs) 2.81 ms; 4 tiles at 3 waves (135 VGPRs, all
// codes inline constants) 3.61 ms: the row reductions over fewer tiles cost
// more than the occupancy returns; 8 tiles held to 3 waves spill (5.3 ms).
static const Fp64Variant kMixedVariants[] = {{"hankel", 0, nullptr, nullptr},
                                             {"blocked_w2", -82, nullptr, nullptr},
                                             {"blocked_nb4_w3", -43, nullptr, nullptr}};
constexpr int kNumMixedVariants = sizeof(kMixedVariants) / sizeof(kMixedVariants[0]);
constexpr int kDefaultMixedVariant = 1;
constexpr int kHankelVariant = 0;

// Refresh period of the blocked form: the largest of 128, 256, 512, 1024 rows
// not above `refresh`; 0: the smallest of 256, 512, 1024 that is at least
// 4 m (1024 above m = 256), so the exact FP64 seeds (m FP64 FMAs per diagonal
// per period) stay near a quarter FMA per cell.  Measured: transportation
// (m = 288) 39.1 ms at 256 rows, 33.6 at 512, 30.7 at 1024 (FP64 path 41 ms);
// the error against the FP64 path stays at 6-7e-4 (it comes from the 16-bit
// operands, not from the walk's length).  Periods must be multiples of 16
// BLK_NB that divide the unit's BLK_UNIT_ROWS.
static int blk_period(int refresh, int m) {
  if (refresh <= 0) return 4 * m <= 256 ? 256 : (4 * m <= 512 ? 512 : 1024);
  int p = 128;
  while (p * 2 <= refresh && p * 2 <= BLK_UNIT_ROWS) p *= 2;
  return p;
}

// ------------------------------------------------------------- tuning
// Launch configuration of a self-join: the tile-kernel variant and the strip
// (rows per work unit).  Chosen, in this order, by SKMP_FP64_VARIANT /
// SKMP_FP32_VARIANT / SKMP_STRIP (sweeps), by the autotuned table (entries
// keyed by precision and the log2 buckets of m and of the longest series'
// window count), or by the built-in defaults.  FP32 units restart from an
// exact FP64 seed, so their strip is always the refresh period.
constexpr int kDefaultFp64Variant = 11;  // C = 8, prefetch 2, register column windows (fastest measured)
// C = 16, prefetch 2, 4 waves per SIMD (128 VGPRs, the spills outside the step
// loop; 10 KB LDS): 2 % faster than 3 waves per SIMD on the water-treatment
// join, 1 % on long series (measured)
constexpr int kDefaultFp32Variant = 10;
static const int kTuneStrips[] = {1024, 2048, 4096};
// The narrowest bands (C = 6 in FP64, C = 8 in FP32), for short appends.
constexpr int kNarrowFp64Variant = 5;
constexpr int kNarrowFp32Variant = 4;

struct TuneKey {
  int prec, mlog, nlog;
  int m;  // not part of the class (ordering ignores it)
  bool operator<(const TuneKey& o) const {
    return prec != o.prec ? prec < o.prec : (mlog != o.mlog ? mlog < o.mlog : nlog < o.nlog);
  }
};
struct TuneChoice {
  int variant, strip;
  double ms;
};
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneChoice> g_tune;

static int ceil_log2(int64_t x) {
  int b = 0;
  while ((1ll << b) < x) ++b;
  return b;
}

static TuneKey tune_key(int prec, int m, int64_t n_series, const int64_t* offsets) {
  int64_t nmax = 1;
  for (int64_t s = 0; s < n_series; ++s) nmax = std::max<int64_t>(nmax, offsets[s + 1] - offsets[s] - m + 1);
  return TuneKey{prec, ceil_log2(m), ceil_log2(nmax), m};
}

static int env_int(const char* name, int lo, int hi) {
  const char* e = getenv(name);
  if (!e) return -1;
  const int v = atoi(e);
  return (v >= lo && v <= hi) ? v : -1;
}

static const Fp64Variant* variants_of(int prec, int* count) {
  if (prec == SKMP_FP32) {
    *count = kNumFp32Variants;
    return kFp32Variants;
  }
  if (prec == SKMP_BF16X3 || prec == SKMP_FP16X3) {
    *count = kNumMixedVariants;
    return kMixedVariants;
  }
  *count = kNumFp64Variants;
  return kFp64Variants;
}

static void tuning_file_autoload();

static void select_config(int prec, int refresh, const TuneKey& key, int* vidx, int* strip) {
  tuning_file_autoload();
  static const int env64 = env_int("SKMP_FP64_VARIANT", 0, kNumFp64Variants - 1);
  static const int env32 = env_int("SKMP_FP32_VARIANT", 0, kNumFp32Variants - 1);
  static const int envmx = env_int("SKMP_MIXED_VARIANT", 0, kNumMixedVariants - 1);
  static const int env_strip = env_int("SKMP_STRIP", 256, 1 << 20);
  if (prec == SKMP_BF16X3 || prec == SKMP_FP16X3) {
    // a refresh period below the blocked form's shortest (128 rows) asks for
    // more exactness than its walk gives: the Hankel-direct tiles (no walk)
    int v = (refresh > 0 && refresh < 128) ? kHankelVariant : kDefaultMixedVariant;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end() && !(refresh > 0 && refresh < 128)) v = it->second.variant;
    }
    if (envmx >= 0) v = envmx;
    *vidx = v;
    *strip = blk_period(refresh, key.m);
    return;
  }
  int v = (prec == SKMP_FP32) ? kDefaultFp32Variant : kDefaultFp64Variant;
  int sp = DEFAULT_STRIP;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      v = it->second.variant;
      sp = it->second.strip;
    }
  }
  const int env_v = (prec == SKMP_FP32) ? env32 : env64;
  if (env_v >= 0) v = env_v;
  if (env_strip > 0) sp = env_strip;
  if (prec == SKMP_FP32) sp = refresh > 0 ? refresh : default_refresh(key.m);
  *vidx = v;
  *strip = sp;
}

static int grid_for(const void* kernel, int block, size_t lds) {
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) ncu = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess || per_cu < 1) per_cu = 4;
  return ncu * per_cu;
}

}  // namespace skmp

using namespace skmp;

// k <= 64: the groups whose bit is set in group_mask.
static int active_groups(int32_t k, uint64_t group_mask, GroupList& gl) {
  gl.count = 0;
  for (int g = 0; g < k; ++g)
    if ((group_mask >> g) & 1ull) gl.g[gl.count++] = (int8_t)g;
  return gl.count;
}

extern "C" size_t mp_selfjoin_workspace(int64_t n_series, const int64_t* offsets, int32_t k, int32_t m,
                                        int32_t prec) {
  if (n_series < 1 || !offsets || k < 1 || k > MAX_GROUPS || m < 4) return 0;
  k = std::min(k, 64);  // more groups run in blocks of 64 through the same workspace
  const bool mfma = (prec == SKMP_BF16X3 || prec == SKMP_FP16X3);
  int nv = 0;
  const Fp64Variant* vs = variants_of(prec, &nv);
  size_t need = 0;
  // the largest over the compiled variants, so a tuned choice always fits
  for (int v = 0; v < nv; ++v) {
    PlanInfo pl;
    if (make_plan(n_series, offsets, m, std::max(1, m / 4), k, vs[v].C, DEFAULT_STRIP, pl, false) != SKMP_OK)
      return 0;
    Carve cv(nullptr, 0);
    SJBuffers b;
    carve_sj(cv, pl, n_series, k, prec, b, mfma && vs[v].C < 0);
    need = std::max(need, cv.used + 256);
  }
  return need;
}

static int validate_selfjoin(const double* R, int64_t ldr, int64_t n_series, const int64_t* offsets, int32_t k,
                             int32_t m, int32_t excl, int32_t prec, int32_t refresh, double* P, int64_t* I,
                             int64_t ldp) {
  SKMP_REQUIRE(R && P && I && offsets, "null pointer argument");
  SKMP_REQUIRE(n_series >= 1 && n_series < (1 << 30), "n_series out of range");
  SKMP_REQUIRE(k >= 1 && k <= MAX_GROUPS, "k must lie in [1, 128]");
  SKMP_REQUIRE(m >= 4 && m <= 2048, "m must lie in [4, 2048]");
  SKMP_REQUIRE(excl >= 1, "excl must be >= 1 (a subsequence is its own trivial match)");
  SKMP_REQUIRE(prec >= SKMP_FP64 && prec <= SKMP_FP16X3, "unknown precision");
  SKMP_REQUIRE(refresh == 0 || (refresh >= 64 && refresh <= (1 << 20)), "refresh must be 0 or in [64, 2^20]");
  SKMP_REQUIRE(offsets[0] == 0, "offsets[0] must be 0");
  for (int64_t s = 0; s < n_series; ++s) SKMP_REQUIRE(offsets[s + 1] >= offsets[s], "offsets must be non-decreasing");
  const int64_t N = offsets[n_series];
  SKMP_REQUIRE(ldr >= N && ldp >= N, "row strides must be >= the total number of samples");
  for (int64_t s = 0; s < n_series; ++s)
    SKMP_REQUIRE(offsets[s + 1] - offsets[s] <= MAX_SERIES_LEN, SERIES_TOO_LONG);
  const bool mfma = (prec == SKMP_BF16X3 || prec == SKMP_FP16X3);
  SKMP_REQUIRE(!mfma || m <= 1024, "the BF16x3 / FP16x3 self-join supports m <= 1024");
  return SKMP_OK;
}

// Where a series' sketch rows are read and its profile rows written.
struct JoinIO {
  const double* r0;
  int64_t ldr;
  double* p0;  // NULL: not written
  int64_t* i0;
  int64_t ldp;
};

// Everything after validation, with an explicit launch configuration: the
// self-join of every series (ab = false) or the AB-join of series 0 and 1.
// keep: as in make_plan (an append), NULL otherwise.
static int run_join(int64_t n_series, const int64_t* offsets, bool ab, const JoinIO* io, int32_t m, int32_t excl,
                    int32_t prec, const GroupList& gl, void* workspace, size_t ws_bytes, hipStream_t st,
                    const Fp64Variant& var, int strip, const int64_t* keep = nullptr) {
  const bool mfma = (prec == SKMP_BF16X3 || prec == SKMP_FP16X3);
  const bool blocked = mfma && var.C < 0;
  const int kact = gl.count;
  PlanInfo pl;
  int rc = make_plan(n_series, offsets, m, excl, kact, mfma ? std::min(var.C, 0) : var.C, strip, pl, true, ab, keep);
  if (rc) return rc;
  // the persistent kernels number their units with 32-bit queue entries (one
  // past the last is read by every block of the grid before it stops)
  if (pl.total_units > (int64_t)UINT32_MAX - (1 << 20)) {
    set_error("the join needs " + std::to_string(pl.total_units) +
              " work units, more than 2^32 - 2^20: split the groups over calls (group_mask) or raise refresh");
    return SKMP_EINVAL;
  }
  for (int64_t q = 0; q < n_series; ++q) {
    SeriesPlan& p = pl.sp[q];
    p.r0 = io[q].r0;
    p.ldr = io[q].ldr;
    p.p0 = io[q].p0;
    p.i0 = io[q].i0;
    p.ldp = io[q].ldp;
    p.cr0 = io[p.cs].r0;
    p.cldr = io[p.cs].ldr;
  }
  Carve cv(workspace, ws_bytes);
  SJBuffers b;
  carve_sj(cv, pl, n_series, kact, prec, b, blocked);
  if (!workspace || !cv.fits()) {
    set_error("workspace too small: need " + std::to_string(cv.used) + " bytes");
    return SKMP_ENOMEM;
  }
  if (int rc = upload_async(b.plan, pl.sp.data(), sizeof(SeriesPlan) * n_series, st)) return rc;

  SJState s;
  s.plan = b.plan;
  s.n_series = (int32_t)n_series;
  s.m = m;
  s.excl = excl;
  s.key_bits = pl.key_bits;
  s.gstride = pl.gstride;
  s.groups = gl;
  s.dfdg = b.dfdg;
  s.invn = b.invn;
  s.cdfdg = b.cdfdg;
  s.cinvn = b.cinvn;
  s.cstride = mfma ? (blocked ? 8 : 7) : var.C - 1;
  s.bplanes = b.bplanes;
  s.bprec = prec;
  s.fdfdg = b.fdfdg;
  s.finvn = b.finvn;
  s.fcdfdg = b.fcdfdg;
  s.fcinvn = b.fcinvn;
  s.mu = b.mu;
  s.scale = b.scale;
  s.rowkey = b.rowkey;
  s.colkey = b.colkey;
  s.flat_first = b.flat_first;
  s.flat_last = b.flat_last;
  s.flat_blk = b.flat_blk;
  s.blk_stride = pl.blk_stride;
  s.counter = b.counter;
  s.total_units = pl.total_units;
  s.total_chunks = pl.total_chunks;
  s.strip = strip;
  s.kgroup = 1;

  const dim3 fb(256);
  {
    const int64_t n_sg = (int64_t)n_series * kact, n_blk = (int64_t)kact * pl.blk_stride;
    const int64_t big = std::max<int64_t>(std::max<int64_t>(n_sg, n_blk), 64);
    hipLaunchKernelGGL(init_small, dim3((unsigned)std::min<int64_t>((big + 255) / 256, 4096)), fb, 0, st, s, n_sg,
                       n_blk);
  }
  SKMP_CHECK_HIP(hipGetLastError());

  // a short append: every series has at most append_direct_max(m) new windows
  // (SKMP_APPEND_DIRECT overrides the limit, 0 turns the direct kernel off)
  static const int env_direct = env_int("SKMP_APPEND_DIRECT", 0, APPEND_DIRECT);
  const int direct_max = env_direct >= 0 ? env_direct : append_direct_max(m);
  bool direct = keep != nullptr && !mfma && direct_max > 0;
  for (int64_t q = 0; direct && q < n_series; ++q)
    if (pl.sp[q].n_sub - pl.sp[q].keep > direct_max) direct = false;
  // the direct kernel, the MFMA tiles and the merge read only mu and invn
  s.walk_stats = (mfma || direct) ? 0 : 1;

  const dim3 cg((unsigned)pl.total_chunks);
  {
    StageTimer tm(SKMP_TIMER_SUBSTATS, st);
    hipLaunchKernelGGL(scale_kernel, dim3((unsigned)((pl.total_chunks + SCALE_CHUNKS - 1) / SCALE_CHUNKS)), fb, 0, st,
                       s);
    hipLaunchKernelGGL(substats_kernel, cg, fb, sizeof(double) * (256 + m + 1 + 256), st, s);
  }
  SKMP_CHECK_HIP(hipGetLastError());

  if (direct) {
    StageTimer tm(SKMP_TIMER_TILES, st);
    hipLaunchKernelGGL(append_direct_kernel, cg, fb, sizeof(double) * (256 + m - 1 + APPEND_DIRECT + m - 1 + 3), st,
                       s);
  } else if (pl.total_units > 0) {
    StageTimer tm(SKMP_TIMER_TILES, st);
    if (blocked) {
      rc = launch_sj_blk(prec, (-var.C) / 10, (-var.C) % 10, s, pl.total_units, st);
      if (rc) return rc;
    } else if (mfma) {
      rc = launch_sj_mfma(prec, s, pl.total_units, st);
      if (rc) return rc;
    } else {
      const int grid = (int)std::min<int64_t>(grid_for(var.fn, 64, 0), pl.total_units);
      var.launch(dim3(grid), st, s);
      if (var.group > 1) s.kgroup = var.group;  // its keys name a lane's group of diagonals
    }
  }
  SKMP_CHECK_HIP(hipGetLastError());
  {
    StageTimer tm(SKMP_TIMER_MERGE, st);
    hipLaunchKernelGGL(merge_kernel, cg, fb, sizeof(double) * (256 + m - 1 + 16), st, s);
  }
  SKMP_CHECK_HIP(hipGetLastError());
  return SKMP_OK;
}

static int run_selfjoin(const double* R, int64_t ldr, int64_t n_series, const int64_t* offsets, int32_t k, int32_t m,
                        int32_t excl, int32_t prec, const GroupList& gl, double* P, int64_t* I, int64_t ldp,
                        void* workspace, size_t ws_bytes, hipStream_t st, const Fp64Variant& var, int strip) {
  (void)k;
  std::vector<JoinIO> io((size_t)n_series);
  for (int64_t q = 0; q < n_series; ++q) io[q] = JoinIO{R + offsets[q], ldr, P + offsets[q], I + offsets[q], ldp};
  return run_join(n_series, offsets, false, io.data(), m, excl, prec, gl, workspace, ws_bytes, st, var, strip);
}

extern "C" int mp_selfjoin(const double* R, int64_t ldr, int64_t n_series, const int64_t* offsets, int32_t k,
                           int32_t m, int32_t excl, int32_t prec, int32_t refresh, uint64_t group_mask, double* P,
                           int64_t* I, int64_t ldp, void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  if (int rc = validate_selfjoin(R, ldr, n_series, offsets, k, m, excl, prec, refresh, P, I, ldp)) return rc;
  SKMP_REQUIRE(k <= 64 || group_mask == ~0ull, "with more than 64 groups every group is joined (group_mask = ~0)");
  int vidx = 0, strip = DEFAULT_STRIP;
  select_config(prec, refresh, tune_key(prec, m, n_series, offsets), &vidx, &strip);
  int nv = 0;
  const Fp64Variant* vs = variants_of(prec, &nv);
  // groups in blocks of at most 64 (one launch sequence each, in stream order
  // through the same workspace)
  for (int g0 = 0; g0 < k; g0 += 64) {
    const int kk = std::min(64, k - g0);
    const uint64_t mask = kk < 64 ? group_mask & ((1ull << kk) - 1) : group_mask;
    GroupList gl;
    if (active_groups(kk, mask, gl) == 0) continue;
    if (int rc = run_selfjoin(R + (int64_t)g0 * ldr, ldr, n_series, offsets, kk, m, excl, prec, gl,
                              P + (int64_t)g0 * ldp, I + (int64_t)g0 * ldp, ldp, workspace, ws_bytes,
                              static_cast<hipStream_t>(stream), vs[vidx], strip))
      return rc;
  }
  return SKMP_OK;
}

// ------------------------------------------------------------- AB-join
extern "C" size_t mp_abjoin_workspace(int64_t na, int64_t nb, int32_t k, int32_t m, int32_t prec) {
  if (na < 1 || nb < 1 || (prec != SKMP_FP64 && prec != SKMP_FP32)) return 0;
  const int64_t offs[3] = {0, na, na + nb};
  return mp_selfjoin_workspace(2, offs, k, m, prec);
}

extern "C" int mp_abjoin(const double* RA, int64_t lda, int64_t na, const double* RB, int64_t ldb, int64_t nb,
                         int32_t k, int32_t m, int32_t prec, int32_t refresh, uint64_t group_mask, double* PA,
                         int64_t* IA, int64_t ldpa, double* PB, int64_t* IB, int64_t ldpb, void* workspace,
                         size_t ws_bytes, void* stream) {
  clear_error();
  SKMP_REQUIRE(RA && RB && PA && IA, "null pointer argument");
  SKMP_REQUIRE((PB == nullptr) == (IB == nullptr), "PB and IB are given together or not at all");
  SKMP_REQUIRE(k >= 1 && k <= 64, "k must lie in [1, 64]");
  SKMP_REQUIRE(m >= 4 && m <= 2048, "m must lie in [4, 2048]");
  SKMP_REQUIRE(prec == SKMP_FP64 || prec == SKMP_FP32, "the AB-join runs in FP64 or FP32 (with FP64 refresh)");
  SKMP_REQUIRE(refresh == 0 || (refresh >= 64 && refresh <= (1 << 20)), "refresh must be 0 or in [64, 2^20]");
  SKMP_REQUIRE(na >= m && nb >= m, "both series need at least m samples");
  SKMP_REQUIRE(na <= MAX_SERIES_LEN && nb <= MAX_SERIES_LEN, SERIES_TOO_LONG);
  SKMP_REQUIRE(lda >= na && ldb >= nb && ldpa >= na && (PB == nullptr || ldpb >= nb),
               "row strides must be >= the series lengths");
  if (k < 64) group_mask &= (1ull << k) - 1;
  GroupList gl;
  if (active_groups(k, group_mask, gl) == 0) return SKMP_OK;
  const int64_t offs[3] = {0, na, na + nb};
  int vidx = 0, strip = DEFAULT_STRIP;
  select_config(prec, refresh, tune_key(prec, m, 2, offs), &vidx, &strip);
  int nv = 0;
  const Fp64Variant* vs = variants_of(prec, &nv);
  const JoinIO io[2] = {JoinIO{RA, lda, PA, IA, ldpa}, JoinIO{RB, ldb, PB, IB, ldpb}};
  return run_join(2, offs, true, io, m, 0, prec, gl, workspace, ws_bytes, static_cast<hipStream_t>(stream), vs[vidx],
                  strip);
}

// ------------------------------------------------------------- streaming append
// Series s occupies columns [starts[s], starts[s] + n_new[s]) of R, P and I;
// the join sees the compact layout offs (series back to back) and reads and
// writes through per-series pointers.
static int append_layout(int64_t n_series, const int64_t* starts, const int64_t* n_old, const int64_t* n_new,
                         int32_t m, int64_t ldr, int64_t ldp, std::vector<int64_t>& offs, std::vector<int64_t>& keep,
                         int64_t* max_new_windows) {
  SKMP_REQUIRE(starts && n_old && n_new, "null pointer argument");
  offs.assign((size_t)n_series + 1, 0);
  keep.assign((size_t)n_series, 0);
  int64_t most = 0;
  for (int64_t s = 0; s < n_series; ++s) {
    SKMP_REQUIRE(n_new[s] >= m, "every series needs n_new >= m samples");
    SKMP_REQUIRE(n_old[s] >= 0 && n_old[s] <= n_new[s], "n_old must lie in [0, n_new]");
    SKMP_REQUIRE(n_new[s] <= MAX_SERIES_LEN, SERIES_TOO_LONG);
    SKMP_REQUIRE(starts[s] >= 0 && starts[s] + n_new[s] <= ldr && starts[s] + n_new[s] <= ldp,
                 "a series runs past the row stride");
    SKMP_REQUIRE(s == 0 || starts[s] >= starts[s - 1] + n_new[s - 1], "series must be ascending and disjoint");
    offs[s + 1] = offs[s] + n_new[s];
    keep[s] = n_old[s] >= m ? n_old[s] - m + 1 : 0;
    most = std::max<int64_t>(most, (n_new[s] - m + 1) - keep[s]);
  }
  *max_new_windows = most;
  return SKMP_OK;
}

// Appends of fewer new windows than this walk the narrowest compiled bands:
// a band passes 64 (C - 1) old steps before its last lane reaches a new column.
constexpr int64_t kAppendNarrowBelow = 2048;

extern "C" size_t mp_selfjoin_append_workspace(int64_t n_series, const int64_t* n_new, int32_t k, int32_t m,
                                               int32_t prec) {
  if (n_series < 1 || !n_new || (prec != SKMP_FP64 && prec != SKMP_FP32)) return 0;
  std::vector<int64_t> offs((size_t)n_series + 1, 0);
  for (int64_t s = 0; s < n_series; ++s) {
    if (n_new[s] < 1) return 0;
    offs[s + 1] = offs[s] + n_new[s];
  }
  return mp_selfjoin_workspace(n_series, offs.data(), k, m, prec);
}

extern "C" int mp_selfjoin_append(const double* R, int64_t ldr, int64_t n_series, const int64_t* starts,
                                  const int64_t* n_old, const int64_t* n_new, int32_t k, int32_t m, int32_t excl,
                                  int32_t prec, int32_t refresh, uint64_t group_mask, double* P, int64_t* I,
                                  int64_t ldp, void* workspace, size_t ws_bytes, void* stream) {
  clear_error();
  SKMP_REQUIRE(R && P && I, "null pointer argument");
  SKMP_REQUIRE(n_series >= 1 && n_series < (1 << 30), "n_series out of range");
  SKMP_REQUIRE(k >= 1 && k <= 64, "k must lie in [1, 64]");
  SKMP_REQUIRE(m >= 4 && m <= 2048, "m must lie in [4, 2048]");
  SKMP_REQUIRE(excl >= 1, "excl must be >= 1 (a subsequence is its own trivial match)");
  SKMP_REQUIRE(prec == SKMP_FP64 || prec == SKMP_FP32, "appends run in FP64 or FP32 (with FP64 refresh)");
  SKMP_REQUIRE(refresh == 0 || (refresh >= 64 && refresh <= (1 << 20)), "refresh must be 0 or in [64, 2^20]");
  std::vector<int64_t> offs, keep;
  int64_t most = 0;
  if (int rc = append_layout(n_series, starts, n_old, n_new, m, ldr, ldp, offs, keep, &most)) return rc;
  if (k < 64) group_mask &= (1ull << k) - 1;
  GroupList gl;
  if (active_groups(k, group_mask, gl) == 0 || most == 0) return SKMP_OK;
  int vidx = 0, strip = DEFAULT_STRIP;
  select_config(prec, refresh, tune_key(prec, m, n_series, offs.data()), &vidx, &strip);
  int nv = 0;
  const Fp64Variant* vs = variants_of(prec, &nv);
  static const int env64 = env_int("SKMP_FP64_VARIANT", 0, kNumFp64Variants - 1);
  static const int env32 = env_int("SKMP_FP32_VARIANT", 0, kNumFp32Variants - 1);
  if (most < kAppendNarrowBelow && (prec == SKMP_FP32 ? env32 : env64) < 0)
    vidx = (prec == SKMP_FP32) ? kNarrowFp32Variant : kNarrowFp64Variant;
  std::vector<JoinIO> io((size_t)n_series);
  for (int64_t q = 0; q < n_series; ++q) {
    const bool fresh = n_new[q] > n_old[q];
    io[q] = JoinIO{R + starts[q], ldr, fresh ? P + starts[q] : nullptr, I + starts[q], ldp};
  }
  return run_join(n_series, offs.data(), false, io.data(), m, excl, prec, gl, workspace, ws_bytes,
                  static_cast<hipStream_t>(stream), vs[vidx], strip, keep.data());
}

extern "C" int mp_selfjoin_autotune(const double* R, int64_t ldr, int64_t n_series, const int64_t* offsets,
                                    int32_t k, int32_t m, int32_t excl, int32_t prec, int32_t refresh, double* P,
                                    int64_t* I, int64_t ldp, void* workspace, size_t ws_bytes, void* stream,
                                    int32_t reps, int32_t* variant, int32_t* strip, double* best_ms) {
  clear_error();
  if (int rc = validate_selfjoin(R, ldr, n_series, offsets, k, m, excl, prec, refresh, P, I, ldp)) return rc;

  SKMP_REQUIRE(reps >= 1 && reps <= 100, "reps must lie in [1, 100]");
  SKMP_REQUIRE(k <= 64, "autotuning takes at most 64 groups (tune on a block of them)");
  hipStream_t st = static_cast<hipStream_t>(stream);
  SKMP_REQUIRE(!stream_capturing(st), "autotuning waits for the GPU and cannot run under graph capture");
  tuning_file_autoload();
  GroupList gl;
  active_groups(k, k < 64 ? (1ull << k) - 1 : ~0ull, gl);
  int nv = 0;
  const Fp64Variant* vs = variants_of(prec, &nv);
  std::vector<int> strips;
  const bool mixed = (prec == SKMP_BF16X3 || prec == SKMP_FP16X3);
  if (prec == SKMP_FP32) strips.push_back(refresh > 0 ? refresh : default_refresh(m));
  else if (mixed) strips.push_back(blk_period(refresh, m));
  else strips.assign(std::begin(kTuneStrips), std::end(kTuneStrips));
  hipEvent_t e0, e1;
  SKMP_CHECK_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_error("hipEventCreate failed");
    return SKMP_EDEVICE;
  }
  int best_v = -1, best_s = 0, rc = SKMP_OK;
  double best = 1e300;
  for (int v = 0; v < nv && rc == SKMP_OK; ++v) {
    // the blocked form walks at most `refresh` rows from a seed: below its
    // shortest period only the Hankel-direct form is a candidate
    if (mixed && refresh > 0 && refresh < 128 && vs[v].C != 0) continue;
    for (int sp : strips) {
      rc = run_selfjoin(R, ldr, n_series, offsets, k, m, excl, prec, gl, P, I, ldp, workspace, ws_bytes, st, vs[v],
                        sp);  // warm-up
      if (rc) break;
      double t_min = 1e300;
      for (int r = 0; r < reps && rc == SKMP_OK; ++r) {
        float ms = 0.f;
        if (hipEventRecord(e0, st) != hipSuccess) rc = SKMP_EDEVICE;
        if (!rc) rc = run_selfjoin(R, ldr, n_series, offsets, k, m, excl, prec, gl, P, I, ldp, workspace, ws_bytes,
                                   st, vs[v], sp);
        if (!rc && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          rc = SKMP_EDEVICE;
        if (!rc) t_min = std::min(t_min, (double)ms);
      }
      if (rc) break;
      if (t_min < best) {
        best = t_min;
        best_v = v;
        best_s = sp;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    if (rc == SKMP_EDEVICE) set_error("HIP event timing failed during autotuning");
    return rc;
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(prec, m, n_series, offsets)] = TuneChoice{best_v, best_s, best};
  }
  if (const char* f = getenv("SKMP_TUNING_FILE")) {
    if (*f && (rc = skmp_tuning_save(f)) != SKMP_OK) return rc;
  }
  if (variant) *variant = best_v;
  if (strip) *strip = best_s;
  if (best_ms) *best_ms = best;
  return SKMP_OK;
}

extern "C" size_t skmp_tile_variants(int32_t prec, char* buf, size_t len) {
  std::string text;
  if (prec >= SKMP_FP64 && prec <= SKMP_FP16X3) {
    int nv = 0;
    const Fp64Variant* vs = variants_of(prec, &nv);
    for (int i = 0; i < nv; ++i) text += std::string(vs[i].name) + "\n";
  }
  if (buf && len > 0) {
    const size_t n = std::min(len - 1, text.size());
    memcpy(buf, text.data(), n);
    buf[n] = '\0';
  }
  return text.size() + 1;
}

static std::string tuning_text() {
  std::string text;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& kv : g_tune) {
    // variants are named, not numbered: a table stays valid across builds
    // whose variant lists differ
    int nv = 0;
    const Fp64Variant* vs = variants_of(kv.first.prec, &nv);
    char line[200];
    snprintf(line, sizeof(line), "%d %d %d %s %d %.6f\n", kv.first.prec, kv.first.mlog, kv.first.nlog,
             vs[kv.second.variant].name, kv.second.strip, kv.second.ms);
    text += line;
  }
  return text;
}

extern "C" size_t skmp_tuning_export(char* buf, size_t len) {
  tuning_file_autoload();
  const std::string text = tuning_text();
  if (buf && len > 0) {
    const size_t n = std::min(len - 1, text.size());
    memcpy(buf, text.data(), n);
    buf[n] = '\0';
  }
  return text.size() + 1;
}

extern "C" int skmp_tuning_import(const char* text) {
  clear_error();
  SKMP_REQUIRE(text, "null pointer argument");
  std::vector<std::pair<TuneKey, TuneChoice>> rows;
  const char* p = text;
  while (*p) {
    const char* e = strchr(p, '\n');
    std::string line(p, e ? (size_t)(e - p) : strlen(p));
    p = e ? e + 1 : p + line.size();
    if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
    int prec, mlog, nlog, sp;
    double ms;
    char name[64], extra;
    if (sscanf(line.c_str(), "%d %d %d %63s %d %lf %c", &prec, &mlog, &nlog, name, &sp, &ms, &extra) != 6) {
      set_error("malformed tuning line: " + line);
      return SKMP_EINVAL;
    }
    SKMP_REQUIRE(prec >= SKMP_FP64 && prec <= SKMP_FP16X3, "tuning line for an unknown precision");
    int nv = 0, v = -1;
    const Fp64Variant* vs = variants_of(prec, &nv);
    for (int i = 0; i < nv; ++i)
      if (strcmp(vs[i].name, name) == 0) v = i;
    if (v < 0) {
      set_error(std::string("tuning line names a variant this build does not have: ") + name);
      return SKMP_EINVAL;
    }
    SKMP_REQUIRE(sp >= 64 && sp <= (1 << 20), "tuning line strip out of range");
    SKMP_REQUIRE(mlog >= 0 && mlog <= 12 && nlog >= 0 && nlog <= 32, "tuning line shape class out of range");
    rows.push_back({TuneKey{prec, mlog, nlog, 0}, TuneChoice{v, sp, ms}});
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const auto& r : rows) g_tune[r.first] = r.second;
  return SKMP_OK;
}

extern "C" int skmp_tuning_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  return SKMP_OK;
}

// The stamp a tuning file is written under: the current device's
// architecture (with its feature flags) and the HIP runtime version.  A file
// whose stamp differs was measured on other hardware or software and is not
// loaded.
static int tuning_stamp(std::string& out) {
  int dev = 0, rt = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
      hipRuntimeGetVersion(&rt) != hipSuccess) {
    (void)hipGetLastError();
    set_error("tuning file: no HIP device to stamp the table with");
    return SKMP_EDEVICE;
  }
  char line[320];
  snprintf(line, sizeof(line), "# sketchmp-tuning v1 arch=%s hip=%d", prop.gcnArchName, rt);
  out = line;
  return SKMP_OK;
}

extern "C" int skmp_tuning_save(const char* path) {
  clear_error();
  SKMP_REQUIRE(path && *path, "null or empty path");
  std::string stamp;
  if (int rc = tuning_stamp(stamp)) return rc;
  const std::string text = stamp + "\n" + tuning_text();
  // written beside the target and renamed over it, so a reader never sees a
  // partial file
  const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) {
    set_error("tuning file: cannot write " + tmp);
    return SKMP_EINVAL;
  }
  const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
  if (fclose(f) != 0 || !ok || rename(tmp.c_str(), path) != 0) {
    (void)remove(tmp.c_str());
    set_error(std::string("tuning file: cannot write ") + path);
    return SKMP_EINVAL;
  }
  return SKMP_OK;
}

extern "C" int skmp_tuning_load(const char* path) {
  clear_error();
  SKMP_REQUIRE(path && *path, "null or empty path");
  FILE* f = fopen(path, "rb");
  if (!f) return 0;  // no cache yet
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  fclose(f);
  std::string stamp;
  if (int rc = tuning_stamp(stamp)) return rc;
  const size_t eol = text.find('\n');
  const std::string first = text.substr(0, eol);
  if (first.rfind("# sketchmp-tuning ", 0) != 0) {
    set_error(std::string("tuning file: not a tuning table: ") + path);
    return SKMP_EINVAL;
  }
  if (first != stamp) return 0;  // measured under another device or runtime
  const std::string body = eol == std::string::npos ? std::string() : text.substr(eol + 1);
  if (int rc = skmp_tuning_import(body.c_str())) return rc;
  int lines = 0;
  for (char c : body) lines += (c == '\n');
  return lines;
}

// With SKMP_TUNING_FILE set, the first tuning lookup of the process loads
// that file (a missing or stale file loads nothing, an unreadable one is
// ignored), and every autotuning result is saved to it.
namespace skmp {
static void tuning_file_autoload() {
  static std::once_flag once;
  std::call_once(once, [] {
    const char* f = getenv("SKMP_TUNING_FILE");
    if (f && *f) (void)skmp_tuning_load(f);
  });
}
}  // namespace skmp
