// Mixed-precision self-join tiles on MFMA (BF16x3 / FP16x3), paper Def. 3 and
// Def. 6 (self-join variant of Section III-B).
//
// A 128 x 128 tile of (row i, column j) cells is a product of Hankel
// matrices of the centred sketch.  Rows (and columns) are split into centring
// blocks of BC = 16 (m <= 64) or 128 windows; with a[x] = r[i0 + x] - c for the
// block starting at window i0 (c: the mean of the block's middle window), and
// b likewise for the column block,
//   acc_ij = sum_{t < m} a[i - i0 + t] b[j - j0 + t],
//   C_ij   = acc_ij - m (mu_i - c)(mu_j - c')            (centred covariance),
//   rho_ij = C_ij / (m sigma_i sigma_j).
// The 16-bit representation error of a, b is relative to |r - c|, so it grows
// with (mu_i - c) / sigma_i; short windows (small m) vary more against their
// own sigma within a tile, hence the narrower centring blocks.
// Each operand is split into hi + lo 16-bit parts and the product keeps
// hi*hi + hi*lo + lo*hi, accumulated in FP32 by v_mfma_f32_16x16x32_{f16,bf16}.
// Because the operands are Hankel, a tile needs only the two short vectors a
// and b (128 + m values each), not 128 x m matrices: they are staged in LDS as
// eight copies shifted by one element, so every lane's 8-element K fragment is
// one aligned 16-byte LDS read.
//
// Work unit: one row panel (128 rows) times a segment of MFMA_SEG column
// tiles of one (series, group).  4 waves, each a 64 x 64 quarter of the tile
// (4 x 4 MFMA blocks).  Epilogue per cell: covariance correction, normalise,
// key = bits(1 - rho + 2^-10) with the diagonal offset inside the segment in
// the low 10 bits, running row minima (kept across the segment) and column
// minima (flushed per tile); keys merge into the same global row/column key
// arrays (as 3 - key, maxima) as the FP64 kernel's, so the FP64 merge and
// polish are shared.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "skmp_common.hpp"

namespace skmp {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int PREC>
struct Elem;

template <>
struct Elem<SKMP_FP16X3> {
  typedef _Float16 T;
  typedef f16x8 V;
  static __device__ __forceinline__ T cvt(float x) { return (T)x; }
  static __device__ __forceinline__ float back(T x) { return (float)x; }
  static __device__ __forceinline__ f32x4 mfma(V a, V b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Elem<SKMP_BF16X3> {
  typedef __bf16 T;
  typedef bf16x8 V;
  static __device__ __forceinline__ T cvt(float x) { return (T)x; }
  static __device__ __forceinline__ float back(T x) { return (float)x; }
  static __device__ __forceinline__ f32x4 mfma(V a, V b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

constexpr int MT = MFMA_TILE;         // 128
constexpr int SEG_COLS = MT * MFMA_SEG;
constexpr int CODE_BITS = 10;         // diagonal offset inside a segment: [-127, SEG_COLS - 1]
constexpr uint32_t CODE_MASK = (1u << CODE_BITS) - 1;
constexpr int CODE_TOP = SEG_COLS - 1;  // code = CODE_TOP - delta_seg in [0, CODE_TOP + 127]
static_assert(CODE_TOP + 127 <= (int)CODE_MASK, "segment too wide for the key code");

static __host__ __device__ inline int mpad(int m) { return (m + 31) & ~31; }
static __host__ __device__ inline int centring_block(int m) { return m <= 64 ? 16 : MT; }
// per centring block: the block's windows plus m - 1 samples, padded
static __host__ __device__ inline int block_len(int m) { return centring_block(m) + mpad(m); }
static __host__ __device__ inline int block_stride(int m) { return block_len(m) + 8; }

// staged positions per centring block (the copies read up to block_len + 6)
static __host__ __device__ inline int stage_len(int m) { return block_len(m) + 8; }

size_t mfma_lds_bytes(int m) {
  const int nb = MT / centring_block(m);
  // a and b: nb blocks x 2 parts x 8 copies x block_stride 16-bit elements;
  // staging: nb blocks x 2 parts x stage_len 16-bit elements
  return (size_t)2 * nb * 16 * block_stride(m) * 2 + (size_t)nb * 2 * stage_len(m) * 2;
}

// For every centring block q, v_q[x] = r[base + q BC + x] - c_q (0 past the
// series) is split once into 16-bit hi + lo (hi = v rounded, lo = v - hi
// rounded; v - hi is exact in FP32) and staged; then the eight copies are
// assembled from the staged halves: copy s of block q holds v_q[P + s] at
// position P, so a lane's 8-element K fragment is one aligned 16-byte read.
// Layout: copies ((q * 2 + part) * 8 + s) * bs + P; staging (q * 2 + part) *
// stage_len + x.
template <int PREC>
__device__ __forceinline__ void build_vectors(typename Elem<PREC>::T* dst, uint16_t* st16,
                                              const double* __restrict__ r, const double* __restrict__ mu,
                                              int64_t base, int64_t n, int n_sub, int m, int tid) {
  using E = Elem<PREC>;
  using T = typename E::T;
  const int bc = centring_block(m), nbk = MT / bc, blen = block_len(m), bs = block_stride(m);
  const int sl = stage_len(m);
  for (int w = tid; w < nbk * sl; w += 256) {
    const int q = w / sl, x = w - q * sl;
    const int64_t g = base + q * bc + x;
    const double c = mu[min((int)base + q * bc + bc / 2, n_sub - 1)];
    const float f = (g < n) ? (float)(r[g] - c) : 0.0f;
    const T h = E::cvt(f);
    const T l = E::cvt(f - E::back(h));
    st16[(q * 2 + 0) * sl + x] = __builtin_bit_cast(uint16_t, h);
    st16[(q * 2 + 1) * sl + x] = __builtin_bit_cast(uint16_t, l);
  }
  __syncthreads();
  const int nblk = blen / 8;
  for (int w = tid; w < nbk * 2 * 8 * nblk; w += 256) {
    const int qp = w / (8 * nblk);  // q * 2 + part
    const int rem = w - qp * 8 * nblk;
    const int s = rem / nblk, blk = rem - s * nblk;
    const uint16_t* src = st16 + qp * sl + blk * 8 + s;
    uint4 v;
    v.x = (uint32_t)src[0] | ((uint32_t)src[1] << 16);
    v.y = (uint32_t)src[2] | ((uint32_t)src[3] << 16);
    v.z = (uint32_t)src[4] | ((uint32_t)src[5] << 16);
    v.w = (uint32_t)src[6] | ((uint32_t)src[7] << 16);
    *reinterpret_cast<uint4*>(dst + (qp * 8 + s) * bs + blk * 8) = v;
  }
}

// Local keys: bits of the float 1 - rho + 2^-10 (ordered by minimum) with the
// diagonal code in the low CODE_BITS bits; invalid cells carry 0xFFFFFFFF.
// The bias keeps the key positive while rho <= 1 + 2^-10 (the 16-bit operand
// error is ~1e-5 in rho; a negative key would read as an invalid cell) and
// shifts every key alike.  The global (merged) keys order by maximum:
// 3 + 2^-10 - f = rho + 2.
constexpr float KEY_ONE = 1.0f + 9.765625e-4f;  // 1 + 2^-10
constexpr uint32_t KEY_NONE = 0xFFFFFFFFu;

__device__ __forceinline__ unsigned long long global_key(uint32_t key) {
  const double v = (3.0 + 9.765625e-4) - (double)__uint_as_float(key & ~CODE_MASK);
  return (unsigned long long)__double_as_longlong(v);
}

template <int PREC>
__global__ __launch_bounds__(256, 2) void sj_mfma_kernel(SJState st) {
  using E = Elem<PREC>;
  using T = typename E::T;
  using V = typename E::V;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  __shared__ unsigned int s_unit;
  // per row of the panel: -m (mu_i - c) and invn_i (kept in LDS, not in registers)
  __shared__ float2 rowdat[MT];
  const int m = st.m;
  const int mp = mpad(m);
  const int bc = centring_block(m);
  const int bs = block_stride(m);
  const int nbk = MT / bc;
  T* acp = reinterpret_cast<T*>(lds);
  T* bcp = acp + nbk * 16 * bs;
  uint16_t* stage = reinterpret_cast<uint16_t*>(bcp + nbk * 16 * bs);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, lg = lane >> 4;
  const unsigned long long GMAX = (1ull << st.key_bits) - 1;
  // fragment bases: the lane reads 8 elements starting at o = (row within its
  // centring block) + t, from copy o & 7 of that block's vector
  const int s_lane = l16 & 7;
  int abase[4], bbase[4];
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int ra = 64 * wr + 16 * x, rb_ = 64 * wc + 16 * x;
    abase[x] = ((ra / bc) * 16 + s_lane) * bs + (ra % bc) + 8 * lg + (l16 & 8);
    bbase[x] = ((rb_ / bc) * 16 + s_lane) * bs + (rb_ % bc) + 8 * lg + (l16 & 8);
  }
  // code = CODE_TOP - delta_seg, delta_seg = (j - Jseg0) - (i - I0); lane part:
  const int code_lane = CODE_TOP - (64 * wc + l16) + (64 * wr + 4 * lg);

  for (;;) {
    if (tid == 0) s_unit = atomicAdd(st.counter, 1u);
    __syncthreads();
    const unsigned int unit = __builtin_amdgcn_readfirstlane(s_unit);
    __syncthreads();
    if ((int64_t)unit >= st.total_units) break;
    const UnitPos up = decode_unit(st, unit);
    const int n_sub = (int)up.sp.n_sub;
    const int p = up.inner;
    const int I0 = p * MT;
    const int jt_first = max(p, (I0 + st.excl - (MT - 1) + MT - 1) / MT);
    const int jt_last = (n_sub - 1) / MT;
    const int jt0 = jt_first + up.outer * MFMA_SEG;
    if (jt0 > jt_last) continue;
    const int jt1 = min(jt0 + MFMA_SEG - 1, jt_last);
    const int Jseg0 = jt0 * MT;

    const int64_t sbase = (int64_t)up.gi * st.gstride + up.sp.stat_base + PADL;
    const double* __restrict__ mu = st.mu + sbase;
    const double* __restrict__ invn = st.invn + sbase;
    const double* __restrict__ r = up.sp.r0 + (int64_t)st.groups.g[up.gi] * up.sp.ldr;
    unsigned long long* gro = st.rowkey + sbase;
    unsigned long long* gco = st.colkey + sbase;

    build_vectors<PREC>(acp, stage, r, mu, I0, up.sp.n, n_sub, m, tid);

    // per-row epilogue data of the panel (read back per row block in the
    // epilogue; the column loop's first barrier orders these writes)
    if (tid < MT) {
      const int i = I0 + tid;
      const double c = mu[min(I0 + (tid / bc) * bc + bc / 2, n_sub - 1)];
      const bool ok = i < n_sub;
      rowdat[tid] = make_float2(ok ? (float)(-(double)m * (mu[i] - c)) : 0.f, ok ? (float)invn[i] : 0.f);
    }
    uint32_t rowacc[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) rowacc[rb][v] = KEY_NONE;

    for (int jt = jt0; jt <= jt1; ++jt) {
      const int J0 = jt * MT;
      __syncthreads();  // previous tile's readers of bcp / stage are done
      build_vectors<PREC>(bcp, stage, r, mu, J0, up.sp.n, n_sub, m, tid);
      __syncthreads();
      float bj[4], cj[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int jl = 64 * wc + 16 * cb + l16;
        const int j = J0 + jl;
        const double c = mu[min(J0 + (jl / bc) * bc + bc / 2, n_sub - 1)];
        const bool ok = j < n_sub;
        bj[cb] = ok ? (float)(mu[j] - c) : 0.f;
        cj[cb] = ok ? (float)invn[j] : 0.f;
      }

      f32x4 acc[4][4];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = f32x4{0.f, 0.f, 0.f, 0.f};

      for (int c = 0; c < mp / 32; ++c) {
        V ah[4], al[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          ah[rb] = *reinterpret_cast<const V*>(acp + abase[rb] + 32 * c);
          al[rb] = *reinterpret_cast<const V*>(acp + 8 * bs + abase[rb] + 32 * c);
        }
        const int tfirst = 32 * c + 8 * lg;
        const int nv = m - tfirst;  // K padding: only t < m contributes
        // one column block's fragments at a time (fewer live registers)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          V bh = *reinterpret_cast<const V*>(bcp + bbase[cb] + 32 * c);
          V bl = *reinterpret_cast<const V*>(bcp + 8 * bs + bbase[cb] + 32 * c);
          if (nv < 8) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
              if (e >= nv) {
                bh[e] = E::cvt(0.f);
                bl[e] = E::cvt(0.f);
              }
          }
#pragma unroll
          for (int rb = 0; rb < 4; ++rb) {
            acc[rb][cb] = E::mfma(ah[rb], bh, acc[rb][cb]);
            acc[rb][cb] = E::mfma(ah[rb], bl, acc[rb][cb]);
            acc[rb][cb] = E::mfma(al[rb], bh, acc[rb][cb]);
          }
        }
      }

      // epilogue
      const int code_tile = code_lane - (J0 - Jseg0);
      const bool masked = (J0 - (I0 + MT - 1) < st.excl) || (J0 + MT > n_sub) || (I0 + MT > n_sub);
      uint32_t colp[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) colp[cb] = KEY_NONE;
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        float ma[4], ri[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float2 rd = rowdat[64 * wr + 16 * rb + 4 * lg + v];
          ma[v] = rd.x;
          ri[v] = rd.y;
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float C = __builtin_fmaf(ma[v], bj[cb], acc[rb][cb][v]);
            const float kf = __builtin_fmaf(-(C * cj[cb]), ri[v], KEY_ONE);  // 1 - rho + 2^-10
            uint32_t key = (__float_as_uint(kf) & ~CODE_MASK) | (uint32_t)(code_tile + 16 * (rb - cb) + v);
            if (masked) {
              const int i = I0 + 64 * wr + 16 * rb + 4 * lg + v;
              const int j = J0 + 64 * wc + 16 * cb + l16;
              if (j - i < st.excl || j >= n_sub || i >= n_sub) key = KEY_NONE;
            }
            rowacc[rb][v] = min(rowacc[rb][v], key);
            colp[cb] = min(colp[cb], key);
          }
      }
      // column maxima: combine the four lane groups holding the same column
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        colp[cb] = min(colp[cb], (uint32_t)__shfl_xor((int)colp[cb], 16));
        colp[cb] = min(colp[cb], (uint32_t)__shfl_xor((int)colp[cb], 32));
      }
      if (lg == 0) {
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          const uint32_t key = colp[cb];
          if (key < 0x7F800000u) {
            const int j = J0 + 64 * wc + 16 * cb + l16;
            const int delta = (Jseg0 - I0) + (CODE_TOP - (int)(key & CODE_MASK));
            atomicMax(gco + j, (global_key(key) & ~GMAX) | (GMAX - (unsigned long long)delta));
          }
        }
      }
    }
    // row maxima: combine the sixteen lanes holding the same row
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        uint32_t x = rowacc[rb][v];
        x = min(x, (uint32_t)__shfl_xor((int)x, 1));
        x = min(x, (uint32_t)__shfl_xor((int)x, 2));
        x = min(x, (uint32_t)__shfl_xor((int)x, 4));
        x = min(x, (uint32_t)__shfl_xor((int)x, 8));
        rowacc[rb][v] = x;
      }
    if (l16 == 0) {
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const uint32_t key = rowacc[rb][v];
          if (key < 0x7F800000u) {
            const int i = I0 + 64 * wr + 16 * rb + 4 * lg + v;
            const int delta = (Jseg0 - I0) + (CODE_TOP - (int)(key & CODE_MASK));
            atomicMax(gro + i, (global_key(key) & ~GMAX) | (GMAX - (unsigned long long)delta));
          }
        }
    }
  }
}

int launch_sj_mfma(int prec, const SJState& s, int64_t total_units, hipStream_t st) {
  const size_t lds = mfma_lds_bytes(s.m);
  int dev = 0, ncu = 256, per_cu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const void* fn = prec == SKMP_FP16X3 ? reinterpret_cast<const void*>(&sj_mfma_kernel<SKMP_FP16X3>)
                                       : reinterpret_cast<const void*>(&sj_mfma_kernel<SKMP_BF16X3>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds) != hipSuccess || per_cu < 1) per_cu = 1;
  const int grid = (int)std::min<int64_t>((int64_t)ncu * per_cu, total_units);
  if (grid <= 0) return SKMP_OK;
  if (prec == SKMP_FP16X3)
    hipLaunchKernelGGL(sj_mfma_kernel<SKMP_FP16X3>, dim3(grid), dim3(256), lds, st, s);
  else
    hipLaunchKernelGGL(sj_mfma_kernel<SKMP_BF16X3>, dim3(grid), dim3(256), lds, st, s);
  SKMP_CHECK_HIP(hipGetLastError());
  return SKMP_OK;
}

}  // namespace skmp
