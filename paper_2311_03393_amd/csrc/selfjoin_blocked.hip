// Mixed-precision self-join tiles on MFMA in the blocked-recurrence form
// (BF16x3 / FP16x3), paper Def. 3 and Def. 6 (self-join variant of Section
// III-B).
//
// The centred covariance C(i, j) = sum_{t<m} (r[i+t] - mu_i)(r[j+t] - mu_j)
// obeys C(i+1, j+1) = C(i, j) + df_i dg_j + df_j dg_i with df_x = (r[x+m] -
// r[x]) / 2 and dg_x = (r[x+m] - mu_{x+1}) + (r[x] - mu_x) (algebra on the
// definition of C).  Summed over 16 consecutive rows, a 16 x 16 tile of C
// moves 16 rows down its diagonals by a rank-32 update:
//   C(I+16+a, J+16+b) = C(I+a, J+b) + sum_{u<16} df_{I+a+u} dg_{J+b+u} + dg_{I+a+u} df_{J+b+u}
//                     = C(I+a, J+b) + ([F_I | G_I] [G_J ; F_J])[a][b],
// F_I[a][u] = df_{I+a+u}, G_I[a][u] = dg_{I+a+u} (Hankel), and likewise for J:
// one 16 x 16 x 32 product whose depth is 32 whatever the window length m.
// The tile's accumulator carries C from step to step in FP32; the operands
// are split into 16-bit hi + lo parts (scaled by a power of two chosen for the
// format's exponent range) and the product keeps hi*hi + hi*lo + lo*hi, three
// v_mfma_f32_16x16x32_{bf16,f16} per tile step.
//
// Seeds: every refresh period (P rows) the walk restarts from exact FP64
// values.  At the period's first row I the exact C(I, c) is computed for every
// column c the period's tiles start on (one row of seeds per diagonal); a
// tile's starting values follow from its diagonal's seed by the partial
// recurrence C(I+a, J+b) = C(I, J+b-a) + sum_{u >= 16-a} ..., which is the
// same rank-32 product taken from rows I - 16 with the terms of rows below I
// masked out of the row operand.
//
// Geometry: a work unit is one (series, group), one strip of UR = 1024 rows
// and one group of Q bands; a band is NB tiles side by side (NB = 8: 128
// diagonals, Q = 4; NB = 4: Q = 8), so a unit covers 512 diagonals.  One wave per unit walks the
// bands one after the other, 16 rows per step, and the 8 tiles of a band
// share the row operand; tile t at step s needs the column operand that tile
// t + 1 used at step s - 1, so the column fragments rotate through registers
// (the step loop is unrolled by NB) and each step loads one new fragment.
// Epilogue per cell: normalise (rho = C / (m sigma_i sigma_j)), key = bits of
// 1 - rho + 2^-6 (a positive float, ordered like an unsigned integer) with
// the cell's diagonal within the unit in the low 10 bits, row minima over the
// band's tiles (then over the 16 lanes of a row) and column minima over the
// steps a column spends in the band (then over the 4 lane groups).  Both go to
// LDS key arrays that cover the unit's rows and columns and are flushed once
// per unit into the global key arrays (as rho + 2, maxima), so the FP64 merge
// and polish are those of the other tile kernels.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>
#include <utility>

#include "skmp_common.hpp"

namespace skmp {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 h16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 b16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int UR = BLK_UNIT_ROWS;   // rows per unit
constexpr int UNIT_TILES = BLK_DIAGS / 16;  // tiles side by side per unit: NB per band x Q bands
constexpr int NSEED = BLK_DIAGS + 15;  // seeds per period: columns J0 - 15 .. J0 + BLK_DIAGS - 1
constexpr int SEED_PER_LANE = (NSEED + 63) / 64;
constexpr int NCOLK = UR + BLK_DIAGS;  // columns a unit touches
constexpr int SCH = 96;                  // samples per exact-seed chunk
constexpr uint32_t CODE_MASK = 1023u;
constexpr uint32_t KEEP = ~CODE_MASK;
constexpr int CODE_TOP = BLK_DIAGS - 1;  // code = CODE_TOP - (delta - first diagonal of the unit)
static_assert(CODE_TOP + 15 <= (int)CODE_MASK, "unit too wide for the 10-bit diagonal code");
// 1 - rho + 2^-6 stays positive while rho <= 1 + 2^-6: the 16-bit operands'
// error in rho (about 1e-5, up to ~1e-3 across large variance changes inside
// a period) cannot turn the best match of a row into a negative key, which
// would read as padding.  The bias shifts every key alike, so it changes no
// ordering; keys keep 13 fraction bits (relative resolution 2^-13 above the
// bias, about 2e-6 absolute in rho below it), and the global form adds it
// back (3 + 2^-6 - key = rho + 2).
constexpr float KEY_ONE = 1.0f + 0.015625f;
constexpr double KEY_BACK = 3.0 + 0.015625;
// Invalid cells: above every real key and every NaN key, with room for the
// lane's part of the code to be added without wrapping.
constexpr uint32_t KEY_NONE = 0xFF000000u;

template <int PREC>
__device__ __forceinline__ f32x4 mfma16(u32x4 a, u32x4 b, f32x4 c) {
  if constexpr (PREC == SKMP_FP16X3)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h16x8, a), __builtin_bit_cast(h16x8, b), c, 0,
                                                  0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b16x8, a), __builtin_bit_cast(b16x8, b), c, 0,
                                                   0, 0);
}

__device__ __forceinline__ u32x4 ld128(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
  return __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
}

// f(std::integral_constant<int, I>) for I = 0 .. N - 1, as compile-time
// constants (the per-cell codes are immediate operands).
template <typename F, int... I>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// v_min3_u32 as an opaque step: the running minima fold each cell's key in
// as soon as it exists (left to itself the compiler reassociates the chains
// and keeps every key of a step alive until the last use).
__device__ __forceinline__ uint32_t min3u(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_min3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// Minimum over the four 16-lane rows of the wave for each lane position
// (lanes l, l + 16, l + 32, l + 48): swaps of rows 0 <-> 1, 2 <-> 3, then of
// the halves.
__device__ __forceinline__ uint32_t cross4_min(uint32_t x) {
  auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
  x = min((uint32_t)p[0], (uint32_t)p[1]);
  auto q = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return min((uint32_t)q[0], (uint32_t)q[1]);
}

// Minimum over the 16 lanes of a DPP row (lanes 16 g .. 16 g + 15): swaps
// within pairs and quads, then the mirrored halves and rows.
// (old = ~0, the identity of the minimum, so each step folds into one
// v_min_u32 with a DPP operand.)
__device__ __forceinline__ uint32_t row16_min(uint32_t x) {
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x141, 0xF, 0xF, false));  // row_half_mirror
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)x, 0x140, 0xF, 0xF, false));  // row_mirror
  return x;
}

// Codes of the cells: 16 (NB - 1 - t) + v for tile t, row v of the lane's
// four.  Those above 64 (not inline constants) of tiles t >= 1 are held in
// VGPRs, index below; tile 0's come with the band's edge mask folded in
// (code0 in the kernel).
constexpr int code_slot(uint32_t code) { return code <= 67 ? (int)code - 65 : 3 + ((int)code / 16 - 5) * 4 + (int)code % 16; }
constexpr int NCODEV = 11;

// Key of a cell: the bits of kf with the low 10 bits replaced by the cell's
// code CODE, one v_and_or_b32 (gfx9 VOP3 takes no literal, so the mask and
// the larger codes sit in VGPRs, set once per kernel).
template <uint32_t CODE>
__device__ __forceinline__ uint32_t key_of(float kf, uint32_t keep_v, const uint32_t (&codev)[NCODEV]) {
  uint32_t r;
  if constexpr (CODE <= 64)
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(__float_as_uint(kf)), "v"(keep_v), "i"(CODE));
  else
    asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(__float_as_uint(kf)), "v"(keep_v), "v"(codev[code_slot(CODE)]));
  return r;
}

// The same with the code in a VGPR (tile 0: the code with the edge mask).
__device__ __forceinline__ uint32_t key_with(float kf, uint32_t keep_v, uint32_t code_v) {
  uint32_t r;
  asm("v_and_or_b32 %0, %1, %2, %3" : "=v"(r) : "v"(__float_as_uint(kf)), "v"(keep_v), "v"(code_v));
  return r;
}

}  // namespace

template <int PREC, int WPE, int NB>
__global__ __launch_bounds__(64, WPE) void sj_blk_kernel(SJState st) {
  static_assert(NB == 4 || NB == 8, "4 or 8 tiles per band");
  constexpr int Q = UNIT_TILES / NB;  // bands per unit
  __shared__ uint32_t rowk[UR];
  __shared__ uint32_t colk[NCOLK];
  // the exact-seed stage (FP64 samples) and, once the seeds are computed, the
  // seeds themselves (FP32) share one buffer
  __shared__ __align__(16) double sstage[SCH + SEED_PER_LANE * 64 + SCH];
  float* sseed = reinterpret_cast<float*>(sstage);
  const int lane = threadIdx.x;
  const int l16 = lane & 15, lg = lane >> 4;
  uint32_t keep_v;  // the key mask, held in a VGPR
  asm volatile("v_mov_b32 %0, %1" : "=v"(keep_v) : "i"(KEEP));
  uint32_t codev[NCODEV];  // codes above 64 (8 tiles per band only; 4 tiles' codes are all inline)
#pragma unroll
  for (int q = 0; q < NCODEV; ++q) {
    if constexpr (NB == 8) {
      const uint32_t code = q < 3 ? 65u + q : 80u + 16u * ((q - 3) / 4) + (q - 3) % 4;
      asm volatile("v_mov_b32 %0, %1" : "=v"(codev[q]) : "v"(code));
    } else {
      codev[q] = 0u;
    }
  }
  const int P = st.strip;        // refresh period (rows), a divisor of UR and a multiple of 16 NB
  const int m = st.m;
  const unsigned long long GMAX = (1ull << st.key_bits) - 1;
  for (int x = lane; x < UR; x += 64) rowk[x] = KEY_NONE;
  for (int x = lane; x < NCOLK; x += 64) colk[x] = KEY_NONE;

  auto take = [&]() -> unsigned int {
    unsigned int u = 0;
    if (lane == 0) u = atomicAdd(st.counter, 1u);
    return __builtin_amdgcn_readfirstlane(__shfl(u, 0)) + gridDim.x;
  };
  for (unsigned int unit = blockIdx.x; (int64_t)unit < st.total_units; unit = take()) {
    const UnitPos up = decode_unit(st, unit);
    const SeriesPlan& sp = up.sp;
    const int n_sub = (int)sp.n_sub;
    const int n_cols = (int)sp.n_cols;
    const int dbg = sp.d0 + up.inner * BLK_DIAGS;  // first diagonal of the unit
    const int I0 = up.outer * UR;                     // first row of the unit
    const int row_end = min(n_sub, n_cols - dbg);     // rows that have a partner on a diagonal >= dbg
    if (I0 >= row_end) continue;
    const int gi = up.gi;
    const int64_t gbase = (int64_t)gi * st.gstride + sp.stat_base;
    const int64_t cgbase = (int64_t)gi * st.gstride + sp.cstat_base;
    const int g = st.groups.g[gi];
    const double* __restrict__ r = sp.r0 + (int64_t)g * sp.ldr;
    const double* __restrict__ rc = sp.cr0 + (int64_t)g * sp.cldr;
    const double* __restrict__ mu = st.mu + gbase + PADL;
    const double* __restrict__ muc = st.mu + cgbase + PADL;
    const double sc = blk_scale(st.scale[(int64_t)up.s * st.groups.count + gi], PREC);
    // operand planes and FP32 window norms of the rows and of the columns
    const __amdgpu_buffer_rsrc_t pa =
        __builtin_amdgcn_make_buffer_rsrc((void*)(st.bplanes + 8 * gbase), 0, (int)(sp.lpad * 16), kBufWord3);
    const __amdgpu_buffer_rsrc_t pb =
        __builtin_amdgcn_make_buffer_rsrc((void*)(st.bplanes + 8 * cgbase), 0, (int)(sp.clpad * 16), kBufWord3);
    const __amdgpu_buffer_rsrc_t ria =
        __builtin_amdgcn_make_buffer_rsrc((void*)(st.finvn + gbase), 0, (int)(sp.lpad * 4), kBufWord3);
    const __amdgpu_buffer_rsrc_t rib =
        __builtin_amdgcn_make_buffer_rsrc((void*)(st.finvn + cgbase), 0, (int)(sp.clpad * 4), kBufWord3);
    const int lpad = (int)sp.lpad, clpad = (int)sp.clpad;
    // lane parts of the fragment offsets (bytes); the uniform parts go in soffset
    const int cA = l16 & 1;
    const int voA = (((cA * 4) + (lg >> 1)) * lpad + l16 + 8 * (lg & 1) + PADL - 16 + cA) * 2;
    const int cB = (dbg + l16) & 1;
    const int voB = (((cB * 4) + 1 - (lg >> 1)) * clpad + l16 + 8 * (lg & 1) + PADL - 16 + cB) * 2;
    const int loA = 2 * lpad * 2, loB = 2 * clpad * 2;  // hi -> lo plane
    const int voRI = (4 * lg + PADL) * 4;
    const int voCI = (l16 + PADL) * 4;
    // mask of the row operand at a period start: keep u >= 16 - a (a = l16), u = 8 (lg & 1) + element
    u32x4 amask;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const int u0 = 8 * (lg & 1) + 2 * d;
      amask[d] = (u0 >= 16 - l16 ? 0x0000FFFFu : 0u) | (u0 + 1 >= 16 - l16 ? 0xFFFF0000u : 0u);
    }

    const int I1 = min(I0 + UR, row_end);
    for (int Ip = I0; Ip < I1; Ip += P) {
      // ---- exact FP64 seeds C(Ip, c), c = J0 - 15 + x, x < NSEED (J0 = Ip + dbg):
      // C = sum_t a_t r[c + t] - mu_c sum_t a_t with a_t = r[Ip + t] - mu_Ip; the
      // row window and the columns' samples are staged in LDS in chunks of SCH
      // samples with coalesced loads, and lane l computes the SEED_PER_LANE
      // consecutive columns c0 + q, c0 = J0 - 15 + SEED_PER_LANE l, from a
      // register window over the staged columns.
      const int J0 = Ip + dbg;
      __builtin_amdgcn_s_setprio(0);
      {
        double* srow = sstage;
        double* scol = sstage + SCH;
        const double mr = mu[Ip];
        const int nl = (int)sp.cn - 1;
        double acc[SEED_PER_LANE];
#pragma unroll
        for (int q = 0; q < SEED_PER_LANE; ++q) acc[q] = 0.0;
        double sa = 0.0;
        for (int x0 = 0; x0 < m; x0 += SCH) {
          __syncthreads();  // the previous chunk (or the last walk's seeds) is consumed
          for (int i = lane; i < SCH; i += 64) srow[i] = (x0 + i < m) ? r[Ip + x0 + i] - mr : 0.0;
          for (int i = lane; i < SEED_PER_LANE * 64 + SCH; i += 64) scol[i] = rc[min(max(J0 - 15 + x0 + i, 0), nl)];
          __syncthreads();
          const int xe = min(SCH, m - x0);
          const double* cw = scol + SEED_PER_LANE * lane;
          int xx = 0;
          for (; xx + SEED_PER_LANE <= xe; xx += SEED_PER_LANE) {
            double w[2 * SEED_PER_LANE - 1];
#pragma unroll
            for (int k = 0; k < 2 * SEED_PER_LANE - 1; ++k) w[k] = cw[xx + k];
#pragma unroll
            for (int dx = 0; dx < SEED_PER_LANE; ++dx) {
              const double a = srow[xx + dx];
              sa += a;
#pragma unroll
              for (int q = 0; q < SEED_PER_LANE; ++q) acc[q] = fma(a, w[dx + q], acc[q]);
            }
          }
          for (; xx < xe; ++xx) {
            const double a = srow[xx];
            sa += a;
#pragma unroll
            for (int q = 0; q < SEED_PER_LANE; ++q) acc[q] = fma(a, cw[xx + q], acc[q]);
          }
        }
        __syncthreads();  // the stage is read; its space holds the seeds
        const int c0 = J0 - 15 + SEED_PER_LANE * lane;
#pragma unroll
        for (int q = 0; q < SEED_PER_LANE; ++q) {
          const int c = c0 + q;
          const double v = fma(-muc[min(max(c, 0), n_cols - 1)], sa, acc[q]);
          sseed[SEED_PER_LANE * lane + q] = (c >= 0 && c < n_cols) ? (float)(v * sc * sc) : 0.0f;
        }
      }
      __builtin_amdgcn_s_setprio(1);
      __syncthreads();
      const int rows_left = min(P, I1 - Ip);
      for (int b = 0; b < Q; ++b) {
        const int db = dbg + 16 * NB * b;  // the band's first tile: columns Ip + db + 16 t
        if (Ip + db >= n_cols) break;
        // steps of this band: rows below the period end and a column inside the matrix
        const int smax = min((rows_left + 15) / 16, (n_cols - (Ip + db) + 15) / 16);
        const int steps = ((smax + NB - 1) / NB) * NB;
        const int lane_base = 16 * NB * (Q - 1 - b) + 15 - l16 + 4 * lg;
        // band 0 of the first unit: its tile 0 holds cells below the first
        // diagonal (j - i < d0, trivial matches) at every step
        // (those cells' keys get KEY_NONE in the same AND-OR that embeds tile 0's code)
        const bool edge = (up.inner == 0 && b == 0);
        uint32_t code0[4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
          code0[v] = (uint32_t)(16 * (NB - 1) + v) | ((edge && l16 < 4 * lg + v) ? KEY_NONE : 0u);
        const int soB0 = (Ip + db) * 2;                // column tile c at soffset soB0 + 32 (c + 1)
        // column fragments of tiles c = -1 .. NB - 2 (slot (c + NB) % NB)
        u32x4 bh[NB], bl[NB];
        float ci[NB];
        uint32_t col[NB];
#pragma unroll
        for (int c = -1; c < NB - 1; ++c) {
          const int sl = (c + NB) % NB;
          bh[sl] = ld128(pb, voB, soB0 + 32 * (c + 1));
          bl[sl] = ld128(pb, voB + loB, soB0 + 32 * (c + 1));
        }
#pragma unroll
        for (int c = 0; c < NB - 1; ++c) {
          ci[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rib, voCI, (Ip + db + 16 * c) * 4, 0));
          col[c] = KEY_NONE;
        }
        col[NB - 1] = KEY_NONE;
        // starting tiles: gathered seeds plus the masked rank-32 product of rows Ip - 16
        f32x4 acc[NB];
        {
          u32x4 ah = ld128(pa, voA, Ip * 2), al = ld128(pa, voA + loA, Ip * 2);
          ah &= amask;
          al &= amask;
#pragma unroll
          for (int t = 0; t < NB; ++t) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t][v] = sseed[16 * (NB * b + t) + 15 + l16 - 4 * lg - v];
            const int sl = (t - 1 + NB) % NB;
            acc[t] = mfma16<PREC>(ah, bh[sl], acc[t]);
            acc[t] = mfma16<PREC>(ah, bl[sl], acc[t]);
            acc[t] = mfma16<PREC>(al, bh[sl], acc[t]);
          }
        }
        // step 0's row operand and row norms; later steps' loads are issued one
        // step ahead, right after tile 0's products have read the slot the
        // entering column tile overwrites
        u32x4 ah = ld128(pa, voA, (Ip + 16) * 2), al = ld128(pa, voA + loA, (Ip + 16) * 2);
        f32x4 ri = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ria, voRI, Ip * 4, 0));
        {
          bh[NB - 1] = ld128(pb, voB, soB0 + 32 * NB);
          bl[NB - 1] = ld128(pb, voB + loB, soB0 + 32 * NB);
          ci[NB - 1] = __builtin_bit_cast(
              float, __builtin_amdgcn_raw_buffer_load_b32(rib, voCI, (Ip + db + 16 * (NB - 1)) * 4, 0));
        }
        for (int s0 = 0; s0 < steps; s0 += NB) {
#pragma unroll
          for (int rr = 0; rr < NB; ++rr) {
            const int s = s0 + rr;
            const int I = Ip + 16 * s;
            // 1 / (sqrt(m) sigma scale) of the lane's rows (the column norms ci
            // carry 1 / scale too: together they remove the covariance's scale^2)
            const f32x4 rs_ = ri;
            u32x4 ahn, aln;
            f32x4 rin;
            uint32_t rowm[4], kprev[4];
            f32x4 part[NB];  // a tile's update after its first and second products
            // Iteration it: the epilogue of tile it, its first product, the
            // second product of tile it - 1 and the third of tile it - 2, so
            // that no two dependent MFMAs are adjacent and each tile's VALU
            // work overlaps the products of the tiles before it.
            static_for<NB + 2>([&](auto ic) {
              constexpr int it = decltype(ic)::value;
              if constexpr (it < NB) {
                constexpr int t = it;
                const int sl = (t + rr) % NB;
                uint32_t key[4];
                static_for<4>([&](auto vc) {
                  constexpr int v = decltype(vc)::value;
                  const float kf = __builtin_fmaf(-(acc[t][v] * ci[sl]), rs_[v], KEY_ONE);
                  if constexpr (t == 0)
                    key[v] = key_with(kf, keep_v, code0[v]);  // cells below the first diagonal: KEY_NONE
                  else
                    key[v] = key_of<(uint32_t)(16 * (NB - 1 - t) + v)>(kf, keep_v, codev);
                });
                // column tile (slot sl): its four rows of this step
                col[sl] = min3u(col[sl], key[0], key[1]);
                col[sl] = min3u(col[sl], key[2], key[3]);
                // rows: over the band's tiles, two tiles per v_min3
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                  if (t == 0) rowm[v] = key[v];
                  else if (t % 2 == 1 && t + 1 < NB) kprev[v] = key[v];
                  else if (t % 2 == 1) rowm[v] = min(rowm[v], key[v]);
                  else rowm[v] = min3u(rowm[v], kprev[v], key[v]);
                }
                // (after the band's last step the update is not used: it reads padding)
                part[t] = mfma16<PREC>(ah, bh[sl], acc[t]);
              }
              if constexpr (it >= 1 && it - 1 < NB) {
                constexpr int t = it - 1;
                part[t] = mfma16<PREC>(ah, bl[(t + rr) % NB], part[t]);
              }
              if constexpr (it >= 2) {
                constexpr int t = it - 2;
                acc[t] = mfma16<PREC>(al, bh[(t + rr) % NB], part[t]);
                if constexpr (t == 0) {
                  // next step: row operand and norms, and the entering column tile
                  // c = s + NB into the slot tile 0's products have just read
                  ahn = ld128(pa, voA, (I + 32) * 2);
                  aln = ld128(pa, voA + loA, (I + 32) * 2);
                  rin = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(ria, voRI, (I + 16) * 4, 0));
                  bh[rr] = ld128(pb, voB, soB0 + 32 * (s + NB + 1));
                  bl[rr] = ld128(pb, voB + loB, soB0 + 32 * (s + NB + 1));
                }
              }
              __builtin_amdgcn_sched_barrier(0);
            });
            // rows Ip + 16 s + 4 lg + v: minimum over the 16 lanes of the lane group
#pragma unroll
            for (int v = 0; v < 4; ++v) rowm[v] = row16_min(rowm[v] + (uint32_t)lane_base);
            const int xr = Ip - I0 + 16 * s + 4 * lg;  // < UR: the period ends inside the unit
            if (l16 == 0) {
#pragma unroll
              for (int v = 0; v < 4; ++v) atomicMin(&rowk[xr + v], rowm[v]);
            }
            // column tile c = s leaves the band: minimum over the four lane groups
            {
              const uint32_t x = cross4_min(col[rr] + (uint32_t)lane_base);
              if (lg == 0) atomicMin(&colk[Ip - I0 + 16 * (NB * b + s) + l16], x);
              col[rr] = KEY_NONE;
            }
            // its norm slot now takes the entering column tile c = s + NB
            ci[rr] = __builtin_bit_cast(
                float, __builtin_amdgcn_raw_buffer_load_b32(rib, voCI, (Ip + db + 16 * (s + NB)) * 4, 0));
            ah = ahn;
            al = aln;
            ri = rin;
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        // column tiles still open when the walk stops (c = steps .. steps + NB - 2)
#pragma unroll
        for (int c = 1; c < NB; ++c) {
          const int sl = (steps + c - 1) % NB;
          const uint32_t x = cross4_min(col[sl] + (uint32_t)lane_base);
          if (lg == 0) atomicMin(&colk[Ip - I0 + 16 * (NB * b + steps - 1 + c) + l16], x);
        }
      }
      __syncthreads();  // the seeds of this period are consumed
    }
    // ---- flush: every row and column of the unit is complete
    __syncthreads();
    unsigned long long* gro = st.rowkey + gbase + PADL;
    unsigned long long* gco = st.colkey + cgbase + PADL;
    auto to_global = [&](uint32_t key) -> unsigned long long {
      const int delta = dbg + CODE_TOP - (int)(key & CODE_MASK);
      const double v = KEY_BACK - (double)__uint_as_float(key & KEEP);
      return ((unsigned long long)__double_as_longlong(v) & ~GMAX) | (GMAX - (unsigned long long)delta);
    };
    for (int x = lane; x < UR; x += 64) {
      const uint32_t key = rowk[x];
      rowk[x] = KEY_NONE;
      const int i = I0 + x;
      if (key < 0x7F800000u && i < n_sub) atomicMax(gro + i, to_global(key));
    }
    for (int y = lane; y < NCOLK; y += 64) {
      const uint32_t key = colk[y];
      colk[y] = KEY_NONE;
      const int j = I0 + dbg + y;
      if (key < 0x7F800000u && j < n_cols) atomicMax(gco + j, to_global(key));
    }
    __syncthreads();
  }
}

int launch_sj_blk(int prec, int tiles_per_band, int waves_per_simd, const SJState& s, int64_t total_units,
                  hipStream_t st) {
  int dev = 0, ncu = 256, per_cu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  void (*k)(SJState) = nullptr;
#define SKMP_BLK_PICK(P, W, N) \
  if (prec == P && waves_per_simd == W && tiles_per_band == N) k = sj_blk_kernel<P, W, N>;
  SKMP_BLK_PICK(SKMP_BF16X3, 2, 8) SKMP_BLK_PICK(SKMP_BF16X3, 3, 4)
  SKMP_BLK_PICK(SKMP_FP16X3, 2, 8) SKMP_BLK_PICK(SKMP_FP16X3, 3, 4)
#undef SKMP_BLK_PICK
  if (!k) {
    set_error("no blocked MFMA kernel for this tile count and occupancy");
    return SKMP_EINVAL;
  }
  const void* fn = reinterpret_cast<const void*>(k);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, 0) != hipSuccess || per_cu < 1) per_cu = 4;
  const int grid = (int)std::min<int64_t>((int64_t)ncu * per_cu, total_units);
  if (grid <= 0) return SKMP_OK;
  hipLaunchKernelGGL(k, dim3(grid), dim3(64), 0, st, s);
  SKMP_CHECK_HIP(hipGetLastError());
  return SKMP_OK;
}

}  // namespace skmp
