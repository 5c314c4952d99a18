// Internal definitions shared by the HIP translation units of libsketchmp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/sketchmp.h"

namespace skmp {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
void clear_error();

#define SKMP_CHECK_HIP(expr)                                                              \
  do {                                                                                    \
    hipError_t e__ = (expr);                                                              \
    if (e__ != hipSuccess) {                                                              \
      ::skmp::set_error(std::string(#expr) + ": " + hipGetErrorString(e__));              \
      return SKMP_EDEVICE;                                                                \
    }                                                                                     \
  } while (0)

#define SKMP_REQUIRE(cond, msg)         \
  do {                                  \
    if (!(cond)) {                      \
      ::skmp::set_error(msg);           \
      return SKMP_EINVAL;               \
    }                                   \
  } while (0)

// -------------------------------------------------------------- constants
// Padding of the per-window statistics arrays: rows may run 64 below 0 (the
// skewed tile start) and up to PADR past n_sub (diagonal ends and tile overshoot).
constexpr int PADL = 64;
constexpr int PADR = 2048;
constexpr double FLAT_REL = 1e-10;
// Groups of a sketch: count and sum sketches up to 128 (sketch_build,
// mp_selfjoin and top_discords); a self-join runs its groups in blocks of 64
// (the 64-bit group masks), Gaussian coefficients up to 64.
constexpr int MAX_GROUPS = 128;
// The tile kernels read a series' per-window statistics through buffer
// resources whose size and offsets are 32-bit byte counts; the widest array is
// 16 bytes per padded window, so a series may have at most 2^27 - 4096
// samples (the padded window count times 16 stays below 2^31).
constexpr int64_t MAX_SERIES_LEN = (int64_t(1) << 27) - 4096;
#define SERIES_TOO_LONG \
  "series too long: the self-join addresses a series' window statistics with 32-bit offsets (at most 2^27 - 4096 samples per series)"
// The column statistics are also stored de-interleaved by a stride cs (plane
// x mod cs, slot x div cs, for the padded index x + PADL) so that 64 lanes
// whose columns are cs apart read 64 adjacent elements; cs = C - 1 for a tile
// kernel whose lanes own C diagonals each.

// ------------------------------------------------------------ workspace
// Bump allocator over the caller's workspace; every region 256-byte aligned.
struct Carve {
  char* base;
  size_t used = 0;
  size_t cap;
  Carve(void* p, size_t c) : base(static_cast<char*>(p)), cap(c) {}
  template <typename T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    return reinterpret_cast<T*>(base ? base + off : nullptr);
  }
  bool fits() const { return used <= cap; }
};

// -------------------------------------------------------------- plan
// One entry per series, device resident (built on the host, copied once per call).
//
// A series' work units pair its windows (the rows) with the windows of a
// column series: itself in a self-join; in an AB-join the other series, the
// two passes covering diagonals j - i >= 0 (rows of A, columns of B) and
// j - i >= 1 (rows of B, columns of A).  The column series is also the one
// the series' nearest neighbours belong to.
struct SeriesPlan {
  int64_t col;         // first column of the series in the caller's concatenated layout
  int64_t n;           // samples
  int64_t n_sub;       // n - m + 1
  int64_t stat_base;   // index of x = -PADL of this series inside one group's stats row
  int64_t unit_base;   // first work unit of this series
  int64_t chunk_base;  // first 256-element chunk of this series (elementwise kernels)
  int64_t blk_base;    // first 256-window block (flat-index summaries)
  int64_t lpad;        // padded windows per group: round_up(n_sub + PADL + PADR, cstride)
  int32_t nb;          // diagonal bands
  int32_t ns;          // strips per band (grid, some empty)
  const double* r0;    // sketch row g of the series at r0 + g * ldr
  int64_t ldr;
  double* p0;          // profile row g at p0 + g * ldp (NULL: not written)
  int64_t* i0;         // index row g at i0 + g * ldp
  int64_t ldp;
  int64_t keep;        // windows [0, keep) already hold a profile in p0 / i0 that is merged, not overwritten
  const double* cr0;   // the column series: sketch rows, samples, windows, stats base, padded length
  int64_t cldr;
  int64_t cn;
  int64_t n_cols;
  int64_t cstat_base;
  int64_t clpad;
  int32_t cs;          // index of the column series
  int32_t d0;          // first diagonal of the units (excl in a self-join; 0 / 1 in an AB-join)
  int32_t pexcl;       // trivial-match zone against the partner series (0 between different series)
  int32_t c0;          // a band's walk starts at step max(0, c0 - first diagonal): 0, or the first step
                       // that can reach a column >= keep (an append)
};

struct GroupList {
  int32_t count;
  int8_t g[64];
};

// Shared by the join kernels (all precisions).
struct SJState {
  const SeriesPlan* plan;
  int32_t n_series;
  int32_t m;
  int32_t excl;
  int32_t key_bits;     // global key: low key_bits of the double hold (2^key_bits - 1 - delta)
  int64_t gstride;      // stride between groups in the stats arrays
  GroupList groups;
  double2* dfdg;        // (df, dg) per window, padded
  double* invn;         // 1 / (sqrt(m) sigma), 0 if flat, NaN in the padding
  double2* cdfdg;       // dfdg de-interleaved by cstride
  double* cinvn;        // invn de-interleaved by cstride
  int32_t cstride;      // de-interleave stride of cdfdg / cinvn
  float2* fdfdg;        // FP32 copies for the FP32 tile kernel (NULL when unused)
  float* finvn;
  float2* fcdfdg;
  float* fcinvn;
  double* mu;           // window mean
  double* scale;        // per (series, group slot): max |r|
  unsigned long long* rowkey;  // best key of row i among partners j > i
  unsigned long long* colkey;  // best key of column j among partners i < j
  int32_t* flat_first;  // per (series, group slot): smallest flat window index (INT_MAX if none)
  int32_t* flat_last;   // largest flat window index (-1 if none)
  int32_t* flat_blk;    // per 256-window block: smallest flat index in the block (INT_MAX if none)
  int64_t blk_stride;   // stride between groups in flat_blk
  unsigned int* counter;  // persistent work-queue head
  int64_t total_units;
  int64_t total_chunks;
  int32_t strip;        // steps per strip (blocked MFMA form: the refresh period in rows)
  int32_t walk_stats;   // 1: substats also writes what the diagonal walks read (df, dg in both layouts, FP32 copies)
  uint16_t* bplanes;    // blocked MFMA form: 16-bit hi / lo operand planes of df, dg (NULL when unused)
  int32_t bprec;        // their format: SKMP_BF16X3 or SKMP_FP16X3
  int32_t kgroup;       // 1: a key's diagonal is its partner's; G > 1: the first of G consecutive
                        // diagonals, one of which holds the partner (the merge finds it exactly)
};

__device__ __forceinline__ int find_series(const SeriesPlan* plan, int n_series, int64_t key,
                                           int64_t SeriesPlan::*field) {
  int lo = 0, hi = n_series - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (plan[mid].*field <= key) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Values that are the same in every lane but come out of vector loads: make
// the compiler keep them (and what derives from them) in scalar registers.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <typename T>
__device__ __forceinline__ T* uni(T* p) {
  return reinterpret_cast<T*>(uni((int64_t)reinterpret_cast<intptr_t>(p)));
}

// Plan entry s (s uniform) with every field the join kernels read forced uniform.
__device__ __forceinline__ SeriesPlan load_plan(const SJState& st, int s) {
  SeriesPlan sp = st.plan[s];
  sp.unit_base = uni(sp.unit_base);
  sp.nb = uni(sp.nb);
  sp.ns = uni(sp.ns);
  sp.n_sub = uni(sp.n_sub);
  sp.stat_base = uni(sp.stat_base);
  sp.lpad = uni(sp.lpad);
  sp.col = uni(sp.col);
  sp.n = uni(sp.n);
  sp.r0 = uni(sp.r0);
  sp.ldr = uni(sp.ldr);
  sp.cr0 = uni(sp.cr0);
  sp.cldr = uni(sp.cldr);
  sp.cn = uni(sp.cn);
  sp.n_cols = uni(sp.n_cols);
  sp.cstat_base = uni(sp.cstat_base);
  sp.clpad = uni(sp.clpad);
  sp.d0 = uni(sp.d0);
  sp.c0 = uni(sp.c0);
  return sp;
}

// Decoded self-join work unit: series s, group slot gi and the two unit
// coordinates (diagonal kernels: strip sigma, band b; MFMA kernel: segment,
// row panel), with the series fields forced uniform.
struct UnitPos {
  SeriesPlan sp;
  int s, gi, outer, inner;
};

__device__ __forceinline__ UnitPos decode_unit(const SJState& st, unsigned int unit) {
  UnitPos u;
  u.s = uni(find_series(st.plan, st.n_series, (int64_t)unit, &SeriesPlan::unit_base));
  u.sp = load_plan(st, u.s);
  const int64_t local = (int64_t)unit - u.sp.unit_base;
  const int64_t per_group = (int64_t)u.sp.nb * u.sp.ns;
  u.gi = (int)(local / per_group);
  const int64_t rem = local - (int64_t)u.gi * per_group;
  u.outer = (int)(rem / u.sp.nb);
  u.inner = (int)(rem - (int64_t)u.outer * u.sp.nb);
  return u;
}

// ---------------------------------------------------------------- timing
// Brackets the launches issued during its lifetime with HIP events on ``st``
// when timing is enabled (skmp_timing_enable); a no-op otherwise.
class StageTimer {
 public:
  StageTimer(int which, hipStream_t st);
  ~StageTimer();
  StageTimer(const StageTimer&) = delete;
  StageTimer& operator=(const StageTimer&) = delete;

 private:
  int which_;
  hipStream_t st_;
  hipEvent_t a_{}, b_{};
  bool live_ = false;
};

// -------------------------------------------------------- host helpers
// True while ``st`` is being captured into a HIP graph.
bool stream_capturing(hipStream_t st);
// Host-to-device copy of a small immutable host table, safe under graph
// capture (the source is served from a library-owned pinned copy).
int upload_async(void* dst, const void* src, size_t bytes, hipStream_t st);
int launch_sketch_coeffs_host(int32_t kind, int32_t k, uint64_t seed, const int64_t* ids, int64_t d, double* S);

// Word 3 of the buffer resources the tile kernels read through (raw buffer
// loads with 32-bit offsets).
constexpr int kBufWord3 = 0x00020000;

// Blocked-recurrence MFMA self-join (selfjoin_blocked.hip): rows and diagonals
// of a work unit (bands of 4 or 8 tiles of 16 x 16).  The refresh period P
// (rows) is one of 128, 256, 512, 1024: a multiple of 128 (16 rows per step,
// the step loop unrolled by the band's tile count) that divides BLK_UNIT_ROWS.
constexpr int BLK_UNIT_ROWS = 1024;
constexpr int BLK_DIAGS = 512;  // diagonals per work unit
int launch_sj_blk(int prec, int tiles_per_band, int waves_per_simd, const SJState& s, int64_t total_units,
                  hipStream_t st);

// Power-of-two scale of the 16-bit operand planes of a series whose largest
// |value| is maxabs (|df| <= max|r|, |dg| <= 4 max|r|; 4 max|r| = f 2^e,
// f in [0.5, 1)).  BF16 (8-bit exponent): 2^-e, the operands lie in [-1, 1].
// FP16 (5-bit exponent): 2^(14 - e), the largest operand near 2^14, so the lo
// part x - hi of an operand stays a normal FP16 number down to |x| of about
// 8e-6 of the largest (at [-1, 1] it would be subnormal below 1/8 of it);
// products stay far inside the FP32 accumulator's range.
__device__ __forceinline__ double blk_scale(double maxabs, int prec) {
  if (!(maxabs > 0.0)) return 1.0;
  int e = 0;
  (void)frexp(4.0 * maxabs, &e);
  return ldexp(1.0, (prec == SKMP_FP16X3 ? 14 : 0) - e);
}

// x split into a 16-bit hi part (x rounded) and lo part (x - hi rounded).
__device__ __forceinline__ void split16(double x, int prec, uint16_t& hi, uint16_t& lo) {
  const float f = (float)x;
  if (prec == SKMP_FP16X3) {
    const _Float16 h = (_Float16)f;
    const _Float16 l = (_Float16)(float)(x - (double)(float)h);
    hi = __builtin_bit_cast(uint16_t, h);
    lo = __builtin_bit_cast(uint16_t, l);
  } else {
    const __bf16 h = (__bf16)f;
    const __bf16 l = (__bf16)(float)(x - (double)(float)h);
    hi = __builtin_bit_cast(uint16_t, h);
    lo = __builtin_bit_cast(uint16_t, l);
  }
}

// The 16-bit operand planes of window xp (padded index) of one (series,
// group slot) whose region starts at element `region` of st.bplanes: 8 planes
// of lpad elements, plane p = copy * 4 + part * 2 + which (which: 0 = df,
// 1 = dg; part: 0 = hi, 1 = lo).  Copy c holds element xp at position xp + c,
// so 8 elements starting at any element are one dword-aligned 16-byte load
// (from the copy given by the parity of the first element).
__device__ __forceinline__ void blk_write_planes(const SJState& st, int64_t region, int64_t lpad, int64_t xp,
                                                 double df, double dg, double scale) {
  uint16_t* pl = st.bplanes + region;
  uint16_t h[2], l[2];
  split16(df * scale, st.bprec, h[0], l[0]);
  split16(dg * scale, st.bprec, h[1], l[1]);
#pragma unroll
  for (int which = 0; which < 2; ++which) {
    pl[(0 * 4 + 0 * 2 + which) * lpad + xp] = h[which];
    pl[(0 * 4 + 1 * 2 + which) * lpad + xp] = l[which];
    if (xp + 1 < lpad) {
      pl[(1 * 4 + 0 * 2 + which) * lpad + xp + 1] = h[which];
      pl[(1 * 4 + 1 * 2 + which) * lpad + xp + 1] = l[which];
    }
  }
}

// MFMA self-join (selfjoin_mixed.hip): tile edge, units per row panel, LDS bytes
constexpr int MFMA_TILE = 128;
constexpr int MFMA_SEG = 4;
size_t mfma_lds_bytes(int m);
int launch_sj_mfma(int prec, const SJState& s, int64_t total_units, hipStream_t st);

}  // namespace skmp
