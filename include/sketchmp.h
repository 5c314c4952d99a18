/*
 * sketchmp: sketched matrix-profile discord mining on MI355X (gfx950).
 *
 * C-ABI of the HIP library libsketchmp.so.  The four calls of the method are
 *   sketch_build        z-normalise every dimension and sketch d series into k
 *                       (paper Section III-A, Algorithm 1);
 *   sketch_update_dims  add / remove dimensions of a built sketch (Section III-C);
 *   mp_selfjoin         z-normalised self-join matrix profile of every sketched
 *                       series (Def. 3, Def. 6, self-join variant of Section III-B);
 *   top_discords        discord time detection over the k profiles and the
 *                       ordered non-overlapping discord list (Algorithm 2;
 *                       Sections IV-B and IV-C).
 *
 * Conventions for every call:
 *   - A multidimensional series T in R^{d x n} (Def. 1) is row-major: dimension j
 *     occupies T[j*ldt .. j*ldt + N).  Several independent series may be
 *     concatenated along time: ``offsets`` (HOST array of n_series+1 int64,
 *     non-decreasing, offsets[0] = 0) gives series s the columns
 *     [offsets[s], offsets[s+1]).  Every per-series output uses the same columns.
 *   - Pointers named *_dev, and all bulk data (T, R, P, I, workspace, outputs
 *     of top_discords) are DEVICE pointers on the current HIP device.  Pointers
 *     documented as host are host memory.  The caller owns every buffer.
 *   - ``stream`` is a hipStream_t (NULL = default stream).  Calls are
 *     asynchronous: the return code covers argument validation and kernel
 *     launch; device faults surface at the caller's next synchronisation.
 *   - ``workspace`` is caller-provided device scratch of at least the size the
 *     matching *_workspace query returns (256-byte aligned).  Its contents need
 *     not be initialised and are clobbered.
 *   - Return value: SKMP_OK (0) or a negative SKMP_E* code; a message for the
 *     last failure on the calling thread is available from skmp_last_error().
 *     On error nothing has been launched.
 *   - HIP graph capture: every call except a sketch call with
 *     SKMP_FLAG_CHECK_FINITE (which reads a flag back on the host, rejected with
 *     SKMP_EINVAL under capture) only enqueues kernels and host-to-device
 *     copies of small host tables (series plans, sketch coefficients), so it
 *     may be captured.  The copies read library-owned pinned copies of those
 *     tables (kept for the life of the process, 64 MiB in total), created by an
 *     uncaptured call: make one call with the same arguments before capturing,
 *     otherwise the captured call fails with SKMP_EINVAL.  A graph replays the
 *     same pointers: keep the captured buffers (including the workspace) alive
 *     and unchanged in size.
 */
#ifndef SKETCHMP_H
#define SKETCHMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SKMP_OK 0
#define SKMP_EINVAL (-1)     /* invalid argument */
#define SKMP_ENOMEM (-2)     /* workspace too small */
#define SKMP_EDEVICE (-3)    /* HIP runtime error */
#define SKMP_ENONFINITE (-4) /* non-finite input (returned only when SKMP_FLAG_CHECK_FINITE is set) */
#define SKMP_ENOTFOUND (-5)  /* unknown dimension id */

/* sketch kinds (Section III-A): R = S * Tbar with S in R^{k x d} */
#define SKMP_SUM 0   /* k = 1, every coefficient +1 (Fig. 1) */
#define SKMP_COUNT 1 /* count sketch: column j has s(j) in {-1,+1} at row h(j) */
#define SKMP_GAUSS 2 /* dense N(0,1) projection */

/* input dtypes */
#define SKMP_F64 0
#define SKMP_F32 1

/* self-join precisions */
#define SKMP_FP64 0   /* FP64 diagonal recurrence */
#define SKMP_FP32 1   /* FP32 diagonal recurrence, exact FP64 seed every `refresh` rows */
#define SKMP_BF16X3 2 /* MFMA, BF16 hi+lo split products, FP32 accumulation */
#define SKMP_FP16X3 3 /* MFMA, FP16 hi+lo split products, FP32 accumulation */
/* Every precision reports the exact FP64 distance of the neighbour it finds.
 * BF16x3 / FP16x3 run in one of two forms (tuning variants): the blocked
 * recurrence (default: 16 x 16 tiles of the centred covariance carried down
 * their diagonals by rank-32 MFMA updates, depth 32 whatever m, restarted
 * from exact FP64 seeds every `refresh` rows) or the Hankel-direct tiles (a
 * 128 x 128 tile is a product of two Hankel matrices of depth m). */

/* flags for sketch_build / sketch_update_dims / sketch_append */
#define SKMP_FLAG_CHECK_FINITE 1u /* synchronise and reject NaN/Inf input */
/* Without the flag non-finite input is marked, never dropped (no host
 * read-back, so the calls stay capturable): a dimension holding NaN or Inf
 * gets the statistics (NaN, NaN), the sketch of its series is NaN, and the
 * self-join reports P = NaN, I = -1 for every window whose sketched samples
 * are not finite (top_discords skips them). */

/* Message describing the last failure on this thread ("" if none). */
const char* skmp_last_error(void);

/* Library version string. */
const char* skmp_version(void);

/*
 * Sketch coefficients S (k x d, row-major, HOST output of k*d doubles) for the
 * dimensions with identifiers dim_ids[0..d) (host; NULL means 0..d-1).
 * Coefficients are pure functions of (kind, k, seed, dimension id):
 *   count: h(id) = ((a*id + b) mod p) mod k, s(id) = 1 - 2*(((a2*id + b2) mod p) mod 2),
 *          p = 2^61 - 1, with (a, b, a2, b2) the first four SplitMix64(seed)
 *          outputs reduced as 1 + o mod (p-1) / o mod p (a 2-universal family,
 *          Section III-A and the Appendix);
 *   gauss: Box-Muller N(0,1) from SplitMix64(seed) outputs 2c+1 and 2c+2,
 *          c = id*64 + g;
 *   sum:   k must be 1, every entry +1.
 * Ids must lie in [0, 2^61 - 1); k in [1, 128] for the count and sum sketches,
 * [1, 64] for the Gaussian one (its draws are keyed by id * 64 + g).
 */
int sketch_coeffs(int32_t kind, int32_t k, uint64_t seed, const int64_t* dim_ids, int64_t d, double* S_host);

/*
 * The number of sketched series for d dimensions: ceil(sqrt(d)), which balances
 * the k self-joins of time detection against the d / k dimensions one group
 * holds for dimension detection (the cost analysis of Section III and the
 * choice of Section IV), capped at the library's 128 groups (the count
 * sketch; a Gaussian sketch takes at most 64).  d >= 1, else
 * SKMP_EINVAL.  Host only.
 */
int32_t sketch_default_k(int64_t d);

/* Workspace bytes needed by sketch_build (offsets host, as in sketch_build); 0 on bad arguments. */
size_t sketch_build_workspace(int64_t d, int64_t n_series, const int64_t* offsets, int32_t k);

/*
 * Normalise and sketch (Section III-A, Algorithm 1).
 *   T        device, d x N (N = offsets[n_series]), row stride ldt >= N, dtype SKMP_F64 or SKMP_F32.
 *   d        number of dimensions (>= 1).
 *   dim_ids  host, d identifiers (NULL: 0..d-1); they key the coefficients.
 *   k, kind, seed  as in sketch_coeffs.
 *   R        device out, k x N doubles, row stride ldr >= N:
 *            R[g][t] = sum_j S[g][j] * (T[j][t] - mu_sj) / sigma_sj for t in series s,
 *            where mu_sj, sigma_sj are the mean and population standard deviation
 *            of dimension j over series s (sigma = 0 contributes 0).
 *   dim_stats device out, n_series x d x 2 doubles: (mu_sj, sigma_sj);
 *            (NaN, NaN) if dimension j of series s holds NaN or Inf (then
 *            R is NaN over series s; with SKMP_FLAG_CHECK_FINITE the call
 *            synchronises and returns SKMP_ENONFINITE instead).
 */
int sketch_build(const void* T, int32_t dtype, int64_t d, int64_t ldt, int64_t n_series, const int64_t* offsets,
                 const int64_t* dim_ids, int32_t k, int32_t kind, uint64_t seed, uint32_t flags, double* R,
                 int64_t ldr, double* dim_stats, void* workspace, size_t ws_bytes, void* stream);

/* Workspace bytes needed by sketch_update_dims for a series of n samples; 0 on bad arguments. */
size_t sketch_update_workspace(int64_t n, int64_t d_add, int64_t d_rem, int32_t k);

/*
 * Add and/or remove dimensions of a single-series sketch in place (Section III-C):
 *   R^(g) += S_g,add * Tbar_add  -  S_g,rem * Tbar_rem.
 *   R        device, k x n, row stride ldr (as written by sketch_build with n_series = 1).
 *   T_add    device, d_add x n (row stride ldt), new dimensions; they must span
 *            all n samples (the paper advises against partial-membership
 *            dimensions).  add_ids host, d_add new identifiers.
 *   add_stats device out, d_add x 2 doubles (mu, sigma) of the added dimensions.
 *   T_rem    device, d_rem x n (row stride ldt), the samples of the removed
 *            dimensions; rem_ids host; rem_stats device, d_rem x 2 doubles,
 *            the (mu, sigma) those dimensions had when they were added.
 *   changed_groups host out (may be NULL): bit g set iff R^(g) changed
 *            (count sketch: the groups h(id); sum / gauss: every group).
 * Either side may be empty (d_add = 0 or d_rem = 0).
 */
int sketch_update_dims(double* R, int64_t ldr, int64_t n, int32_t k, int32_t kind, uint64_t seed, int32_t dtype,
                       int64_t ldt, const void* T_add, int64_t d_add, const int64_t* add_ids, double* add_stats,
                       const void* T_rem, int64_t d_rem, const int64_t* rem_ids, const double* rem_stats,
                       uint32_t flags, uint64_t* changed_groups, void* workspace, size_t ws_bytes, void* stream);

/* Workspace bytes needed by mp_selfjoin (offsets host, as in mp_selfjoin). */
size_t mp_selfjoin_workspace(int64_t n_series, const int64_t* offsets, int32_t k, int32_t m, int32_t prec);

/*
 * Self-join matrix profile of every sketched series (Def. 6 with
 * T_test = T_train, Section III-B), z-normalised Euclidean distance (Def. 3).
 *   R        device, k x N doubles, row stride ldr (sketch_build output).
 *   m        subsequence length, 4 <= m <= 2048 (<= 1024 for BF16x3 / FP16x3);
 *            every series needs m <= n_s <= 2^27 - 4096 samples (the tile
 *            kernels address a series' window statistics with 32-bit offsets).
 *   excl     trivial-match exclusion: (i, j) is excluded iff |i - j| < excl; 1 <= excl.
 *   prec     SKMP_FP64 | SKMP_FP32 | SKMP_BF16X3 | SKMP_FP16X3.
 *   refresh  SKMP_FP32: rows between exact FP64 recomputations of the running
 *            covariance (0 = the larger of 256 and 2.5 m rounded up to a
 *            multiple of 256).  BF16x3 / FP16x3, blocked form: the period is
 *            the largest of 128, 256, 512, 1024 rows not above `refresh`
 *            (0 = the smallest of 256, 512, 1024 that is at least 4 m; 1024
 *            above m = 256); a refresh below 128 selects the Hankel-direct
 *            form, which walks no rows.  Ignored by SKMP_FP64.
 *   k        1 <= k <= 128; more than 64 groups are joined in blocks of 64
 *            (one launch sequence per block, in stream order) and then need
 *            group_mask = ~0.
 *   group_mask bit g selects group g (~0 = all); unselected rows of P/I are untouched.
 *   P        device out, k x N doubles, row stride ldp: P[g][offsets[s] + i] for
 *            i < n_s - m + 1 is the distance from subsequence i of R^(g) in
 *            series s to its nearest admissible neighbour; +inf if none;
 *            NaN if the subsequence's sketched samples are not finite.
 *   I        device out, k x N int64, row stride ldp: that neighbour's index
 *            within the series (0-based), -1 if none.
 *            The last m - 1 columns of every series (no subsequence starts
 *            there) are not written in P or I.
 * Subsequence statistics use the population sigma; a subsequence whose sigma
 * is <= 1e-10 * max|R^(g)| over its series is flat and normalises to the zero
 * vector (dist(flat, flat) = 0, dist(flat, other) = sqrt(m)).  Reported P values
 * are recomputed in FP64 for the reported neighbour: from explicit differences
 * of the normalised subsequences, or (SKMP_FP32, where d^2 >= 0.01 m) from the
 * neighbour's exact FP64 centred correlation, d^2 = 2 m (1 - rho), which the
 * search of its diagonal group has just computed (within 1e-10 of the former
 * at that distance).
 * SKMP_EINVAL (message in skmp_last_error) when the join needs more than
 * 2^32 - 2^20 work units (groups x bands of 64 C diagonals x strips of
 * `refresh` rows, C = 16 in FP32 and 8 in FP64; one series of 12 million
 * windows with k = 8 at refresh 256 is about that): split the groups over
 * calls (group_mask) or raise `refresh`.  The same holds for mp_abjoin and
 * mp_selfjoin_append.
 */
int mp_selfjoin(const double* R, int64_t ldr, int64_t n_series, const int64_t* offsets, int32_t k, int32_t m,
                int32_t excl, int32_t prec, int32_t refresh, uint64_t group_mask, double* P, int64_t* I,
                int64_t ldp, void* workspace, size_t ws_bytes, void* stream);

/*
 * Autotuning of the self-join's launch configuration for batched runs: the
 * tile-kernel variant (diagonals per lane, prefetch depth, waves per SIMD,
 * column-maximum scheme) and, for SKMP_FP64, the strip of rows per work unit
 * (1024, 2048 or 4096; an SKMP_FP32 strip is its refresh period).  Runs
 * mp_selfjoin over every candidate on the caller's input, one warm-up and
 * `reps` timed runs each (HIP events on `stream`, minimum kept), and records
 * the fastest for this process under the shape class (prec, ceil(log2 m),
 * ceil(log2 of the largest series' window count)); later mp_selfjoin calls
 * of that class use it (environment overrides SKMP_FP64_VARIANT,
 * SKMP_FP32_VARIANT, SKMP_MIXED_VARIANT, SKMP_STRIP still win).  Tuning a representative subset of
 * a batch tunes the batch, since the class ignores the number of series.
 * Arguments as for mp_selfjoin (all groups; P, I end up holding a complete
 * result of the last candidate; the workspace size from
 * mp_selfjoin_workspace covers every candidate).  Any precision (BF16x3 /
 * FP16x3 choose between their forms and occupancies; with 0 < refresh < 128
 * only the Hankel-direct form is a candidate); 1 <= reps <= 100.  Synchronous: waits for the GPU, and fails
 * with SKMP_EINVAL under graph capture.
 *   variant, strip, best_ms   host out (may be NULL): the choice and its time.
 */
int mp_selfjoin_autotune(const double* R, int64_t ldr, int64_t n_series, const int64_t* offsets, int32_t k,
                         int32_t m, int32_t excl, int32_t prec, int32_t refresh, double* P, int64_t* I, int64_t ldp,
                         void* workspace, size_t ws_bytes, void* stream, int32_t reps, int32_t* variant,
                         int32_t* strip, double* best_ms);

/* Workspace bytes needed by mp_abjoin (0 for an unsupported precision). */
size_t mp_abjoin_workspace(int64_t na, int64_t nb, int32_t k, int32_t m, int32_t prec);

/*
 * AB-join matrix profile (Def. 6 with distinct test and train series: the
 * join Algorithm 2 runs between a new series and a reference one, Section
 * III-B): for every subsequence of the sketched series A, the distance to its
 * nearest subsequence of the sketched series B, and optionally the converse.
 * The two series are different, so there is no trivial-match zone.  Both
 * directions come from one pass over the na' x nb' cross-distance matrix
 * (na' = na - m + 1, nb' = nb - m + 1): the diagonals j - i >= 0 walked along
 * A's rows, the diagonals i - j >= 1 along B's rows, each cell met once.
 *   RA, RB   device, k x na / k x nb doubles, row strides lda >= na, ldb >= nb
 *            (sketch_build outputs of the two series, same kind, k and seed).
 *   m        subsequence length, 4 <= m <= 2048; na, nb >= m.
 *   prec     SKMP_FP64 | SKMP_FP32 (FP32 recurrence with exact FP64 seeds every
 *            `refresh` rows, as in mp_selfjoin); others give SKMP_EINVAL.
 *   group_mask bit g selects group g (~0 = all); unselected rows are untouched.
 *   PA, IA   device out, k x na' (row stride ldpa >= na): distance from
 *            subsequence i of A to its nearest subsequence of B and that
 *            subsequence's index in B (ties to the smallest index).
 *   PB, IB   device out or both NULL, k x nb' (row stride ldpb >= nb): the same
 *            from B to A.
 * Flat subsequences are judged in each series against its own max|R^(g)|;
 * distances follow mp_selfjoin (FP64 polish of the reported neighbour).
 * Asynchronous on `stream`; the workspace comes from mp_abjoin_workspace.
 */
int mp_abjoin(const double* RA, int64_t lda, int64_t na, const double* RB, int64_t ldb, int64_t nb, int32_t k,
              int32_t m, int32_t prec, int32_t refresh, uint64_t group_mask, double* PA, int64_t* IA, int64_t ldpa,
              double* PB, int64_t* IB, int64_t ldpb, void* workspace, size_t ws_bytes, void* stream);

/* Workspace bytes needed by dim_detect (0 for invalid sizes). */
size_t dim_detect_workspace(int64_t n_train, int32_t n_dims, int32_t m);

/*
 * Discord dimension detection (Algorithm 3): for every dimension j listed in
 * dims (the group J_g* of a discord found on the sketch, Algorithm 2), the
 * z-normalised distance (Def. 3) from the test subsequence starting at i_star
 * in dimension j to its nearest subsequence of the train series in dimension
 * j (the AB-join of that one subsequence, Def. 6), and the position in dims of
 * the first dimension with the strictly largest score (0 when no score exceeds
 * 0).  Dimensions are compared as Algorithm 1 normalises them: a dimension with
 * sigma_j = 0 in its statistics is constant (all its subsequences are flat),
 * otherwise a subsequence is flat when its sigma is <= 1e-10 max|T_j - mu_j|.
 *   T_train, T_test  device, d x n_train / d x n_test, row strides ld_train,
 *            ld_test, dtype SKMP_F64 or SKMP_F32 (the same for both).
 *   stats_train, stats_test  device, d x 2 doubles (mu, sigma) of each
 *            dimension over its series (sketch_build's dim_stats of a
 *            one-series call).
 *   dims     host, n_dims row indices in [0, d) (1 <= n_dims <= 65535).
 *   i_star   start of the test subsequence, 0 <= i_star <= n_test - m.
 *   m        4 <= m <= 2048, n_train, n_test >= m.
 *   excl     0: train and test are different series (no trivial-match zone);
 *            > 0: the self-join setting -- T_test, stats_test, ld_test and
 *            n_test must equal the train ones, and train subsequences t with
 *            |t - i_star| < excl are excluded.
 *   scores, nn  device out, n_dims: the distance and the nearest train
 *            subsequence's index (+inf and -1 when every one is excluded).
 *   best     device out, one int32: the position of j* in dims.
 * Distances are FP64 from explicit differences of the normalised subsequences.
 * Asynchronous on `stream`.
 */
int dim_detect(const void* T_train, int64_t ld_train, int64_t n_train, const double* stats_train, const void* T_test,
               int64_t ld_test, int64_t n_test, const double* stats_test, int32_t dtype, int64_t d,
               const int64_t* dims, int32_t n_dims, int64_t i_star, int32_t m, int32_t excl, double* scores,
               int64_t* nn, int32_t* best, void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------- streaming
 * The streaming extension of Section III-B: the projection of Algorithm 1 is
 * run only on newly arrived samples and the self-join is updated, not redone;
 * and the point update of Section III-C.  A stream keeps, per series, a
 * sketch buffer R and profile buffers P, I with room to grow (columns
 * [start, start + capacity) of row strides ldr / ldp), and the per-dimension
 * statistics (mu, sigma) its sketch was built with: they stay frozen, so a
 * sample's sketched value never changes once written. */

/* Workspace bytes needed by sketch_append (new_offsets host, as in sketch_append). */
size_t sketch_append_workspace(int64_t d, int64_t n_series, const int64_t* new_offsets, int32_t k);

/*
 * Sketch newly arrived samples (Algorithm 1's projection, Section III-B's
 * streaming extension) with frozen statistics:
 *   R[g][dst_cols[s] + t] = sum_j S[g][j] (T_new[j][new_offsets[s] + t] - mu_sj) / sigma_sj
 * for t < new_offsets[s+1] - new_offsets[s]; sigma_sj = 0 contributes 0.
 *   T_new    device, d x N_new (N_new = new_offsets[n_series]), row stride
 *            ldt >= N_new, dtype SKMP_F64 or SKMP_F32: the new samples of every
 *            series, back to back.
 *   new_offsets host, n_series + 1, non-decreasing from 0 (a series may have
 *            no new samples).
 *   dst_cols host, n_series: the column of R that receives series s's first
 *            new sample (for a stream, start_s + samples already sketched);
 *            ascending and disjoint, dst_cols[s] + count_s <= ldr.
 *   dim_ids, k, kind, seed  as given to sketch_build.
 *   dim_stats device, n_series x d x 2 doubles: the (mu, sigma) the series'
 *            sketch was built with (sketch_build's dim_stats).
 *   flags    SKMP_FLAG_CHECK_FINITE rejects NaN/Inf among the new samples.
 * Only the new columns of R are written.  Asynchronous on `stream`.
 */
int sketch_append(const void* T_new, int32_t dtype, int64_t d, int64_t ldt, int64_t n_series,
                  const int64_t* new_offsets, const int64_t* dst_cols, const int64_t* dim_ids, int32_t k,
                  int32_t kind, uint64_t seed, const double* dim_stats, uint32_t flags, double* R, int64_t ldr,
                  void* workspace, size_t ws_bytes, void* stream);

/* Workspace bytes needed by sketch_point_update (0 for n_upd < 1). */
size_t sketch_point_update_workspace(int64_t n_upd, int32_t k);

/*
 * Point updates of a sketch (Section III-C): raising sample `col` of
 * dimension j of series s by delta raises R^(g) at that column by
 * S[g][j] * delta / sigma_sj for every group g (nothing when sigma_sj = 0).
 * Updates apply in the order given (several may hit one column).
 *   R        device, k x n_cols, row stride ldr >= n_cols.
 *   d, dim_ids  the sketch's dimensions (dim_ids host, NULL: 0..d-1).
 *   dim_stats device, n_series x d x 2 (mu, sigma), as in sketch_append.
 *   upd_series host, n_upd series indices (NULL: all 0); upd_dim host, rows
 *            in [0, d); upd_col host, columns of R in [0, n_cols); upd_delta
 *            host, finite changes of the raw samples.
 *   changed_groups host out (may be NULL): bit g set iff some update has a
 *            nonzero coefficient in group g; those groups' profiles must be
 *            recomputed (mp_selfjoin with that group mask): the detection
 *            itself is unchanged.
 * Asynchronous on `stream`.
 */
int sketch_point_update(double* R, int64_t ldr, int64_t n_cols, int32_t k, int32_t kind, uint64_t seed, int64_t d,
                        const int64_t* dim_ids, int64_t n_series, const double* dim_stats, int64_t n_upd,
                        const int64_t* upd_series, const int64_t* upd_dim, const int64_t* upd_col,
                        const double* upd_delta, uint64_t* changed_groups, void* workspace, size_t ws_bytes,
                        void* stream);

/* Workspace bytes needed by mp_selfjoin_append (n_new host, n_series entries;
 * 0 for a precision other than SKMP_FP64 / SKMP_FP32). */
size_t mp_selfjoin_append_workspace(int64_t n_series, const int64_t* n_new, int32_t k, int32_t m, int32_t prec);

/*
 * Streaming self-join update (the streaming matrix profile of Section
 * III-B's streaming extension).  Series s occupies columns
 * [starts[s], starts[s] + n_new[s]) of R, P and I.  On entry P, I hold, for
 * its first n_old[s] - m + 1 subsequences, the self-join profile of its first
 * n_old[s] samples (from mp_selfjoin or an earlier append with the same m,
 * excl and precision); on return they hold the profile of all n_new[s]
 * samples, as mp_selfjoin of the whole series would.  Only pairs with a
 * subsequence that ends in the new samples are computed.  Appends of at most
 * about 2000 / m new subsequences per series (at most 32) compute each new
 * pair directly as an exact FP64 dot product; longer ones walk the diagonal
 * bands from the first step that reaches a new subsequence, about
 * (n_new - n_old + 64 C) (n_new - m + 1) cells per group with C = 6 (FP64) or
 * 8 (FP32) diagonals per lane below 2048 new subsequences, the batch join's C
 * above that.
 *   starts   host, n_series: ascending, disjoint, starts[s] + n_new[s] <= ldr, ldp.
 *   n_old, n_new host, n_series: 0 <= n_old <= n_new, n_new >= m; n_old < m
 *            joins the series afresh; n_old = n_new leaves it untouched.
 *   k, m, excl, refresh, group_mask  as in mp_selfjoin.
 *   prec     SKMP_FP64 | SKMP_FP32; others give SKMP_EINVAL.
 * A stored entry is replaced only by a strictly nearer new neighbour, or an
 * equally near one with a smaller index.  The flat-subsequence threshold
 * (1e-10 max|R^(g)|) is taken over the samples present at each call, so a
 * subsequence whose sigma falls between two calls' thresholds keeps the
 * status it had when its entry was last written.
 * Asynchronous on `stream`.
 */
int mp_selfjoin_append(const double* R, int64_t ldr, int64_t n_series, const int64_t* starts, const int64_t* n_old,
                       const int64_t* n_new, int32_t k, int32_t m, int32_t excl, int32_t prec, int32_t refresh,
                       uint64_t group_mask, double* P, int64_t* I, int64_t ldp, void* workspace, size_t ws_bytes,
                       void* stream);

/*
 * The process's tuning table as text, one line per shape class:
 * "prec mlog nlog variant strip ms", the variant by name (e.g. f32_c16_pd2_w4:
 * diagonals per lane, prefetch depth, waves per SIMD), so a table written by
 * one build means the same kernels in another or is refused.
 * skmp_tuning_export writes at most len bytes (NUL-terminated) into buf (may
 * be NULL) and returns the size needed including the NUL; skmp_tuning_import
 * adds or replaces the entries of such text (SKMP_EINVAL on a malformed line
 * or a variant this build does not have, nothing changed); skmp_tuning_clear
 * empties the table.  Host-only, thread-safe.
 */
size_t skmp_tuning_export(char* buf, size_t len);
/* The names of the compiled tile-kernel variants of prec (any of the four
 * precisions; others: none), one per line, in the form the tuning table uses;
 * buffer and return value as for skmp_tuning_export. */
size_t skmp_tile_variants(int32_t prec, char* buf, size_t len);
int skmp_tuning_import(const char* text);
int skmp_tuning_clear(void);

/*
 * Persistent tuning cache.  skmp_tuning_save writes the table to the file
 * `path` under a first line that stamps it with the current device's
 * architecture (gcnArchName, feature flags included) and the HIP runtime
 * version; the file is written beside `path` and renamed over it.
 * skmp_tuning_load adds the file's entries to the table when its stamp equals
 * the current one and returns the number of entries loaded: 0 when the file
 * does not exist or carries another stamp (nothing changed), SKMP_EINVAL on a
 * file that is not a tuning table or holds a malformed line (nothing changed),
 * SKMP_EDEVICE when no HIP device is present to stamp against.
 * With the environment variable SKMP_TUNING_FILE set, the process's first
 * tuning lookup (a self-join, an autotuning run or skmp_tuning_export) loads
 * that file, and mp_selfjoin_autotune saves the table to it after each run
 * (its error, if the file cannot be written, is the call's).
 * Host only; a file shared by processes that tune at the same time keeps
 * the last writer's table.
 */
int skmp_tuning_save(const char* path);
int skmp_tuning_load(const char* path);

/* Workspace bytes needed by top_discords. */
size_t top_discords_workspace(int64_t n_series, const int64_t* offsets, int32_t k, int32_t m);

/*
 * Ordered list of non-overlapping discords per series (Algorithm 2, Sections IV-B/C).
 * A[i] = max over groups of P[g][i] (the first group on ties, the strict ">"
 * of Algorithm 2); repeatedly take the first maximum of A among unmasked
 * finite entries and mask |i - i*| < halfwidth (0 = m).
 *   idx, group, score device out, n_series x top_k; n_found device out, n_series.
 * Entries past n_found[s] are -1 / -1 / NaN.
 */
int top_discords(const double* P, int64_t ldp, int64_t n_series, const int64_t* offsets, int32_t k, int32_t m,
                 int32_t top_k, int32_t halfwidth, int64_t* idx, int32_t* group, double* score, int32_t* n_found,
                 void* workspace, size_t ws_bytes, void* stream);

/*
 * top_discords without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, semantics and outputs as top_discords
 * minus the workspace: the intermediate arrays live in a device array that
 * the library owns (about 25 MB, held on each device the call runs on until
 * the process ends), and the series table travels as a kernel argument, so
 * the call makes no device or pinned allocation.  Limits: n_series <= 64 and
 * offsets[n_series] <= 2^21 samples in total; larger inputs give SKMP_EINVAL
 * before anything is launched (use top_discords for them).  Every call on a
 * device shares that device's array: calls that overlap on one device (on
 * different streams, or from different threads) race and must be ordered by
 * the caller.  Call with the stream's device current.  The array needs no
 * clearing between calls (every element a call reads it first writes).
 */
int top_discords_noalloc(const double* P, int64_t ldp, int64_t n_series, const int64_t* offsets, int32_t k, int32_t m,
                         int32_t top_k, int32_t halfwidth, int64_t* idx, int32_t* group, double* score,
                         int32_t* n_found, void* stream);

/*
 * Stage timing.  When enabled, each launch of a timed stage is bracketed by HIP
 * events recorded on the stream the stage runs on; skmp_timing_read waits for
 * those events and returns the summed device time (ms) and the number of timed
 * launches since the last reset.  Timers:
 */
#define SKMP_TIMER_SKETCH 0     /* dimstats + projection of sketch_build */
#define SKMP_TIMER_SUBSTATS 1   /* scale + window statistics of mp_selfjoin */
#define SKMP_TIMER_TILES 2      /* the self-join tile kernel (FP64 or mixed) */
#define SKMP_TIMER_MERGE 3      /* key merge + FP64 polish */
#define SKMP_TIMER_DISCORDS 4   /* top_discords */
#define SKMP_TIMER_DIMDETECT 5  /* dim_detect */
#define SKMP_TIMER_COUNT 6
int skmp_timing_enable(int on);
int skmp_timing_read(int32_t which, int32_t reset, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* SKETCHMP_H */
