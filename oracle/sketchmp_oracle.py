"""CPU FP64 oracle for the sketched matrix-profile discord path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module; it exists so that tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` can check and time the HIP library.  It
shares no code with the HIP path.

Every quantity is computed from its plain definition, in float64, with no
blocking, fusion or reordering beyond what the definition states:

* per-dimension z-normalisation (Section III-A: the sketch is applied to the
  z-normalised series; Section I: z-normalised series are unitless shapes);
* the sketch coefficients: count sketch hash pair h:[d]->[k], s:[d]->{-1,+1}
  from a 2-universal family (Section III-A, Appendix "Modeling of
  Algorithm"), the plain sum (Fig. 1), and a dense Gaussian projection;
* the sketch R = S * Tbar, one dimension at a time (Algorithm 1);
* the z-normalised Euclidean distance between subsequences (Def. 3) and the
  self-join matrix profile with its nearest-neighbour index (Def. 6, and the
  self-join variant of Section III-B), with a trivial-match exclusion zone;
* the discord time detection over the k sketched series (Algorithm 2) and
  the ordered non-overlapping discord list (Sections IV-B, IV-C);
* the add/delete-dimension update (Section III-C);
* the AB-join between a test and a train series and the discord dimension
  detection (Algorithm 3), which scores each dimension of the discord's group
  by the AB-join of the test subsequence against that dimension's train
  series;
* the streaming extension (Section III-B): the projection of newly arrived
  samples with frozen statistics, the self-join profile maintained sample by
  sample, and the point update of Section III-C.

Readings where the paper is silent:

* z-normalisation uses the population standard deviation; a constant
  dimension (sigma <= FLAT_REL * max|value|) normalises to all zeros.
* a subsequence is *flat* when its population sigma is <= FLAT_REL times the
  largest |value| of its series; a flat subsequence normalises to the zero
  vector, so dist(flat, flat) = 0 and dist(flat, non-flat) = sqrt(m) exactly.
* a pair (i, j) is a trivial match, and excluded, iff |i - j| < excl.
* nearest-neighbour ties go to the smallest j; a row with no admissible
  partner gets P = +inf and I = -1 and is never reported as a discord.
* in a stream the per-dimension (mu, sigma) stay those the sketch was built
  with, and a point update's delta is the change of the raw sample.
* the discord list is greedy on A[i] = max_g P_g[i] (first g on ties, the
  strict ">" of Algorithm 2); each pick masks |i - i*| < halfwidth (default
  m); ties in A go to the smallest i.
* the hash family is Carter-Wegman ((a x + b) mod p) mod k with p = 2^61 - 1,
  its parameters and the Gaussian coefficients drawn from SplitMix64
  (Steele, Lea & Flood, OOPSLA 2014) used as a counter-based generator, and
  Box-Muller (1958) for N(0,1).
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

FLAT_REL = 1e-10
MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15
MERSENNE61 = (1 << 61) - 1

KINDS = {"sum": 0, "count": 1, "gauss": 2}


# ---------------------------------------------------------------- z-normalise
def znorm_dims(T: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Per-dimension z-normalisation, Section III-A.

    Returns (Tbar, mu, sigma) with mu_j the mean and sigma_j the population
    standard deviation of row j.  A dimension whose sigma is at most FLAT_REL
    times its largest |value| is constant: sigma_j is reported as 0 and its
    normalised row is all zeros.
    """
    T = np.asarray(T, dtype=np.float64)
    d, n = T.shape
    mu = np.empty(d)
    sd = np.empty(d)
    Tbar = np.zeros_like(T)
    for j in range(d):
        x = T[j]
        mu[j] = math.fsum(x) / n
        dev = x - mu[j]
        sd[j] = math.sqrt(math.fsum(dev * dev) / n)
        if sd[j] <= FLAT_REL * float(np.max(np.abs(x))):
            sd[j] = 0.0
        if sd[j] > 0.0:
            Tbar[j] = dev / sd[j]
    return Tbar, mu, sd


# ----------------------------------------------------------- hash / generator
def splitmix64_output(state: int, i: int) -> int:
    """The i-th (i >= 1) SplitMix64 output for initial state ``state``.

    SplitMix64 advances its state by the golden gamma and returns a mixed
    copy; the i-th output is therefore mix(state + i * gamma), a pure function
    of (state, i): a counter-based generator.
    """
    z = (state + i * GOLDEN_GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def count_hash_params(seed: int) -> Tuple[int, int, int, int]:
    """(a, b, a2, b2) of the two Carter-Wegman functions, from outputs 1..4."""
    o = [splitmix64_output(seed, i) for i in (1, 2, 3, 4)]
    a = 1 + o[0] % (MERSENNE61 - 1)
    b = o[1] % MERSENNE61
    a2 = 1 + o[2] % (MERSENNE61 - 1)
    b2 = o[3] % MERSENNE61
    return a, b, a2, b2


def count_hash(seed: int, dim_id: int, k: int) -> Tuple[int, int]:
    """Group h(j) in [k] and sign s(j) in {-1,+1} of a dimension, Section III-A."""
    a, b, a2, b2 = count_hash_params(seed)
    g = ((a * dim_id + b) % MERSENNE61) % k
    s = 1 - 2 * (((a2 * dim_id + b2) % MERSENNE61) % 2)
    return int(g), int(s)


def gauss_coeff(seed: int, dim_id: int, g: int) -> float:
    """N(0,1) coefficient of dimension ``dim_id`` in sketch row g (Box-Muller).

    Counter c = 2 * (dim_id * 64 + g) + {1, 2} into SplitMix64(seed); the first
    output gives u1 in (0, 1], the second u2 in [0, 1).
    """
    c = 2 * (dim_id * 64 + g)
    o1 = splitmix64_output(seed, c + 1)
    o2 = splitmix64_output(seed, c + 2)
    u1 = ((o1 >> 11) + 1) * (2.0 ** -53)
    u2 = (o2 >> 11) * (2.0 ** -53)
    return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def sketch_coeffs(kind: str, k: int, dim_ids: Sequence[int], seed: int) -> np.ndarray:
    """The k x d coefficient matrix S with R = S * Tbar.

    count: column j has the single entry s(j) in row h(j) (Section III-A);
    sum:   k = 1 and every entry is +1 (Fig. 1);
    gauss: dense N(0,1) entries.
    """
    ids = [int(x) for x in dim_ids]
    S = np.zeros((k, len(ids)))
    if kind == "sum":
        if k != 1:
            raise ValueError("sum sketch has k = 1")
        S[0, :] = 1.0
    elif kind == "count":
        for col, j in enumerate(ids):
            g, s = count_hash(seed, j, k)
            S[g, col] = float(s)
    elif kind == "gauss":
        for col, j in enumerate(ids):
            for g in range(k):
                S[g, col] = gauss_coeff(seed, j, g)
    else:
        raise ValueError(kind)
    return S


# --------------------------------------------------------------------- sketch
def sketch(Tbar: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Algorithm 1: start from R = 0 and add S[:, j] * Tbar_j for each dimension j."""
    k, d = S.shape
    R = np.zeros((k, Tbar.shape[1]))
    for j in range(d):
        for g in range(k):
            if S[g, j] != 0.0:
                R[g] += S[g, j] * Tbar[j]
    return R


def build(T: np.ndarray, kind: str, k: int, seed: int, dim_ids=None):
    """z-normalise then sketch (Section III-A).  Returns (R, S, mu, sigma)."""
    d = T.shape[0]
    ids = np.arange(d) if dim_ids is None else np.asarray(dim_ids)
    Tbar, mu, sd = znorm_dims(T)
    S = sketch_coeffs(kind, k, ids, seed)
    return sketch(Tbar, S), S, mu, sd


def update(R: np.ndarray, kind: str, k: int, seed: int,
           T_add=None, add_ids=(), T_rem=None, rem_ids=(), rem_mu=(), rem_sigma=()):
    """Section III-C: R^(g) +/-= S_gj * Tbar_j for added / removed dimensions.

    Added dimensions are z-normalised over their own samples; removed ones use
    the mean and sigma they had when they were added.  The coefficients are
    the same pure functions of (seed, dimension id) used at build time.
    """
    R = np.array(R, dtype=np.float64, copy=True)
    if T_add is not None and len(add_ids):
        Tb, _, _ = znorm_dims(T_add)
        Sa = sketch_coeffs(kind, k, add_ids, seed)
        R += sketch(Tb, Sa)
    if T_rem is not None and len(rem_ids):
        T_rem = np.asarray(T_rem, dtype=np.float64)
        Tb = np.zeros_like(T_rem)
        for q in range(T_rem.shape[0]):
            if rem_sigma[q] > 0.0:
                Tb[q] = (T_rem[q] - rem_mu[q]) / rem_sigma[q]
        Sr = sketch_coeffs(kind, k, rem_ids, seed)
        R -= sketch(Tb, Sr)
    return R


# ---------------------------------------------------------- subsequence stats
def window_stats(r: np.ndarray, m: int):
    """Mean and population sigma of every length-m subsequence (Def. 2), two-pass."""
    r = np.asarray(r, dtype=np.float64)
    W = np.lib.stride_tricks.sliding_window_view(r, m)
    mu = W.mean(axis=1)
    sd = np.sqrt(((W - mu[:, None]) ** 2).mean(axis=1))
    return mu, sd


def flat_mask(r: np.ndarray, sd: np.ndarray, scale: float = None) -> np.ndarray:
    """Flat subsequences: sigma <= FLAT_REL * scale, scale = max |r| of the series
    unless given (a prefix of a longer series is judged on the whole series' scale)."""
    if scale is None:
        scale = float(np.max(np.abs(r))) if r.size else 0.0
    return sd <= FLAT_REL * scale


def znorm_windows(r: np.ndarray, m: int, scale: float = None) -> Tuple[np.ndarray, np.ndarray]:
    """All z-normalised subsequences (n-m+1) x m; flat ones are the zero vector."""
    W = np.lib.stride_tricks.sliding_window_view(np.asarray(r, np.float64), m)
    mu, sd = window_stats(r, m)
    flat = flat_mask(r, sd, scale)
    Z = np.zeros(W.shape)
    ok = ~flat
    Z[ok] = (W[ok] - mu[ok, None]) / sd[ok, None]
    return Z, flat


def dist(x: np.ndarray, y: np.ndarray, scale: float = None) -> float:
    """z-normalised Euclidean distance between two subsequences (Def. 3).

    Computed from explicit differences of the normalised vectors.  ``scale``
    is the largest |value| of the series the subsequences come from: a
    subsequence is flat when its sigma is <= FLAT_REL * scale, the rule
    matrix_profile applies.  Without a series (``scale`` None) the two
    subsequences are taken as the whole series, i.e. scale = their max |value|.
    """
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    m = x.size
    if scale is None:
        scale = max(float(np.max(np.abs(x))), float(np.max(np.abs(y))))
    zx, fx = _znorm_one(x, scale)
    zy, fy = _znorm_one(y, scale)
    if fx and fy:
        return 0.0
    if fx or fy:
        return math.sqrt(m)
    return math.sqrt(float(np.sum((zx - zy) ** 2)))


def _znorm_one(x, scale):
    mu = x.mean()
    sd = math.sqrt(float(((x - mu) ** 2).mean()))
    if sd <= FLAT_REL * scale:
        return np.zeros_like(x), True
    return (x - mu) / sd, False


def profile_row(Z: np.ndarray, flat: np.ndarray, i: int, excl: int) -> Tuple[float, int]:
    """Nearest neighbour of subsequence i among admissible j (Defs. 3, 6)."""
    n_sub, m = Z.shape
    j = np.arange(n_sub)
    ok = np.abs(j - i) >= excl
    if not ok.any():
        return math.inf, -1
    if flat[i]:
        dd = np.where(flat, 0.0, math.sqrt(m))
    else:
        dd = np.sqrt(np.sum((Z - Z[i]) ** 2, axis=1))
        dd = np.where(flat, math.sqrt(m), dd)
    dd = np.where(ok, dd, math.inf)
    jj = int(np.argmin(dd))          # first (smallest j) minimum
    return float(dd[jj]), jj


def matrix_profile(r: np.ndarray, m: int, excl: int, rows=None, scale: float = None) -> Tuple[np.ndarray, np.ndarray]:
    """Self-join matrix profile P (length n-m+1) and index I by brute force.

    Def. 6 with T_test = T_train (the self-join variant of Section III-B).
    ``rows`` restricts the computation to a subset (others are NaN / -2);
    ``scale`` overrides the flat-window scale max |r| (see flat_mask).
    """
    Z, flat = znorm_windows(r, m, scale)
    n_sub = Z.shape[0]
    P = np.full(n_sub, np.nan)
    I = np.full(n_sub, -2, dtype=np.int64)
    for i in (range(n_sub) if rows is None else rows):
        P[i], I[i] = profile_row(Z, flat, int(i), excl)
    return P, I


def ab_join(ra: np.ndarray, rb: np.ndarray, m: int, rows=None) -> Tuple[np.ndarray, np.ndarray]:
    """AB-join profile by brute force: for every subsequence of ``ra`` the
    distance to, and index of, its nearest subsequence of ``rb``.

    Def. 6 with distinct test (ra) and train (rb) series, the AB-join of
    Section III-B / Alg. 2.  The series differ, so there is no trivial-match
    zone; each series' flat subsequences are judged against its own max|r|.
    """
    Za, fa = znorm_windows(ra, m)
    Zb, fb = znorm_windows(rb, m)
    na_sub = Za.shape[0]
    P = np.full(na_sub, np.nan)
    I = np.full(na_sub, -2, dtype=np.int64)
    for i in (range(na_sub) if rows is None else rows):
        i = int(i)
        if fa[i]:
            dd = np.where(fb, 0.0, math.sqrt(m))
        else:
            dd = np.sqrt(np.sum((Zb - Za[i]) ** 2, axis=1))
            dd = np.where(fb, math.sqrt(m), dd)
        jj = int(np.argmin(dd))          # first (smallest j) minimum
        P[i], I[i] = float(dd[jj]), jj
    return P, I


def dimension_detection(T_train: np.ndarray, T_test, i_star: int, dims: Sequence[int], m: int,
                        excl: int = 0) -> Tuple[np.ndarray, np.ndarray, int]:
    """Algorithm 3: for every dimension j of ``dims`` (the group J_g* of the
    discord), the z-normalised distance from the test subsequence starting at
    ``i_star`` in dimension j to its nearest subsequence of the train series in
    dimension j (the AB-join of that one subsequence, Def. 6), and the first
    dimension with the strictly largest score (s_bsf starts at 0; if no score
    exceeds 0 the first dimension is returned).

    Dimensions are z-normalised first (Algorithm 1's normalisation).  With
    ``T_test is None`` the test series is the train series itself (the
    self-join setting): subsequences within ``excl`` of ``i_star`` are trivial
    matches.  Returns (scores, neighbour index per dimension, position of j* in
    ``dims``).
    """
    Tb_train, _, _ = znorm_dims(T_train)
    Tb_test = Tb_train if T_test is None else znorm_dims(T_test)[0]
    scores = np.zeros(len(dims))
    nn = np.zeros(len(dims), dtype=np.int64)
    for q, j in enumerate(dims):
        if T_test is None:
            P, I = matrix_profile(Tb_train[j], m, excl, rows=[i_star])
        else:
            P, I = ab_join(Tb_test[j], Tb_train[j], m, rows=[i_star])
        scores[q], nn[q] = P[i_star], I[i_star]
    s_bsf, best = 0.0, 0
    for q in range(len(dims)):
        if scores[q] > s_bsf:
            s_bsf, best = float(scores[q]), q
    return scores, nn, best


# ------------------------------------------------------------------ discords
def time_detection(P_groups: np.ndarray) -> Tuple[int, int, float]:
    """Algorithm 2 on precomputed per-group profiles: returns (i*, g*, score).

    The best-so-far score starts at 0 and only a strictly larger group score
    replaces it; within a group the top-1 index is the first maximum.
    """
    s_bsf, g_bsf, i_bsf = 0.0, 0, 0
    for g in range(P_groups.shape[0]):
        p = np.where(np.isfinite(P_groups[g]), P_groups[g], -np.inf)
        i = int(np.argmax(p))
        s = float(p[i])
        if s > s_bsf:
            g_bsf, s_bsf, i_bsf = g, s, i
    return i_bsf, g_bsf, s_bsf


def top_discords(P_groups: np.ndarray, m: int, top_k: int, halfwidth: int = 0) -> List[Tuple[int, int, float]]:
    """Ordered list of non-overlapping discords (largest score first).

    A[i] = max over groups of P_g[i] (first g on ties); repeatedly take the
    first maximum of A among unmasked finite entries and mask |i - i*| < h.
    """
    h = m if halfwidth <= 0 else halfwidth
    k, n_sub = P_groups.shape
    A = np.full(n_sub, -np.inf)
    G = np.zeros(n_sub, dtype=np.int64)
    for g in range(k):
        p = np.where(np.isfinite(P_groups[g]), P_groups[g], -np.inf)
        better = p > A
        A = np.where(better, p, A)
        G = np.where(better, g, G)
    out = []
    alive = np.isfinite(A)
    for _ in range(top_k):
        if not alive.any():
            break
        cand = np.where(alive, A, -np.inf)
        i = int(np.argmax(cand))
        out.append((i, int(G[i]), float(A[i])))
        lo, hi = max(0, i - h + 1), min(n_sub, i + h)
        alive[lo:hi] = False
    return out


# ------------------------------------------------------------------ streaming
def sketch_append(T_new: np.ndarray, S: np.ndarray, mu, sigma) -> np.ndarray:
    """Section III-B's streaming extension: the projection of Algorithm 1
    applied to newly arrived samples only.  Each dimension is normalised with
    the (mu, sigma) the sketch was built with (frozen, so earlier sketched
    values never change); sigma_j = 0 marks a constant dimension, which
    contributes 0."""
    T_new = np.asarray(T_new, dtype=np.float64)
    Tb = np.zeros_like(T_new)
    for j in range(T_new.shape[0]):
        if sigma[j] > 0.0:
            Tb[j] = (T_new[j] - mu[j]) / sigma[j]
    return sketch(Tb, S)


def point_update(R: np.ndarray, S: np.ndarray, sigma, updates) -> np.ndarray:
    """Section III-C point update: when sample t of dimension j rises by
    delta, R^(g)_t rises by S_gj times the change of the normalised sample,
    delta / sigma_j (nothing for a constant dimension).  ``updates`` is a list
    of (j, t, delta), applied in order."""
    R = np.array(R, dtype=np.float64, copy=True)
    for j, t, delta in updates:
        if sigma[j] > 0.0:
            for g in range(S.shape[0]):
                if S[g, j] != 0.0:
                    R[g, t] += S[g, j] * (delta / sigma[j])
    return R


def matrix_profile_streaming(r: np.ndarray, m: int, excl: int, n_start: int) -> Tuple[np.ndarray, np.ndarray]:
    """Self-join profile maintained while samples arrive (the streaming matrix
    profile that Section III-B's streaming extension calls for): start from
    the profile of r[:n_start] (Def. 6), then for each arriving sample the one
    new subsequence j is compared (Def. 3, pair by pair) with every earlier
    admissible subsequence i: P[j] is the smallest of those distances (first
    index on ties), and P[i] takes d(i, j) when strictly smaller.  Ties keep
    the earlier, smaller index, as the batch definition does.  Returns the
    profile after the last sample; by construction it must equal
    matrix_profile(r, m, excl)."""
    r = np.asarray(r, dtype=np.float64)
    n = r.size
    scale = float(np.max(np.abs(r))) if n else 0.0   # the series' flat-window scale, as in matrix_profile
    n0 = max(n_start, m - 1)
    if n0 >= m:
        P, I = matrix_profile(r[:n0], m, excl, scale=scale)
        P, I = list(P), list(I)
    else:
        P, I = [], []
    for t in range(n0, n):
        j = t - m + 1                     # the subsequence completed by sample t
        pj, ij = math.inf, -1
        for i in range(j):
            if j - i < excl:
                continue
            dij = dist(r[i:i + m], r[j:j + m], scale)
            if dij < pj:
                pj, ij = dij, i
            if dij < P[i]:
                P[i], I[i] = dij, j
        P.append(pj)
        I.append(ij)
    return np.asarray(P, dtype=np.float64), np.asarray(I, dtype=np.int64)
