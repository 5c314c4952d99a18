"""Pins for the CPU oracle: closed forms, invariants, library routines, brute force.

Each test ties one oracle function to something other than itself (the
mathematics, an independent library routine, a published test vector, or a
construction whose answer is known), chosen so that a plausible slip in the
oracle (a dropped term, a wrong sign, an off-by-one, a transposed operand)
fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import datagen
from oracle import sketchmp_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ z-norm
def test_znorm_moments_and_constant_dim():
    T = datagen.tiny_series(1, 5, 300)
    T[3] = 0.1  # constant dimension (0.1 is inexact in binary: the mean is off by an ulp)
    Tb, mu, sd = O.znorm_dims(T)
    for j in (0, 1, 2, 4):
        assert abs(Tb[j].mean()) < 1e-13
        assert abs(Tb[j].var() - 1.0) < 1e-12          # population variance
    assert np.all(Tb[3] == 0.0) and sd[3] == 0.0
    assert np.allclose(mu, T.mean(axis=1), rtol=1e-14, atol=1e-12)
    assert np.allclose(sd, T.std(axis=1), rtol=1e-13)   # numpy std is ddof=0


def test_znorm_affine_invariant():
    T = datagen.tiny_series(2, 3, 200)
    a = np.array([[3.0], [0.01], [250.0]])
    b = np.array([[-4.0], [1e3], [0.5]])
    Tb1, _, _ = O.znorm_dims(T)
    Tb2, _, _ = O.znorm_dims(a * T + b)
    assert np.max(np.abs(Tb1 - Tb2)) < 1e-10


# --------------------------------------------------------------- generator
def _golden_splitmix():
    rows = []
    with open(os.path.join(GOLDEN, "splitmix64_vectors.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                s, i, v = line.split()
                rows.append((int(s), int(i), int(v)))
    return rows


def test_splitmix64_published_vectors():
    rows = _golden_splitmix()
    assert len(rows) == 8
    for seed, i, v in rows:
        assert O.splitmix64_output(seed, i) == v


def test_count_sketch_structure_and_two_universality():
    d, k = 40, 7
    S = O.sketch_coeffs("count", k, np.arange(d), seed=11)
    assert S.shape == (k, d)
    assert np.all(np.sum(S != 0.0, axis=0) == 1)            # one entry per column
    assert set(np.unique(S[S != 0.0])) <= {-1.0, 1.0}
    # Pr[h(j) = h(j')] = 1/k and Pr[s(j) = s(j')] = 1/2 over the random draw (Appendix)
    seeds = range(3000)
    coll = sum(O.count_hash(s, 3, k)[0] == O.count_hash(s, 17, k)[0] for s in seeds) / 3000
    same_sign = sum(O.count_hash(s, 3, k)[1] == O.count_hash(s, 17, k)[1] for s in seeds) / 3000
    assert abs(coll - 1.0 / k) < 0.03
    assert abs(same_sign - 0.5) < 0.04
    groups = [O.count_hash(s, 5, k)[0] for s in seeds]
    counts = np.bincount(groups, minlength=k) / 3000
    assert np.all(np.abs(counts - 1.0 / k) < 0.03)


def test_gaussian_coefficients_are_standard_normal():
    from scipy import stats
    S = O.sketch_coeffs("gauss", 16, np.arange(400), seed=5)
    x = S.ravel()
    assert abs(x.mean()) < 0.04
    assert abs(x.var() - 1.0) < 0.05
    assert stats.kstest(x, "norm").pvalue > 1e-3
    c = np.corrcoef(S)                     # rows independent of each other
    assert np.max(np.abs(c - np.eye(16))) < 0.2
    # a pure function of (seed, dim id, g): reordering dims permutes columns
    S2 = O.sketch_coeffs("gauss", 16, np.arange(400)[::-1], seed=5)
    assert np.array_equal(S2, S[:, ::-1])


# ----------------------------------------------------------------- sketch
def test_sum_sketch_is_sum_of_normalised_dims():
    T = datagen.tiny_series(3, 6, 257)
    R, S, mu, sd = O.build(T, "sum", 1, seed=0)
    Tb = (T - T.mean(axis=1, keepdims=True)) / T.std(axis=1, keepdims=True)
    assert np.max(np.abs(R[0] - Tb.sum(axis=0))) < 1e-12


def test_sketch_matches_matmul_for_every_kind():
    T = datagen.tiny_series(4, 9, 300)
    Tb, _, _ = O.znorm_dims(T)
    for kind, k in (("count", 4), ("gauss", 5), ("sum", 1)):
        S = O.sketch_coeffs(kind, k, np.arange(9), seed=77)
        R = O.sketch(Tb, S)
        assert np.max(np.abs(R - np.matmul(S, Tb))) < 1e-12


def test_identity_sketch_returns_normalised_input():
    T = datagen.tiny_series(5, 4, 100)
    Tb, _, _ = O.znorm_dims(T)
    assert np.array_equal(O.sketch(Tb, np.eye(4)), Tb)


def test_lemma1_unbiased_and_variance():
    """Lemma 1: E[s(j) R^{h(j)}_i] = T_i^(j); Var = (1/k) sum_{j' != j} (T_i^(j'))^2."""
    rng = np.random.default_rng(0)
    d, k, n = 12, 3, 4
    Tb = rng.standard_normal((d, n))
    j = 2
    est = []
    for seed in range(6000):
        S = O.sketch_coeffs("count", k, np.arange(d), seed)
        R = O.sketch(Tb, S)
        g = int(np.nonzero(S[:, j])[0][0])
        est.append(S[g, j] * R[g])
    est = np.array(est)
    var_th = (np.sum(Tb ** 2, axis=0) - Tb[j] ** 2) / k
    se = np.sqrt(var_th / len(est))
    assert np.all(np.abs(est.mean(axis=0) - Tb[j]) < 5 * se)
    assert np.all(np.abs(est.var(axis=0) / var_th - 1.0) < 0.1)


def test_update_is_linear_and_remove_add_restores():
    T = datagen.tiny_series(6, 10, 400)
    T_new = datagen.tiny_series(7, 3, 400)
    ids = np.arange(10)
    for kind, k in (("count", 3), ("gauss", 4)):
        R, S, mu, sd = O.build(T, kind, k, seed=9, dim_ids=ids)
        rem = [1, 6]
        R_upd = O.update(R, kind, k, 9, T_add=T_new, add_ids=[10, 11, 12], T_rem=T[rem], rem_ids=rem,
                         rem_mu=mu[rem], rem_sigma=sd[rem])
        keep = [q for q in range(10) if q not in rem]
        T_all = np.concatenate([T[keep], T_new])
        R_ref, _, _, _ = O.build(T_all, kind, k, seed=9, dim_ids=np.concatenate([ids[keep], [10, 11, 12]]))
        assert np.max(np.abs(R_upd - R_ref)) < 1e-12
        R_back = O.update(R_upd, kind, k, 9, T_add=T[rem], add_ids=rem)
        R_back = O.update(R_back, kind, k, 9, T_rem=T_new, rem_ids=[10, 11, 12],
                          rem_mu=T_new.mean(axis=1), rem_sigma=T_new.std(axis=1))
        assert np.max(np.abs(R_back - R)) < 1e-12


# --------------------------------------------------------------- distance
def test_distance_closed_forms():
    rng = np.random.default_rng(1)
    for m in (4, 16, 100):
        x = rng.standard_normal(m).cumsum()
        assert O.dist(x, 3.5 * x - 2.0) < 1e-6
        assert abs(O.dist(x, -x) - 2.0 * math.sqrt(m)) < 1e-12
        y = rng.standard_normal(m)
        dxy = O.dist(x, y)
        assert 0.0 <= dxy <= 2.0 * math.sqrt(m)
        rho = np.corrcoef(x, y)[0, 1]
        assert abs(dxy ** 2 - 2.0 * m * (1.0 - rho)) < 1e-9


def test_flat_subsequence_distances():
    m = 8
    c = np.full(m, 2.5)
    x = np.arange(m, dtype=float) ** 1.5
    assert O.dist(c, c + 0.0) == 0.0
    assert O.dist(c, x) == math.sqrt(m)


def _explicit_z(r, m, scale):
    """z-normalised windows written out with numpy (population sigma; flat ->
    zero vector), independent of the oracle's own normalisation code."""
    W = np.lib.stride_tricks.sliding_window_view(np.asarray(r, np.float64), m)
    mu = W.mean(axis=1, keepdims=True)
    sd = W.std(axis=1, keepdims=True)
    flat = sd[:, 0] <= O.FLAT_REL * scale
    Z = np.where(flat[:, None], 0.0, (W - mu) / np.where(sd > 0, sd, 1.0))
    return Z, flat


def _pair_series(seed):
    """A random walk with a flat stretch, a near-flat stretch (sigma tiny but
    nonzero, flat against the series' max |r|), and a scaled exact repeat."""
    rng = np.random.default_rng(seed)
    m = 12
    r = rng.standard_normal(260).cumsum() + 40.0        # max |r| ~ 40-60
    r[30:55] = 7.0                                         # flat windows 30..43
    r[90:118] = 1e-9 * rng.standard_normal(28)             # near-flat: sigma ~1e-9 < 1e-10 * max|r|
    r[200:200 + m] = -2.5 * r[150:150 + m] + 3.0           # window 200 = affine copy of 150 (rho = -1)
    r[230:230 + m] = 0.5 * r[150:150 + m] - 1.0            # window 230 = affine copy of 150 (rho = +1)
    return r, m


@pytest.mark.parametrize("seed,excl", [(11, 3), (12, 12), (13, 1)])
def test_pair_dist_reproduces_every_profile_entry(seed, excl, c_oracle):
    """The checker behind every full-size neighbour check: for every row,
    the exact distance of the pair (i, I[i]) equals the brute-force profile
    entry P[i] bit for bit (flat rows, near-flat rows, exact repeats)."""
    r, m = _pair_series(seed)
    P, I = c_oracle.profile(r, m, excl)
    fin = I >= 0
    rows = np.arange(P.size)[fin]
    d = c_oracle.pair_dist(r, m, rows, I[fin])
    assert np.array_equal(d, P[fin])
    # the constructions are seen: flat and near-flat rows at 0, the rho = +1 copy at 0
    assert P[30] == 0.0 and P[95] == 0.0
    assert P[230] < 1e-6 and I[230] == 150
    # numpy's pairwise distance with the series' scale agrees
    scale = float(np.max(np.abs(r)))
    for i in (0, 30, 95, 150, 200, 230, P.size - 1):
        assert abs(O.dist(r[i:i + m], r[I[i]:I[i] + m], scale) - P[i]) < 1e-12


@pytest.mark.parametrize("seed,excl", [(11, 3), (12, 12), (13, 1), (14, 230), (15, 262)])
def test_diagonal_reference_equals_brute_force(seed, excl, c_oracle):
    """The full-size reference (QT carried down each diagonal in double-double,
    exact recompute every 64 rows) against the brute force, on series with flat
    stretches, a near-flat window, affine copies at rho = +1 and -1, and
    exclusion zones that leave fewer admissible diagonals than one vector
    step of 8 (and rows without any partner): every profile entry within
    1e-12 * 2 sqrt(m) (squared distances near 0), every reported neighbour
    exactly as near as the brute force's, the same rows without a partner."""
    r, m = _pair_series(seed)
    P, I = c_oracle.profile(r, m, excl)
    Pd, Id = c_oracle.profile_diag(r, m, excl)
    fin = np.isfinite(P)
    assert np.array_equal(fin, np.isfinite(Pd)) and np.array_equal(Id < 0, ~fin)
    tol = 1e-12 * 2 * math.sqrt(m)
    err = np.abs(Pd[fin] - P[fin])
    sq = np.abs(Pd[fin] ** 2 - P[fin] ** 2)
    assert np.all((err <= tol) | (sq <= 2 * math.sqrt(m) * tol)), float(err.max())
    rows = np.arange(P.size)[fin]
    d = c_oracle.pair_dist(r, m, rows, Id[fin])
    assert np.all(np.abs(d - P[fin]) <= 1e-9), float(np.max(np.abs(d - P[fin])))
    assert np.all(np.abs(rows - Id[fin]) >= excl)


def test_pair_dist_matches_scipy_cdist_on_random_pairs(c_oracle):
    """pair_dist against scipy cdist of explicitly normalised windows, on
    random pairs that include flat and near-flat windows; d(x, -x) = 2 sqrt(m)."""
    r, m = _pair_series(21)
    scale = float(np.max(np.abs(r)))
    Z, flat = _explicit_z(r, m, scale)
    rng = np.random.default_rng(5)
    pi = rng.integers(0, Z.shape[0], 400)
    pj = rng.integers(0, Z.shape[0], 400)
    pi[:4] = [30, 30, 95, 150]
    pj[:4] = [40, 150, 150, 200]
    d = c_oracle.pair_dist(r, m, pi, pj)
    ref = cdist(Z, Z)[pi, pj]
    assert np.max(np.abs(d - ref)) < 1e-10
    assert d[0] == 0.0 and d[1] == math.sqrt(m) and d[2] == math.sqrt(m)
    assert abs(d[3] - 2.0 * math.sqrt(m)) < 1e-9
    assert flat[30] and flat[95] and not flat[150]


def test_flat_rule_uses_the_series_scale(c_oracle):
    """A window of tiny but nonzero sigma is flat against the series' max |r|
    (not against its own values): pair_dist, the profile and numpy's dist with
    the series' scale all treat it as flat; judged on the two windows alone it
    is a shape like any other."""
    r, m = _pair_series(31)
    scale = float(np.max(np.abs(r)))
    x, y, z = r[95:95 + m], r[100:100 + m], r[150:150 + m]
    assert O.dist(x, y, scale) == 0.0 and O.dist(x, z, scale) == math.sqrt(m)
    assert 0.0 < O.dist(x, y) < 2.0 * math.sqrt(m) and O.dist(x, y) != math.sqrt(m)
    d = c_oracle.pair_dist(r, m, np.array([95, 95]), np.array([100, 150]))
    assert d[0] == 0.0 and d[1] == math.sqrt(m)


def test_streaming_profile_with_near_flat_windows_equals_batch(c_oracle):
    """The pairwise streaming profile judges near-flat windows on the series'
    scale, as the batch profile does, so the two agree."""
    r, m = _pair_series(41)
    excl = 3
    Ps, Is = O.matrix_profile_streaming(r, m, excl, 100)
    P, I = c_oracle.profile(r, m, excl)
    assert np.max(np.abs(Ps - P)) < 1e-12
    assert np.array_equal(Is, I)
    assert Ps[95] == 0.0


def _scipy_profile(r, m, excl):
    W = np.lib.stride_tricks.sliding_window_view(r, m)
    Z = (W - W.mean(axis=1, keepdims=True)) / W.std(axis=1, keepdims=True)
    D = cdist(Z, Z)
    idx = np.arange(len(Z))
    D[np.abs(idx[:, None] - idx[None, :]) < excl] = np.inf
    return D.min(axis=1), D.argmin(axis=1)


@pytest.mark.parametrize("n,m,excl", [(120, 8, 2), (300, 16, 4), (257, 32, 8), (90, 5, 1)])
def test_profile_matches_scipy_cdist(n, m, excl, c_oracle):
    r = datagen.tiny_series(n + m, 1, n, kind="rw")[0]
    P, I = O.matrix_profile(r, m, excl)
    Ps, Is = _scipy_profile(r, m, excl)
    assert np.max(np.abs(P - Ps)) < 1e-9
    assert np.array_equal(I, Is)
    Pc, Ic = c_oracle.profile(r, m, excl)
    assert np.max(np.abs(Pc - P)) < 1e-12
    assert np.array_equal(Ic, I)
    assert len(P) == n - m + 1
    assert np.all((P >= 0) & (P <= 2 * math.sqrt(m) + 1e-12))


def test_profile_of_single_dim_sketch_is_plain_profile(c_oracle):
    """d = 1 with the sum (identity) sketch equals the profile of the raw series."""
    T = datagen.tiny_series(8, 1, 500)
    R, _, _, _ = O.build(T, "sum", 1, seed=0)
    P1, I1 = c_oracle.profile(R[0], 20, 5)
    P2, I2 = c_oracle.profile(T[0], 20, 5)
    assert np.max(np.abs(P1 - P2)) < 1e-8
    assert np.array_equal(I1, I2)
    P3, _ = c_oracle.profile(-3.0 + 0.125 * T[0], 20, 5)
    assert np.max(np.abs(P3 - P2)) < 1e-8


def test_exact_repeat_gives_zero_and_exclusion_boundary(c_oracle):
    rng = np.random.default_rng(3)
    m, excl = 10, 12          # excl > m so the copy does not overlap its source
    base = rng.standard_normal(60)
    # window at 5 repeated (scaled + shifted) at 5 + excl: admissible, distance 0
    r = base.copy()
    r[5 + excl:5 + excl + m] = 4.0 * r[5:5 + m] + 1.0
    P, I = c_oracle.profile(r, m, excl)
    assert P[5] < 1e-6 and I[5] == 5 + excl
    assert P[5 + excl] < 1e-6 and I[5 + excl] == 5
    # the same repeat at distance excl - 1 is a trivial match: it must be excluded
    r2 = base.copy()
    r2[5 + excl - 1:5 + excl - 1 + m] = 4.0 * r2[5:5 + m] + 1.0
    P2, I2 = c_oracle.profile(r2, m, excl)
    assert P2[5] > 1e-3 and I2[5] != 5 + excl - 1
    Pn, In = O.matrix_profile(r2, m, excl)
    assert np.array_equal(In, I2)


def test_flat_windows_in_profile(c_oracle):
    rng = np.random.default_rng(4)
    m, excl = 8, 2
    r = rng.standard_normal(100).cumsum()
    r[20:40] = 3.0         # flat windows 20..32 (13 of them)
    P, I = c_oracle.profile(r, m, excl)
    Pn, In = O.matrix_profile(r, m, excl)
    assert np.array_equal(I, In) and np.max(np.abs(P - Pn)) < 1e-12
    for i in range(20, 33):
        assert P[i] == 0.0
        assert I[i] == (20 if i - 20 >= excl else i + excl)   # smallest admissible flat j
    # a single flat window has only non-flat partners: sqrt(m), smallest admissible j
    r2 = rng.standard_normal(100).cumsum()
    r2[50:58] = -1.0
    P2, I2 = c_oracle.profile(r2, m, excl)
    assert P2[50] == math.sqrt(m) and I2[50] == 0


def test_row_without_partner_is_infinite(c_oracle):
    r = datagen.tiny_series(9, 1, 20)[0]
    m, excl = 8, 10           # n_sub = 13; rows 3..9 have no j with |i-j| >= 10
    P, I = c_oracle.profile(r, m, excl)
    Pn, In = O.matrix_profile(r, m, excl)
    assert np.isinf(P[5]) and I[5] == -1
    assert np.array_equal(np.isinf(P), np.isinf(Pn)) and np.array_equal(I, In)
    assert all(np.isfinite(s) for _, _, s in O.top_discords(P[None], m, 5))


# ------------------------------------------------------------------ AB-join
def _scipy_ab(ra, rb, m):
    """Row minima of the full cross-distance matrix, explicit windows through scipy."""
    def z(r):
        W = np.lib.stride_tricks.sliding_window_view(r, m)
        mu = W.mean(axis=1, keepdims=True)
        sd = W.std(axis=1, keepdims=True)
        flat = (sd[:, 0] <= 1e-10 * np.max(np.abs(r)))
        Z = np.where(flat[:, None], 0.0, (W - mu) / np.where(sd > 0, sd, 1.0))
        return Z, flat
    Za, fa = z(ra)
    Zb, fb = z(rb)
    D = cdist(Za, Zb)
    D[fa[:, None] ^ fb[None, :]] = math.sqrt(m)   # flat vs non-flat
    D[fa[:, None] & fb[None, :]] = 0.0
    return D


@pytest.mark.parametrize("na,nb,m", [(150, 300, 8), (400, 90, 16), (257, 257, 32), (40, 45, 5)])
def test_ab_join_matches_scipy_cdist(na, nb, m, c_oracle):
    ra = datagen.tiny_series(na + 7, 1, na)[0]
    rb = datagen.tiny_series(nb + 11, 1, nb)[0]
    rb[20:20 + 2 * m] = 1.5      # flat windows in b
    ra[10:10 + m + 3] = -2.0      # and in a
    D = _scipy_ab(ra, rb, m)
    P, I = O.ab_join(ra, rb, m)
    assert np.max(np.abs(P - D.min(axis=1))) < 1e-9
    assert np.array_equal(I, D.argmin(axis=1))
    Pc, Ic = c_oracle.ab_profile(ra, rb, m)
    assert np.max(np.abs(Pc - P)) < 1e-12 and np.array_equal(Ic, I)
    # the other direction is the column minima of the same matrix
    Pb, Ib = c_oracle.ab_profile(rb, ra, m)
    assert np.max(np.abs(Pb - D.min(axis=0))) < 1e-9 and np.array_equal(Ib, D.argmin(axis=0))
    assert np.all((P >= 0) & (P <= 2 * math.sqrt(m) + 1e-12))


def test_ab_join_planted_copy_and_self(c_oracle):
    rng = np.random.default_rng(12)
    m = 12
    ra = rng.standard_normal(200).cumsum()
    rb = rng.standard_normal(300).cumsum()
    rb[137:137 + m] = 2.5 * ra[40:40 + m] - 7.0       # an affine copy of a's window 40 inside b
    P, I = c_oracle.ab_profile(ra, rb, m)
    assert P[40] < 1e-6 and I[40] == 137
    Pb, Ib = c_oracle.ab_profile(rb, ra, m)
    assert Pb[137] < 1e-6 and Ib[137] == 40
    # a series joined with itself: every window is its own nearest neighbour (no exclusion zone)
    Ps, Is = c_oracle.ab_profile(ra, ra, m)
    assert np.max(Ps) < 1e-6 and np.array_equal(Is, np.arange(ra.size - m + 1))
    # reported distances are the exact pair distances
    d = c_oracle.ab_pair_dist(ra, rb, m, np.arange(ra.size - m + 1), I)
    assert np.max(np.abs(d - P)) < 1e-12


# ------------------------------------------------- dimension detection
def test_dimension_detection_finds_the_planted_dimension(c_oracle):
    """A discord planted in one dimension of the test series is attributed to it,
    and each score is the AB-join distance of the test subsequence in that
    dimension (affine-invariant: raw or normalised dimensions give the same)."""
    rng = np.random.default_rng(31)
    d, n, m = 7, 1200, 32
    T_train = datagen.tiny_series(41, d, n)
    T_test = datagen.tiny_series(42, d, 900)
    i_star, j0 = 400, 5
    loc = T_test[j0, i_star:i_star + m].std()
    T_test[j0, i_star:i_star + m] += 6 * loc * np.sin(np.linspace(0, 9 * np.pi, m) ** 1.3)
    dims = [0, 2, 3, 5, 6]
    scores, nn, best = O.dimension_detection(T_train, T_test, i_star, dims, m)
    assert dims[best] == j0
    for q, j in enumerate(dims):
        P, I = c_oracle.ab_profile(T_test[j], T_train[j], m, rows=[i_star])
        assert abs(P[0] - scores[q]) < 1e-9 and I[0] == nn[q]
    # strict ">" from 0: the first of equal scores wins
    same = np.stack([T_train[1]] * 3)
    s2, _, b2 = O.dimension_detection(same, np.stack([T_test[1]] * 3), i_star, [0, 1, 2], m)
    assert s2[0] == s2[1] == s2[2] and b2 == 0
    # self-join setting: the exclusion zone around i_star applies
    s3, nn3, _ = O.dimension_detection(T_test, None, i_star, dims, m, excl=m // 4)
    assert np.all(np.abs(nn3 - i_star) >= m // 4)
    for q, j in enumerate(dims):
        P, I = c_oracle.profile(T_test[j], m, m // 4, rows=[i_star])
        assert abs(P[0] - s3[q]) < 1e-9 and I[0] == nn3[q]


# ---------------------------------------------------------------- discords
def test_time_detection_strict_greater_keeps_first_group():
    P = np.array([[0.1, 0.9, 0.2],
                  [0.3, 0.9, 0.1],     # ties the best score: group 0 keeps it
                  [0.2, 0.4, 0.5]])
    assert O.time_detection(P) == (1, 0, 0.9)
    P2 = np.array([[0.1, 0.2], [0.4, 0.3]])
    assert O.time_detection(P2) == (0, 1, 0.4)
    assert O.time_detection(np.zeros((3, 4))) == (0, 0, 0.0)


def test_top_discords_ordering_and_masking():
    m = 3
    P = np.zeros((2, 20))
    P[0, 5] = 9.0
    P[1, 6] = 8.0       # within |i - 5| < 3 of the first pick: masked
    P[1, 12] = 7.0
    P[0, 8] = 7.0       # first maximum among 8 and 12 after masking is 8 (smallest i)
    P[0, 15] = np.inf   # no admissible partner: never reported
    out = O.top_discords(P, m, 4)
    assert [(i, g) for i, g, _ in out] == [(5, 0), (8, 0), (12, 1), (0, 0)]
    assert [s for _, _, s in out][:3] == [9.0, 7.0, 7.0]
    # the greedy list's first element is Algorithm 2's answer
    i, g, s = O.time_detection(np.where(np.isinf(P), 0, P))
    assert (i, g, s) == out[0]


def test_planted_discord_is_recovered_on_random_walk_small(c_oracle):
    w = datagen.make("random-walk-small")
    R, S, mu, sd = O.build(w.T, w.kind, w.k, w.sketch_seed)
    P, I = c_oracle.profile(R[0], w.m, w.excl)
    top = O.top_discords(P[None], w.m, 10)
    (_, _, o, _), = w.planted
    assert abs(top[0][0] - o) <= w.m // 2
    assert len(top) == 10 and all(top[q][2] >= top[q + 1][2] for q in range(9))


# ---------------------------------------------------------------- streaming
def _frozen_normalise(T, mu, sd):
    """Each row normalised with given statistics (sigma = 0: zeros), in numpy."""
    safe = np.where(sd > 0, sd, 1.0)
    return np.where((sd > 0)[:, None], (T - mu[:, None]) / safe[:, None], 0.0)


@pytest.mark.parametrize("n,m,excl,n0,flat", [
    (160, 8, 2, 0, None),           # from the first sample on
    (220, 16, 4, 150, (180, 205)),  # flat block among the new samples
    (200, 12, 40, 60, (20, 45)),    # flat block among the old samples, wide exclusion zone
    (60, 12, 40, 30, None),         # rows without an admissible partner before and after
])
def test_streaming_profile_equals_batch(n, m, excl, n0, flat, c_oracle):
    """Growing the profile sample by sample (pairwise Def. 3 distances) ends
    at the batch profile of the whole series (Def. 6), computed by the C
    brute force; rows with no admissible partner stay +inf / -1."""
    r = datagen.tiny_series(20 + n, 1, n)[0]
    if flat is not None:
        r[flat[0]:flat[1]] = 1.25
    Ps, Is = O.matrix_profile_streaming(r, m, excl, n0)
    P, I = c_oracle.profile(r, m, excl)
    assert np.array_equal(np.isinf(Ps), np.isinf(P))
    fin = np.isfinite(P)
    assert np.max(np.abs(Ps[fin] - P[fin]), initial=0.0) < 1e-12
    assert np.array_equal(Is, I)
    if n == 60:
        assert np.isinf(Ps[20]) and Is[20] == -1


def test_sketch_append_continues_the_frozen_projection():
    """New samples sketched with the build's statistics equal the matching
    columns of S times the frozen normalisation of the whole series (numpy
    matmul); appending in pieces equals appending at once."""
    T = datagen.tiny_series(21, 7, 500)
    T[3] = 2.0                                   # a constant dimension
    n0 = 300
    for kind, k in (("count", 3), ("gauss", 4), ("sum", 1)):
        R0, S, mu, sd = O.build(T[:, :n0], kind, k, seed=5)
        assert sd[3] == 0.0
        Rn = O.sketch_append(T[:, n0:], S, mu, sd)
        full = np.matmul(S, _frozen_normalise(T, mu, sd))
        assert np.max(np.abs(R0 - full[:, :n0])) < 1e-12
        assert np.max(np.abs(Rn - full[:, n0:])) < 1e-12
        Ra = O.sketch_append(T[:, n0:401], S, mu, sd)
        Rb = O.sketch_append(T[:, 401:], S, mu, sd)
        assert np.array_equal(np.concatenate([Ra, Rb], axis=1), Rn)


def test_point_update_equals_resketch_of_changed_samples():
    """Point updates (Section III-C) equal the frozen sketch of the changed
    series; a constant dimension's update changes nothing; a count sketch
    changes only the updated dimensions' groups, at the updated columns."""
    T = datagen.tiny_series(22, 6, 200)
    T[2] = -1.0
    updates = [(0, 5, 0.7), (4, 5, -1.3), (0, 5, 2.0), (2, 10, 5.0), (5, 199, 0.1), (1, 0, -0.25)]
    for kind, k in (("count", 3), ("gauss", 4), ("sum", 1)):
        R, S, mu, sd = O.build(T, kind, k, seed=3)
        Ru = O.point_update(R, S, sd, updates)
        T2 = T.copy()
        for j, t, dl in updates:
            T2[j, t] += dl
        ref = np.matmul(S, _frozen_normalise(T2, mu, sd))
        assert np.max(np.abs(Ru - ref)) < 1e-12
        cols = sorted({t for j, t, _ in updates if j != 2})
        other = np.setdiff1d(np.arange(200), cols)
        assert np.array_equal(Ru[:, other], R[:, other])
        assert np.array_equal(Ru[:, 10], R[:, 10])           # only the constant dimension touched column 10
        if kind == "count":
            groups = {int(np.nonzero(S[:, j])[0][0]) for j, _, _ in updates if j != 2}
            for g in set(range(k)) - groups:
                assert np.array_equal(Ru[g], R[g])
