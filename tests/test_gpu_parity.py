"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Profiles are compared element by element at sizes the oracle finishes in
seconds (several tiles, bands and strips, ragged tails); at the full
water-treatment size rows are sampled and the top-10 discords are certified
exactly from the GPU's witnesses.  FP64 tolerance: 1e-9 * 2 sqrt(m) on P (or
the squared-distance form near P = 0).  Neighbour indices must be admissible
and attain the oracle's nearest-neighbour distance; where several neighbours
are equally near, any of them is accepted.
"""
import math
import sys

import numpy as np
import pytest

import datagen
from oracle import sketchmp_oracle as O
from tests.helpers import certified_top, check_neighbours, discords_equivalent, fp64_tol, mixed_tol, profile_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    import paper_2311_03393_amd as skmp
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    skmp.lib()
    return torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _to_dev(torch, T, dev):
    return torch.from_numpy(np.ascontiguousarray(T)).to(dev)


def _run_selfjoin(torch, dev, R_np, offsets, k, m, excl, prec="fp64", refresh=0):
    import paper_2311_03393_amd as skmp
    R = _to_dev(torch, R_np, dev)
    P, I = skmp.mp_selfjoin(R, offsets, k, m, excl, prec=prec, refresh=refresh)
    torch.cuda.synchronize()
    return P.cpu().numpy(), I.cpu().numpy()


# ------------------------------------------------------------------ sketch
@pytest.mark.parametrize("case", ["random-walk-small", "water_treatment_small", "count", "batch_f32"])
def test_sketch_build_parity(dev, case):
    import torch
    import paper_2311_03393_amd as skmp
    _say("sketch parity", case)
    if case == "random-walk-small":
        w = datagen.make("random-walk-small")
    elif case == "water_treatment_small":
        w = datagen.make("water-treatment", scale=0.1)
    elif case == "count":
        w = datagen.make("random-walk-small")
        w.kind, w.k = "count", 3
    else:
        w = datagen.make("merchant-batch", scale=0.05, n_series=6)
    T = _to_dev(torch, w.T, dev)
    R, stats = skmp.sketch_build(T, w.offsets, w.k, w.kind, w.sketch_seed, dim_ids=w.dim_ids)
    torch.cuda.synchronize()
    R, stats = R.cpu().numpy(), stats.cpu().numpy()
    for s in range(w.n_series):
        a, b = w.offsets[s], w.offsets[s + 1]
        R_o, S_o, mu_o, sd_o = O.build(w.T[:, a:b].astype(np.float64), w.kind, w.k, w.sketch_seed, w.dim_ids)
        scale = max(1.0, float(np.max(np.abs(R_o))))
        assert np.max(np.abs(R[:, a:b] - R_o)) <= 1e-12 * scale
        assert np.allclose(stats[s, :, 0], mu_o, rtol=1e-13, atol=1e-12)
        assert np.allclose(stats[s, :, 1], sd_o, rtol=1e-12, atol=0)


# (input dtype, k, series lengths, d, leading columns of the view): the projection's
# column groups per lane (4 / 2 / 1), tiles across series boundaries and past the
# end, dimension slices, and the padded group counts 1, 4, 8, 16, 32, 64
PROJ_CASES = [
    ("f32", 5, [1, 3, 130, 257, 7], 9, 0),    # short series inside one tile, N % 4 = 2
    ("f32", 4, [300] * 20, 12, 0),             # 4 columns per lane, boundaries inside tiles
    ("f32", 16, [2049, 4096], 33, 0),          # odd N: 1 column per lane
    ("f32", 3, [4000], 20, 1),                 # view off by one column: unaligned rows
    ("f64", 8, [5001, 64], 51, 0),             # slices of the dimensions, ragged tail
    ("f64", 17, [1000, 23], 40, 0),            # 32 padded groups
    ("f64", 33, [515], 70, 0),                 # 64 padded groups
    ("f64", 1, [3000], 5, 1),                  # k = 1, unaligned rows
    ("f64", 64, [2000], 3000, 0),              # many dimensions: chunks of them across blocks
    ("f32", 20, [900, 1100], 2600, 0),         # the same with FP32 input and two series
]


@pytest.mark.parametrize("case", PROJ_CASES)
def test_sketch_projection_layouts(dev, case):
    import torch
    import paper_2311_03393_amd as skmp
    dt, k, lens, d, lead = case
    _say("projection layout", case)
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    N = int(offsets[-1])
    T = np.concatenate([datagen.tiny_series(70 + q, d, L) for q, L in enumerate(lens)], axis=1)
    if dt == "f32":
        T = T.astype(np.float32)
    wide = np.zeros((d, N + lead), dtype=T.dtype)
    wide[:, lead:] = T
    Tw = _to_dev(torch, wide, dev)[:, lead:]
    R, stats = skmp.sketch_build(Tw, offsets, k, "gauss", 19)
    torch.cuda.synchronize()
    R, stats = R.cpu().numpy(), stats.cpu().numpy()
    for s in range(len(lens)):
        a, b = offsets[s], offsets[s + 1]
        R_o, _, mu_o, sd_o = O.build(T[:, a:b].astype(np.float64), "gauss", k, 19)
        scale = max(1.0, float(np.max(np.abs(R_o))))
        assert np.max(np.abs(R[:, a:b] - R_o)) <= 1e-12 * scale, (case, s)
        assert np.allclose(stats[s, :, 1], sd_o, rtol=1e-12, atol=0)


def test_count_sketch_many_dimensions(dev):
    """d = 4000 dimensions of 3000 samples, count sketch k = 64: coefficients drawn on
    the device, the dimensions split into chunks across blocks."""
    import torch
    import paper_2311_03393_amd as skmp
    d, n, k = 4000, 3000, 64
    T = np.random.default_rng(5).standard_normal((d, n)).cumsum(axis=1)
    R, _ = skmp.sketch_build(_to_dev(torch, T, dev), [0, n], k, "count", 77)
    torch.cuda.synchronize()
    R_o, _, _, _ = O.build(T, "count", k, 77)
    assert np.max(np.abs(R.cpu().numpy() - R_o)) <= 1e-12 * np.max(np.abs(R_o))


@pytest.mark.parametrize("d", [1, 10, 50])
def test_sketch_default_k(dev, d):
    """k = 0 takes ceil(sqrt(d)) groups (1, 4, 8 here): the same sketch as that k
    passed explicitly, and the oracle's for that k."""
    import torch
    import paper_2311_03393_amd as skmp
    n = 700
    T = datagen.tiny_series(900 + d, d, n)
    R0, _ = skmp.sketch_build(_to_dev(torch, T, dev), [0, n], 0, "count", 5)
    k = {1: 1, 10: 4, 50: 8}[d]
    R1, _ = skmp.sketch_build(_to_dev(torch, T, dev), [0, n], k, "count", 5)
    torch.cuda.synchronize()
    assert R0.shape == (k, n) and torch.equal(R0, R1)
    R_o, _, _, _ = O.build(T, "count", k, 5)
    assert np.max(np.abs(R0.cpu().numpy() - R_o)) <= 1e-12 * max(1.0, np.max(np.abs(R_o)))


@pytest.mark.parametrize("kind,k", [("count", 7), ("count", 64), ("sum", 1)])
def test_device_drawn_coefficients_large_ids(dev, kind, k):
    """Count and sum coefficients are drawn on the device: large dimension ids
    (up to 2^61 - 2) hash exactly as in the oracle."""
    import torch
    import paper_2311_03393_amd as skmp
    d, n = 40, 700
    ids = np.array([0, 1, 2 ** 61 - 2, 2 ** 40 + 3, 999999937] + list(range(1000, 1000 + d - 5)), dtype=np.int64)
    T = datagen.tiny_series(83, d, n)
    R, _ = skmp.sketch_build(_to_dev(torch, T, dev), [0, n], k, kind, 2024, dim_ids=ids)
    torch.cuda.synchronize()
    R_o, _, _, _ = O.build(T, kind, k, 2024, ids)
    assert np.max(np.abs(R.cpu().numpy() - R_o)) <= 1e-12 * max(1.0, np.max(np.abs(R_o)))
    R2, _ = skmp.sketch_build(_to_dev(torch, T, dev), [0, n], k, kind, 2024)   # ids 0 .. d - 1
    torch.cuda.synchronize()
    R2_o, _, _, _ = O.build(T, kind, k, 2024, np.arange(d))
    assert np.max(np.abs(R2.cpu().numpy() - R2_o)) <= 1e-12 * max(1.0, np.max(np.abs(R2_o)))


@pytest.mark.parametrize("n", [4096, 4097])
def test_update_dims_fp32_input(dev, n):
    """Add and remove with FP32 input: 4 columns per lane (n = 4096) and 1 (odd n)."""
    import torch
    import paper_2311_03393_amd as skmp
    d, k = 24, 6
    T = datagen.tiny_series(81, d, n).astype(np.float32)
    T_add = datagen.tiny_series(82, 3, n).astype(np.float32)
    ids = np.arange(d)
    rem = np.array([2, 5, 11, 20])
    R, stats = skmp.sketch_build(_to_dev(torch, T, dev), [0, n], k, "gauss", 23, dim_ids=ids)
    Td = _to_dev(torch, T, dev)
    rem_idx = torch.from_numpy(rem).to(dev)
    skmp.sketch_update_dims(R, "gauss", k, 23, T_add=_to_dev(torch, T_add, dev), add_ids=[30, 31, 32],
                            T_rem=Td[rem_idx].contiguous(), rem_ids=rem,
                            rem_stats=stats[0].index_select(0, rem_idx).contiguous())
    torch.cuda.synchronize()
    keep = np.setdiff1d(ids, rem)
    R_ref, _, _, _ = O.build(np.concatenate([T[keep], T_add]).astype(np.float64), "gauss", k, 23,
                             np.concatenate([keep, [30, 31, 32]]))
    assert np.max(np.abs(R.cpu().numpy() - R_ref)) <= 1e-11 * np.max(np.abs(R_ref))


def test_sketch_constant_dimension_and_nonfinite(dev):
    import torch
    import paper_2311_03393_amd as skmp
    T = datagen.tiny_series(11, 4, 500)
    T[2] = 0.1
    R, stats = skmp.sketch_build(_to_dev(torch, T, dev), [0, 500], 2, "gauss", 5)
    torch.cuda.synchronize()
    R_o, _, mu_o, sd_o = O.build(T, "gauss", 2, 5)
    assert stats[0, 2, 1].item() == 0.0 and sd_o[2] == 0.0
    assert np.max(np.abs(R.cpu().numpy() - R_o)) < 1e-12 * np.max(np.abs(R_o))
    T[1, 17] = np.nan
    with pytest.raises(skmp.SketchMPError):
        skmp.sketch_build(_to_dev(torch, T, dev), [0, 500], 2, "gauss", 5, check_finite=True)


def test_count_sketch_more_than_64_groups(dev, c_oracle):
    """k = 100 (the k = ceil(sqrt d) of d = 10,000 in Section IV-A): the count
    sketch is projected in blocks of 64 groups, the self-join runs its groups in
    blocks of 64, top_discords combines all 100; each against the oracle."""
    import torch
    import paper_2311_03393_amd as skmp
    d, n, k, m, excl, seed = 400, 1200, 100, 32, 8, 17
    T = datagen.tiny_series(61, d, n)
    R, _ = skmp.sketch_build(_to_dev(torch, T, dev), [0, n], k, "count", seed)
    P, I = skmp.mp_selfjoin(R, [0, n], k, m, excl)
    idx, grp, score, nf = skmp.top_discords(P, [0, n], k, m, 5)
    torch.cuda.synchronize()
    R_o, _, _, _ = O.build(T, "count", k, seed)
    Rg = R.cpu().numpy()
    assert np.max(np.abs(Rg - R_o)) <= 1e-12 * np.max(np.abs(R_o))
    n_sub = n - m + 1
    P, I = P.cpu().numpy()[:, :n_sub], I.cpu().numpy()[:, :n_sub]
    Ps = []
    for g in range(k):
        P_o, _ = c_oracle.profile(R_o[g], m, excl)
        Ps.append(P_o)
        if g in (0, 1, 63, 64, 65, 99):
            ok, err = profile_close(P[g], P_o, m, fp64_tol(m))
            assert ok.all(), (g, err)
            check_neighbours(c_oracle, R_o[g], m, excl, np.arange(n_sub), I[g], P_o, fp64_tol(m))
    Ps = np.stack(Ps)
    ok, err = profile_close(P, Ps, m, fp64_tol(m))
    assert ok.all(), err
    ref = O.top_discords(Ps, m, 5)
    got = [(int(i), int(g), float(v)) for i, g, v in zip(idx[0].cpu(), grp[0].cpu(), score[0].cpu())]
    A_o = np.max(np.where(np.isfinite(Ps), Ps, -np.inf), axis=0)
    discords_equivalent(got, ref, A_o, m, fp64_tol(m))
    assert int(nf[0]) == 5 and all(0 <= g < k for _, g, _ in got)


@pytest.mark.parametrize("bad,prec", [(np.nan, "fp64"), (np.inf, "fp64"), (-np.inf, "fp64"), (np.nan, "fp32"),
                                      (np.inf, "bf16x3")])
def test_nonfinite_input_is_marked_without_the_check_flag(dev, c_oracle, bad, prec):
    """Without SKMP_FLAG_CHECK_FINITE (no host read-back: capture-safe) a NaN
    or Inf sample is never dropped silently: its dimension's statistics come
    back as (NaN, NaN), the sketch of that series is NaN, its windows get
    P = NaN and I = -1 (no admissible partner would be +inf), they have no
    discords, and the other series of the batch are unaffected."""
    import torch
    import paper_2311_03393_amd as skmp
    m, excl, k = 32, 8, 2
    lens = [900, 1100]
    offsets = np.concatenate([[0], np.cumsum(lens)])
    T = np.concatenate([datagen.tiny_series(300 + q, 4, L) for q, L in enumerate(lens)], axis=1)
    T[1, offsets[1] + 517] = bad          # series 1, dimension 1
    R, stats = skmp.sketch_build(_to_dev(torch, T, dev), offsets, k, "gauss", 9)
    P, I = skmp.mp_selfjoin(R, offsets, k, m, excl, prec=prec)
    idx, grp, score, nf = skmp.top_discords(P, offsets, k, m, 5)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    assert np.isnan(st[1, 1]).all() and np.isfinite(st[1, [0, 2, 3]]).all() and np.isfinite(st[0]).all()
    Rn, P, I = R.cpu().numpy(), P.cpu().numpy(), I.cpu().numpy()
    a, b = offsets[1], offsets[2]
    n_sub1 = lens[1] - m + 1
    assert np.isnan(Rn[:, a:b]).all()
    assert np.isnan(P[:, a:a + n_sub1]).all() and (I[:, a:a + n_sub1] == -1).all()
    assert int(nf[1]) == 0 and (idx[1].cpu().numpy() == -1).all()
    # series 0 is the sketch and profile of its own samples
    R_o, _, _, _ = O.build(T[:, :offsets[1]], "gauss", k, 9)
    assert np.max(np.abs(Rn[:, :offsets[1]] - R_o)) < 1e-12 * np.max(np.abs(R_o))
    n_sub0 = lens[0] - m + 1
    tol = fp64_tol(m) if prec == "fp64" else mixed_tol(m)
    for g in range(k):
        P_o, _ = c_oracle.profile(R_o[g], m, excl)
        ok, err = profile_close(P[g, :n_sub0], P_o, m, tol)
        assert ok.all(), err
        check_neighbours(c_oracle, R_o[g], m, excl, np.arange(n_sub0), I[g, :n_sub0], P_o, tol)
    assert int(nf[0]) == 5


# --------------------------------------------------------------- self-join
SMALL = [  # (n, m, excl, k, seed)
    (300, 16, 4, 2, 1),
    (777, 8, 2, 1, 2),
    (1500, 32, 8, 3, 3),
    (4100, 64, 16, 2, 4),      # several bands (512 diagonals each) and strips
    (2600, 100, 25, 1, 5),
    (700, 4, 1, 1, 6),         # smallest m, excl = 1
    (530, 64, 470, 1, 7),      # excl close to n_sub: few admissible pairs, rows without partners
]


@pytest.mark.parametrize("n,m,excl,k,seed", SMALL)
def test_selfjoin_fp64_matches_oracle(dev, c_oracle, n, m, excl, k, seed):
    import torch
    _say("selfjoin fp64", n, m, excl, k, seed)
    T = datagen.tiny_series(seed, 5, n)
    R_np, _, _, _ = O.build(T, "gauss", k, seed)
    P, I = _run_selfjoin(torch, dev, R_np, [0, n], k, m, excl)
    n_sub = n - m + 1
    tol = fp64_tol(m)
    for g in range(k):
        P_o, I_o = c_oracle.profile(R_np[g], m, excl)
        ok, err = profile_close(P[g, :n_sub], P_o, m, tol)
        assert ok.all(), f"group {g}: {np.count_nonzero(~ok)} rows out of tolerance, max err {err}"
        check_neighbours(c_oracle, R_np[g], m, excl, np.arange(n_sub), I[g, :n_sub], P_o, tol)
        assert np.all(np.isnan(P[g, n_sub:])) and np.all(I[g, n_sub:] == -2)  # tail untouched


def test_selfjoin_random_walk_small_and_top10(dev, c_oracle):
    import torch
    import paper_2311_03393_amd as skmp
    w = datagen.make("random-walk-small")
    R_np, _, _, _ = O.build(w.T, w.kind, w.k, w.sketch_seed)
    R = _to_dev(torch, R_np, dev)
    P, I = skmp.mp_selfjoin(R, w.offsets, w.k, w.m, w.excl)
    idx, grp, score, nf = skmp.top_discords(P, w.offsets, w.k, w.m, 10)
    torch.cuda.synchronize()
    P, I = P.cpu().numpy(), I.cpu().numpy()
    P_o, I_o = c_oracle.profile(R_np[0], w.m, w.excl)
    n_sub = len(P_o)
    ok, err = profile_close(P[0, :n_sub], P_o, w.m, fp64_tol(w.m))
    assert ok.all(), err
    top_o = O.top_discords(P_o[None], w.m, 10)
    gpu = [(int(i), int(g), float(s)) for i, g, s in zip(idx[0].cpu(), grp[0].cpu(), score[0].cpu())]
    assert int(nf[0]) == 10
    assert [i for i, _, _ in gpu] == [i for i, _, _ in top_o]
    (_, _, o, _), = w.planted
    assert abs(gpu[0][0] - o) <= w.m // 2


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("seed", [12, 13, 14])
def test_selfjoin_flat_windows_and_exclusion_boundary(dev, c_oracle, prec, seed):
    """Flat stretches, a single flat window, scaled exact repeats (rho = 1 up to
    rounding: the 32-bit keys must stay positive) and a neighbour just outside
    the exclusion zone, in every precision."""
    import torch
    from tests.helpers import mixed_tol
    rng = np.random.default_rng(seed)
    m, excl = 16, 4
    r = rng.standard_normal(3000).cumsum()
    r[400:460] = 2.0            # long flat stretch
    r[1500:1516] = -7.0         # single flat window (its partners are the flat stretch above)
    r[2000:2016] = 3.0 * r[1000:1016] + 5.0   # exact repeat far away: P = 0
    r[2600:2616] = 0.25 * r[2300:2316] - 1.0  # another scaled repeat
    # window 2800 + excl = 1.1 (window 2800) + 1: an exact repeat excl apart (the windows overlap, so the
    # samples are filled in order; a factor of 2 would grow the values 16-fold over the window, and the
    # 16-bit recurrences lose accuracy on diagonals that cross such a jump in variance)
    for t in range(m):
        r[2800 + excl + t] = 1.1 * r[2800 + t] + 1.0
    R_np = r[None, :]
    _say("flat/repeats", prec, seed)
    P, I = _run_selfjoin(torch, dev, R_np, [0, r.size], 1, m, excl, prec=prec)
    P_o, I_o = c_oracle.profile(r, m, excl)
    n_sub = len(P_o)
    tol = fp64_tol(m) if prec == "fp64" else mixed_tol(m)
    ok, err = profile_close(P[0, :n_sub], P_o, m, tol)
    assert ok.all(), (np.nonzero(~ok)[0][:10], err)
    flat = np.arange(400, 460 - m + 1)
    assert np.all(P[0, flat] == 0.0) and np.array_equal(I[0, flat], I_o[flat])
    assert P[0, 1500] == 0.0 and I[0, 1500] == 400     # flat: nearest admissible flat window
    assert P[0, 1000] < 1e-5 and I[0, 1000] == 2000
    assert P[0, 2300] < 1e-5 and I[0, 2300] == 2600
    assert P[0, 2800] < 1e-5 and I[0, 2800] == 2800 + excl   # partner exactly at the zone's edge
    check_neighbours(c_oracle, r, m, excl, np.arange(n_sub), I[0, :n_sub], P_o, tol)


def test_selfjoin_batched_uneven_series(dev, c_oracle):
    import torch
    m, excl, k = 32, 8, 2
    lens = [40, 700, 33, 2500, 1200, 64, 5000]     # includes n_sub < excl + 1 (no admissible pair)
    offsets = np.concatenate([[0], np.cumsum(lens)])
    T = np.concatenate([datagen.tiny_series(100 + q, 3, L) for q, L in enumerate(lens)], axis=1)
    R_np = np.zeros((k, offsets[-1]))
    for s in range(len(lens)):
        a, b = offsets[s], offsets[s + 1]
        R_np[:, a:b], _, _, _ = O.build(T[:, a:b], "gauss", k, 77)
    P, I = _run_selfjoin(torch, dev, R_np, offsets, k, m, excl)
    for s in range(len(lens)):
        a, b = offsets[s], offsets[s + 1]
        n_sub = b - a - m + 1
        for g in range(k):
            P_o, I_o = c_oracle.profile(R_np[g, a:b], m, excl)
            ok, err = profile_close(P[g, a:a + n_sub], P_o, m, fp64_tol(m))
            assert ok.all(), (s, g, err)
            check_neighbours(c_oracle, R_np[g, a:b], m, excl, np.arange(n_sub), I[g, a:a + n_sub], P_o, fp64_tol(m))


def test_selfjoin_group_mask_and_repeatability(dev):
    import torch
    import paper_2311_03393_amd as skmp
    T = datagen.tiny_series(21, 6, 3000)
    R_np, _, _, _ = O.build(T, "gauss", 4, 3)
    R = _to_dev(torch, R_np, dev)
    P1, I1 = skmp.mp_selfjoin(R, [0, 3000], 4, 48, 12)
    P2, I2 = skmp.mp_selfjoin(R, [0, 3000], 4, 48, 12)
    P3, I3 = skmp.mp_selfjoin(R, [0, 3000], 4, 48, 12, group_mask=0b0101)
    torch.cuda.synchronize()
    same = lambda a, b: torch.allclose(a, b, rtol=0.0, atol=0.0, equal_nan=True)   # bitwise, NaN tails equal
    assert same(P1, P2) and torch.equal(I1, I2)               # deterministic
    assert same(P3[0], P1[0]) and same(P3[2], P1[2]) and torch.equal(I3[0], I1[0])
    assert torch.isnan(P3[1]).all() and torch.isnan(P3[3]).all()   # untouched groups


def test_top_discords_matches_oracle_on_same_profiles(dev):
    import torch
    import paper_2311_03393_amd as skmp
    rng = np.random.default_rng(5)
    k, m = 3, 10
    lens = [300, 80, 1000]
    offsets = np.concatenate([[0], np.cumsum(lens)])
    P = np.full((k, offsets[-1]), np.nan)
    for s, L in enumerate(lens):
        a = offsets[s]
        n_sub = L - m + 1
        x = np.round(rng.random((k, n_sub)) * 20) / 4     # many exact ties
        x[rng.random((k, n_sub)) < 0.05] = np.inf           # rows without partners
        P[:, a:a + n_sub] = x
    idx, grp, score, nf = skmp.top_discords(_to_dev(torch, P, dev), offsets, k, m, 12)
    torch.cuda.synchronize()
    for s, L in enumerate(lens):
        a = offsets[s]
        n_sub = L - m + 1
        ref = O.top_discords(P[:, a:a + n_sub], m, 12)
        got = [(int(i), int(g), float(v)) for i, g, v in zip(idx[s].cpu(), grp[s].cpu(), score[s].cpu())][:len(ref)]
        assert int(nf[s]) == len(ref)
        assert got == ref


@pytest.mark.parametrize("case", ["wide_mask", "exhaust", "long_series"])
def test_top_discords_block_maxima_edge_cases(dev, case):
    """The selection keeps maxima per block of windows (256 windows, more for
    series above 2^20 windows): masks wider than a block, ties across block
    boundaries, more picks than the series can hold, series without windows,
    and a series long enough to need larger blocks."""
    import torch
    import paper_2311_03393_amd as skmp
    rng = np.random.default_rng({"wide_mask": 6, "exhaust": 7, "long_series": 8}[case])
    if case == "wide_mask":
        k, m, top_k, hw = 2, 700, 25, 0
        lens = [30000, 500, 9000]
    elif case == "exhaust":
        k, m, top_k, hw = 3, 64, 200, 1000
        lens = [5000, 2048, 63]
    else:
        k, m, top_k, hw = 2, 300, 20, 0
        lens = [1_200_299]
    _say("top discords", case, lens, m, top_k, hw)
    offsets = np.concatenate([[0], np.cumsum(lens)])
    P = np.full((k, offsets[-1]), np.nan)
    for s, L in enumerate(lens):
        a = offsets[s]
        n_sub = max(L - m + 1, 0)
        x = np.round(rng.random((k, n_sub)) * 8) / 2      # many exact ties, also across blocks
        x[rng.random((k, n_sub)) < 0.02] = np.inf
        P[:, a:a + n_sub] = x
    idx, grp, score, nf = skmp.top_discords(_to_dev(torch, P, dev), offsets, k, m, top_k, halfwidth=hw)
    torch.cuda.synchronize()
    for s, L in enumerate(lens):
        a = offsets[s]
        n_sub = max(L - m + 1, 0)
        ref = O.top_discords(P[:, a:a + n_sub], m, top_k, halfwidth=hw) if n_sub else []
        got = [(int(i), int(g), float(v)) for i, g, v in zip(idx[s].cpu(), grp[s].cpu(), score[s].cpu())][:len(ref)]
        assert int(nf[s]) == len(ref), (case, s, int(nf[s]), len(ref))
        assert got == ref, (case, s)


# ------------------------------------------------------------------ update
def test_update_dims_matches_rebuild(dev, c_oracle):
    import torch
    import paper_2311_03393_amd as skmp
    w = datagen.make("large-series", scale=1.0 / 256)           # d = 256, n = 4096, same recipe as the large case
    n = w.T.shape[1]
    ids = w.dim_ids
    rem = w.update["rem_ids"]
    T_add = w.update["T_add"]
    add_ids = w.update["add_ids"]
    T = _to_dev(torch, w.T, dev)
    R, stats = skmp.sketch_build(T, w.offsets, w.k, w.kind, w.sketch_seed, dim_ids=ids)
    rem_stats = stats[0, rem].contiguous()
    add_stats, mask = skmp.sketch_update_dims(R, w.kind, w.k, w.sketch_seed, T_add=_to_dev(torch, T_add, dev),
                                              add_ids=add_ids, T_rem=T[rem].contiguous(), rem_ids=rem,
                                              rem_stats=rem_stats)
    torch.cuda.synchronize()
    keep = np.setdiff1d(ids, rem)
    R_ref, _, mu_a, sd_a = O.build(np.concatenate([w.T[keep], T_add]), w.kind, w.k, w.sketch_seed,
                                   np.concatenate([keep, add_ids]))
    Rg = R.cpu().numpy()
    assert np.max(np.abs(Rg - R_ref)) <= 1e-11 * np.max(np.abs(R_ref))
    assert mask == (1 << w.k) - 1
    assert np.allclose(add_stats.cpu().numpy()[:, 1], sd_a[-len(add_ids):], rtol=1e-12)
    # the profile of the updated sketch equals the profile of a fresh build
    P_u, I_u = skmp.mp_selfjoin(R, w.offsets, w.k, w.m, w.excl, group_mask=0b11)
    torch.cuda.synchronize()
    for g in range(2):
        P_o, _ = c_oracle.profile(R_ref[g], w.m, w.excl)
        ok, err = profile_close(P_u[g].cpu().numpy()[:len(P_o)], P_o, w.m, 1e-8 * 2 * math.sqrt(w.m))
        assert ok.all(), err


def test_update_count_sketch_changed_groups(dev):
    import torch
    import paper_2311_03393_amd as skmp
    T = datagen.tiny_series(31, 12, 800)
    ids = np.arange(12)
    R, stats = skmp.sketch_build(_to_dev(torch, T, dev), [0, 800], 5, "count", 9, dim_ids=ids)
    Tn = datagen.tiny_series(32, 2, 800)
    _, mask = skmp.sketch_update_dims(R, "count", 5, 9, T_add=_to_dev(torch, Tn, dev), add_ids=[40, 41])
    expect = 0
    for i in (40, 41):
        expect |= 1 << O.count_hash(9, i, 5)[0]
    assert mask == expect
    torch.cuda.synchronize()
    R_ref, _, _, _ = O.build(np.concatenate([T, Tn]), "count", 5, 9, np.concatenate([ids, [40, 41]]))
    assert np.max(np.abs(R.cpu().numpy() - R_ref)) < 1e-12 * np.max(np.abs(R_ref))


# -------------------------------------------------- full water-treatment size
def test_selfjoin_c1_full_size_sampled_and_certified(dev, c_oracle):
    import torch
    import paper_2311_03393_amd as skmp
    w = datagen.make("water-treatment")
    _say("water-treatment full size", w.T.shape)
    T = _to_dev(torch, w.T, dev)
    R, _ = skmp.sketch_build(T, w.offsets, w.k, w.kind, w.sketch_seed, dim_ids=w.dim_ids)
    P, I = skmp.mp_selfjoin(R, w.offsets, w.k, w.m, w.excl)
    idx, grp, score, nf = skmp.top_discords(P, w.offsets, w.k, w.m, 10)
    torch.cuda.synchronize()
    R_np = R.cpu().numpy()
    R_o, _, _, _ = O.build(w.T, w.kind, w.k, w.sketch_seed, w.dim_ids)
    assert np.max(np.abs(R_np - R_o)) <= 1e-12 * np.max(np.abs(R_o))
    n_sub = w.T.shape[1] - w.m + 1
    P, I = P.cpu().numpy()[:, :n_sub], I.cpu().numpy()[:, :n_sub]
    tol = fp64_tol(w.m)
    rng = np.random.default_rng(0)
    rows = np.unique(np.concatenate([rng.choice(n_sub, 96, replace=False), [0, 1, n_sub - 2, n_sub - 1],
                                     [o + q for (_, _, o, _) in w.planted for q in (-5, 0, 5)]]))
    for g in range(w.k):
        P_o, _ = c_oracle.profile(R_np[g], w.m, w.excl, rows=rows)
        ok, err = profile_close(P[g, rows], P_o, w.m, tol)
        assert ok.all(), (g, err)
        check_neighbours(c_oracle, R_np[g], w.m, w.excl, rows, I[g, rows], P_o, tol)
    picks, exact, U = certified_top(c_oracle, R_np, w.m, w.excl, P, I, 10)
    # the GPU's reported distance is the exact distance of its reported neighbour
    fin = np.isfinite(P)
    assert np.max(np.abs(P[fin] - U[fin])) < 1e-9
    gpu = [(int(i), int(g), float(s)) for i, g, s in zip(idx[0].cpu(), grp[0].cpu(), score[0].cpu())]
    A_ex = np.full(n_sub, -np.inf)
    for i, (v, g) in exact.items():
        A_ex[i] = v
    if [i for i, _, _ in gpu] != [i for i, _, _ in picks]:
        # near ties: accept an eps-greedy sequence on the exact values
        for (i, g, s), (io, go, so) in zip(gpu, picks):
            assert i in exact and exact[i][0] >= so - 2 * tol
    _say("water-treatment top10", [i for i, _, _ in gpu])


# ------------------------------------------------------- mixed precisions
MIXED = ["fp32", "bf16x3", "fp16x3"]


@pytest.mark.parametrize("prec", MIXED)
@pytest.mark.parametrize("n,m,excl,k,seed", SMALL)
def test_selfjoin_mixed_matches_oracle(dev, c_oracle, prec, n, m, excl, k, seed):
    import torch
    from tests.helpers import mixed_tol
    _say("selfjoin", prec, n, m, excl, k, seed)
    T = datagen.tiny_series(seed, 5, n)
    R_np, _, _, _ = O.build(T, "gauss", k, seed)
    P, I = _run_selfjoin(torch, dev, R_np, [0, n], k, m, excl, prec=prec)
    n_sub = n - m + 1
    tol = mixed_tol(m)
    for g in range(k):
        P_o, _ = c_oracle.profile(R_np[g], m, excl)
        ok, err = profile_close(P[g, :n_sub], P_o, m, tol)
        assert ok.all(), f"{prec} group {g}: {np.count_nonzero(~ok)} rows out of tolerance, max err {err}"
        check_neighbours(c_oracle, R_np[g], m, excl, np.arange(n_sub), I[g, :n_sub], P_o, tol)
        # the reported distance is the exact FP64 distance of the reported neighbour
        fin = I[g, :n_sub] >= 0
        if fin.any():
            dd = c_oracle.pair_dist(R_np[g], m, np.arange(n_sub)[fin], I[g, :n_sub][fin])
            assert np.max(np.abs(dd - P[g, :n_sub][fin])) < 1e-9


@pytest.mark.parametrize("prec", MIXED)
def test_selfjoin_mixed_batched_flat_and_top10(dev, c_oracle, prec):
    import torch
    import paper_2311_03393_amd as skmp
    from tests.helpers import mixed_tol
    m, excl, k = 32, 8, 2
    lens = [40, 700, 2500, 64, 3000]
    offsets = np.concatenate([[0], np.cumsum(lens)])
    T = np.concatenate([datagen.tiny_series(200 + q, 3, L) for q, L in enumerate(lens)], axis=1)
    T[:, offsets[4] + 500:offsets[4] + 560] = 1.0         # constant stretch: flat windows in every group
    R_np = np.zeros((k, offsets[-1]))
    for s in range(len(lens)):
        a, b = offsets[s], offsets[s + 1]
        R_np[:, a:b], _, _, _ = O.build(T[:, a:b], "gauss", k, 77)
    R = _to_dev(torch, R_np, dev)
    P, I = skmp.mp_selfjoin(R, offsets, k, m, excl, prec=prec)
    idx, grp, score, nf = skmp.top_discords(P, offsets, k, m, 10)
    torch.cuda.synchronize()
    P, I = P.cpu().numpy(), I.cpu().numpy()
    tol = mixed_tol(m)
    for s in range(len(lens)):
        a, b = offsets[s], offsets[s + 1]
        n_sub = b - a - m + 1
        Ps = []
        for g in range(k):
            P_o, _ = c_oracle.profile(R_np[g, a:b], m, excl)
            ok, err = profile_close(P[g, a:a + n_sub], P_o, m, tol)
            assert ok.all(), (s, g, err)
            check_neighbours(c_oracle, R_np[g, a:b], m, excl, np.arange(n_sub), I[g, a:a + n_sub], P_o, tol)
            Ps.append(P_o)
        if n_sub > 0:
            ref = O.top_discords(np.stack(Ps), m, 10)
            A_o = np.max(np.where(np.isfinite(np.stack(Ps)), np.stack(Ps), -np.inf), axis=0)
            got = [(int(i), int(g), float(v)) for i, g, v in zip(idx[s].cpu(), grp[s].cpu(), score[s].cpu())][:len(ref)]
            assert int(nf[s]) == len(ref)
            discords_equivalent(got, ref, A_o, m, tol)


@pytest.mark.parametrize("refresh", [100, 512, 4096])
def test_selfjoin_fp32_refresh_periods(dev, c_oracle, refresh):
    """FP32 with a refresh period that is not a multiple of the tile length (a
    unit is one period), one that re-seeds inside a unit, and one longer than
    the series (no re-seed at all)."""
    import torch
    from tests.helpers import mixed_tol
    n, m, excl, k, seed = 5200, 48, 12, 2, 21
    _say("fp32 refresh", refresh, n, m)
    T = datagen.tiny_series(seed, 4, n)
    R_np, _, _, _ = O.build(T, "gauss", k, seed)
    P, I = _run_selfjoin(torch, dev, R_np, [0, n], k, m, excl, prec="fp32", refresh=refresh)
    n_sub = n - m + 1
    tol = mixed_tol(m)
    for g in range(k):
        P_o, _ = c_oracle.profile(R_np[g], m, excl)
        ok, err = profile_close(P[g, :n_sub], P_o, m, tol)
        assert ok.all(), f"refresh {refresh} group {g}: {np.count_nonzero(~ok)} rows out of tolerance, max err {err}"
        check_neighbours(c_oracle, R_np[g], m, excl, np.arange(n_sub), I[g, :n_sub], P_o, tol)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_selfjoin_long_windows_and_many_groups(dev, c_oracle, prec):
    """Window lengths near the limit (the exact seeds stage several chunks of
    the window; the padding covers m - 1 samples past the end) and k = 64."""
    import torch
    from tests.helpers import mixed_tol
    tol_of = fp64_tol if prec == "fp64" else mixed_tol
    for (n, m, excl, k, seed) in [(4500, 1500, 375, 2, 51), (5000, 2048, 512, 1, 52), (700, 16, 4, 64, 53)]:
        _say("long/many", prec, n, m, excl, k)
        T = datagen.tiny_series(seed, 6, n)
        R_np, _, _, _ = O.build(T, "gauss", k, seed)
        P, I = _run_selfjoin(torch, dev, R_np, [0, n], k, m, excl, prec=prec)
        n_sub = n - m + 1
        tol = tol_of(m)
        for g in range(k):
            P_o, _ = c_oracle.profile(R_np[g], m, excl)
            ok, err = profile_close(P[g, :n_sub], P_o, m, tol)
            assert ok.all(), (n, m, k, g, err)
            check_neighbours(c_oracle, R_np[g], m, excl, np.arange(n_sub), I[g, :n_sub], P_o, tol)


def test_mfma_precisions_reject_long_windows(dev):
    import torch
    import paper_2311_03393_amd as skmp
    R = torch.zeros((1, 4000), dtype=torch.float64, device=dev)
    for prec in ("bf16x3", "fp16x3"):
        with pytest.raises(skmp.SketchMPError):
            skmp.mp_selfjoin(R, [0, 4000], 1, 1100, 275, prec=prec)
