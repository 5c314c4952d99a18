"""GPU parity of the streaming path (Section III-B's streaming extension and
the point update of Section III-C) through the C-ABI against the CPU oracle.

* ``mp_selfjoin_append``: a profile grown by appends of ragged sizes (one
  sample, a few, several bands' worth) must equal, after every append, the
  oracle's batch profile of the series seen so far (the definition of the
  streaming profile), element by element, in FP64 and FP32; rows with no
  admissible partner before the append gain one; flat blocks arrive among the
  new samples; batched series in a layout with gaps (one joined afresh, one
  unchanged) leave every column they do not own untouched; a group mask
  restricts the update.
* ``sketch_append``: new samples sketched with the build's frozen statistics
  equal the oracle's projection, for every sketch kind, FP64 and FP32 input,
  several series with gaps in R and a series with no new samples.
* ``sketch_point_update``: equals the oracle's point updates (repeated
  columns, a constant dimension) and reports the changed groups.
* the whole stream (build, join, append samples, sketch, join, discords)
  against the oracle's discords of the final series.
"""
import math
import sys

import numpy as np
import pytest

import datagen
from oracle import sketchmp_oracle as O
from tests.helpers import check_neighbours, discords_equivalent, fp64_tol, mixed_tol, profile_close

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


def _sketched(seed, k, n, flat=()):
    """k x n sketched series (Gaussian sketch of 5 random-walk dimensions) with exact flat blocks."""
    T = datagen.tiny_series(seed, 5, n)
    R, _, _, _ = O.build(T, "gauss", k, seed)
    for a, b in flat:
        R[:, a:b] = 0.5
    return np.ascontiguousarray(R)


def _check_profile(c_oracle, R_np, m, excl, P, I, tol, what):
    k, n = R_np.shape
    n_sub = n - m + 1
    for g in range(k):
        P_o, _ = c_oracle.profile(R_np[g], m, excl)
        ok, err = profile_close(P[g, :n_sub], P_o, m, tol)
        assert ok.all(), f"{what} group {g}: {np.count_nonzero(~ok)} rows out of tolerance, max err {err}"
        check_neighbours(c_oracle, R_np[g], m, excl, np.arange(n_sub), I[g, :n_sub], P_o, tol)


APPEND_CASES = [  # (prec, n, m, excl, n0, appends, flat blocks)
    ("fp64", 3000, 32, 8, 1000, [1, 7, 64, 500, 1428], ()),
    ("fp32", 3000, 32, 8, 1000, [1, 7, 64, 500, 1428], ()),
    ("fp64", 9000, 64, 16, 2500, [3000, 10, 1990, 1500], ((7000, 7200),)),   # a wide append (>= 2048 windows)
    ("fp32", 9000, 64, 16, 2500, [3000, 10, 1990, 1500], ((3000, 3150),)),
    ("fp64", 2200, 16, 600, 500, [700, 1000], ()),       # old rows had no admissible partner
    ("fp64", 5000, 300, 75, 4000, [2, 998], ((1000, 1400),)),  # long windows, flat block among old samples
    ("fp32", 1500, 8, 2, 0, [20, 480, 1000], ()),        # from nothing: the first call joins afresh
]


@pytest.mark.parametrize("case", APPEND_CASES, ids=lambda c: f"{c[0]}-n{c[1]}-m{c[2]}-x{c[3]}")
def test_append_matches_oracle_after_every_call(dev, c_oracle, case):
    import torch
    import paper_2311_03393_amd as skmp
    prec, n, m, excl, n0, appends, flat = case
    assert n0 + sum(appends) == n
    k = 3
    _say("append", case)
    R_np = _sketched(7 + n, k, n, flat)
    R = torch.from_numpy(R_np).to(dev)
    P = torch.full((k, n), float("nan"), dtype=torch.float64, device=dev)
    I = torch.full((k, n), -2, dtype=torch.int64, device=dev)
    tol = fp64_tol(m) if prec == "fp64" else mixed_tol(m)
    cur = n0
    if n0 >= m:
        skmp.mp_selfjoin(R[:, :n0], [0, n0], k, m, excl, prec=prec, P=P, I=I)
    for a in appends:
        skmp.mp_selfjoin_append(R, P, I, [0], [cur], [cur + a], k, m, excl, prec=prec)
        cur += a
        torch.cuda.synchronize()
        Ph, Ih = P.cpu().numpy(), I.cpu().numpy()
        _check_profile(c_oracle, R_np[:, :cur], m, excl, Ph[:, :cur], Ih[:, :cur], tol, f"after {cur} samples")
        assert np.all(np.isnan(Ph[:, cur - m + 1:])) and np.all(Ih[:, cur - m + 1:] == -2), "columns past the windows"


def test_append_batched_series_with_gaps(dev, c_oracle):
    """Three series in a layout with room to grow: one appended to, one joined
    afresh (n_old < m), one unchanged (bit for bit); the gaps keep their
    sentinel values."""
    import torch
    import paper_2311_03393_amd as skmp
    k, m, excl = 2, 48, 12
    starts, caps = [0, 5000, 9000], [4000, 3000, 2500]
    n_old, n_new = [1200, 20, 2000], [2500, 1500, 2000]
    ld = 12000
    R_np = np.zeros((k, ld))
    for s in range(3):
        R_np[:, starts[s]:starts[s] + caps[s]] = _sketched(40 + s, k, caps[s])
    R = torch.from_numpy(R_np).to(dev)
    P = torch.full((k, ld), 7.0, dtype=torch.float64, device=dev)
    I = torch.full((k, ld), -7, dtype=torch.int64, device=dev)
    for s in (0, 2):
        a = starts[s]
        skmp.mp_selfjoin(R[:, a:a + n_old[s]], [0, n_old[s]], k, m, excl, P=P[:, a:a + n_old[s]],
                         I=I[:, a:a + n_old[s]])
    torch.cuda.synchronize()
    before = (P.cpu().numpy().copy(), I.cpu().numpy().copy())
    skmp.mp_selfjoin_append(R, P, I, starts, n_old, n_new, k, m, excl)
    torch.cuda.synchronize()
    Ph, Ih = P.cpu().numpy(), I.cpu().numpy()
    for s in (0, 1):
        a, nn = starts[s], n_new[s]
        _check_profile(c_oracle, R_np[:, a:a + nn], m, excl, Ph[:, a:a + nn], Ih[:, a:a + nn], fp64_tol(m),
                       f"series {s}")
    a = starts[2]
    assert np.array_equal(Ph[:, a:a + 2000], before[0][:, a:a + 2000]), "unchanged series was rewritten"
    assert np.array_equal(Ih[:, a:a + 2000], before[1][:, a:a + 2000])
    owned = np.zeros(ld, bool)
    for s in range(3):
        owned[starts[s]:starts[s] + n_new[s] - m + 1] = True
    assert np.all(Ph[:, ~owned] == 7.0) and np.all(Ih[:, ~owned] == -7), "a column outside the windows changed"


def test_append_group_mask(dev, c_oracle):
    import torch
    import paper_2311_03393_amd as skmp
    k, n, n0, m, excl = 4, 2600, 1800, 32, 8
    R_np = _sketched(51, k, n)
    R = torch.from_numpy(R_np).to(dev)
    P = torch.full((k, n), float("nan"), dtype=torch.float64, device=dev)
    I = torch.full((k, n), -2, dtype=torch.int64, device=dev)
    skmp.mp_selfjoin(R[:, :n0], [0, n0], k, m, excl, P=P, I=I)
    torch.cuda.synchronize()
    P0, I0 = P.cpu().numpy().copy(), I.cpu().numpy().copy()
    skmp.mp_selfjoin_append(R, P, I, [0], [n0], [n], k, m, excl, group_mask=0b1010)
    torch.cuda.synchronize()
    Ph, Ih = P.cpu().numpy(), I.cpu().numpy()
    for g in (0, 2):
        assert np.array_equal(Ph[g], P0[g], equal_nan=True) and np.array_equal(Ih[g], I0[g])
    _check_profile(c_oracle, R_np[[1, 3]], m, excl, Ph[[1, 3]], Ih[[1, 3]], fp64_tol(m), "masked")


def test_append_equals_batch_join_fp64(dev):
    """FP64: after appends, every row whose neighbour agrees with a batch join
    of the whole series carries the same distance bit for bit (both polish
    the same pair), and neighbours differ only where the oracle-level
    distances tie."""
    import torch
    import paper_2311_03393_amd as skmp
    k, n, m, excl = 3, 6000, 64, 16
    R_np = _sketched(61, k, n)
    R = torch.from_numpy(R_np).to(dev)
    P = torch.full((k, n), float("nan"), dtype=torch.float64, device=dev)
    I = torch.full((k, n), -2, dtype=torch.int64, device=dev)
    skmp.mp_selfjoin(R[:, :2000], [0, 2000], k, m, excl, P=P, I=I)
    cur = 2000
    for a in (1, 999, 3000):
        skmp.mp_selfjoin_append(R, P, I, [0], [cur], [cur + a], k, m, excl)
        cur += a
    Pb, Ib = skmp.mp_selfjoin(R, [0, n], k, m, excl)
    torch.cuda.synchronize()
    n_sub = n - m + 1
    Ps, Is = P.cpu().numpy()[:, :n_sub], I.cpu().numpy()[:, :n_sub]
    Pb, Ib = Pb.cpu().numpy()[:, :n_sub], Ib.cpu().numpy()[:, :n_sub]
    same = Is == Ib
    assert same.mean() > 0.999
    assert np.array_equal(Ps[same], Pb[same])
    assert np.max(np.abs(Ps[~same] - Pb[~same]), initial=0.0) < fp64_tol(m)


# ------------------------------------------------------------------ sketch
@pytest.mark.parametrize("kind,k,dtype", [("count", 4, "f64"), ("gauss", 5, "f64"), ("sum", 1, "f32"),
                                          ("count", 8, "f32")])
def test_sketch_append_matches_oracle(dev, kind, k, dtype):
    """Two series in a capacity layout: series 0 gets 700 new samples, series 1
    none at first and then 1300; columns outside the new ones keep their values."""
    import torch
    import paper_2311_03393_amd as skmp
    d, n0s, adds, caps, starts = 9, [2000, 1500], [700, 1300], [3000, 3000], [0, 3500]
    T = [datagen.tiny_series(70 + s, d, n0s[s] + adds[s]) for s in range(2)]
    T[1][4] = -3.0                                    # a constant dimension
    tdt = torch.float64 if dtype == "f64" else torch.float32
    if dtype == "f32":
        T = [t.astype(np.float32).astype(np.float64) for t in T]
    # build both prefixes in one call (sketch_build's layout: back to back)
    pre = np.concatenate([T[0][:, :n0s[0]], T[1][:, :n0s[1]]], axis=1)
    Tp = torch.from_numpy(np.ascontiguousarray(pre)).to(dev, tdt)
    Rb, stats = skmp.sketch_build(Tp, [0, n0s[0], n0s[0] + n0s[1]], k, kind, 33)
    ld = 7000
    R = torch.full((k, ld), 9.0, dtype=torch.float64, device=dev)
    R[:, starts[0]:starts[0] + n0s[0]] = Rb[:, :n0s[0]]
    R[:, starts[1]:starts[1] + n0s[1]] = Rb[:, n0s[0]:]
    st = stats.cpu().numpy()
    S = O.sketch_coeffs(kind, k, np.arange(d), 33)
    expect = np.full((k, ld), 9.0)
    expect[:, :n0s[0]] = Rb[:, :n0s[0]].cpu().numpy()
    expect[:, starts[1]:starts[1] + n0s[1]] = Rb[:, n0s[0]:].cpu().numpy()
    cur = list(n0s)
    for step_adds in ([adds[0], 0], [0, adds[1]]):
        new = np.concatenate([T[s][:, cur[s]:cur[s] + step_adds[s]] for s in range(2)], axis=1)
        offs = [0, step_adds[0], step_adds[0] + step_adds[1]]
        dst = [starts[s] + cur[s] for s in range(2)]
        Tn = torch.from_numpy(np.ascontiguousarray(new)).to(dev, tdt)
        skmp.sketch_append(Tn, offs, dst, R, stats, k, kind, 33)
        for s in range(2):
            if step_adds[s]:
                blk = T[s][:, cur[s]:cur[s] + step_adds[s]]
                expect[:, dst[s]:dst[s] + step_adds[s]] = O.sketch_append(blk, S, st[s, :, 0], st[s, :, 1])
                cur[s] += step_adds[s]
    torch.cuda.synchronize()
    got = R.cpu().numpy()
    scale = max(1.0, float(np.max(np.abs(expect))))
    assert np.max(np.abs(got - expect)) < 1e-12 * scale * d


@pytest.mark.parametrize("kind,k", [("count", 4), ("gauss", 3), ("sum", 1)])
def test_point_update_matches_oracle(dev, kind, k):
    import torch
    import paper_2311_03393_amd as skmp
    d, n = 7, 1200
    T = datagen.tiny_series(80, d, n)
    T[5] = 1.5                                       # a constant dimension
    Tt = torch.from_numpy(T).to(dev)
    R, stats = skmp.sketch_build(Tt, [0, n], k, kind, 44)
    torch.cuda.synchronize()
    R0 = R.cpu().numpy().copy()
    st = stats.cpu().numpy()[0]
    S = O.sketch_coeffs(kind, k, np.arange(d), 44)
    rng = np.random.default_rng(5)
    dims = rng.integers(0, d, 300)
    cols = rng.integers(0, n, 300)
    cols[10:20] = 77                                 # several updates to one column
    dims[10:20] = np.arange(10) % d
    deltas = rng.standard_normal(300)
    mask = skmp.sketch_point_update(R, stats, k, kind, 44, dims, cols, deltas)
    torch.cuda.synchronize()
    want = O.point_update(R0, S, st[:, 1], list(zip(dims.tolist(), cols.tolist(), deltas.tolist())))
    got = R.cpu().numpy()
    assert np.max(np.abs(got - want)) < 1e-12 * max(1.0, float(np.max(np.abs(want))))
    groups = {g for j in set(dims.tolist()) for g in range(k) if S[g, j] != 0.0}
    assert mask == sum(1 << g for g in groups)


def test_stream_end_to_end_discords(dev, c_oracle):
    """Build on the first samples, then append chunks (sketch + join) and rank
    discords: the sketch, every group's profile and the top-5 discords of the
    final series agree with the oracle's."""
    import torch
    import paper_2311_03393_amd as skmp
    d, k, m, excl, n0, n = 12, 4, 64, 16, 3000, 5000
    T = datagen.tiny_series(90, d, n)
    T[3, 4200:4264] += 4.0 * np.sin(np.linspace(0, 9, 64))     # an anomaly among the new samples
    Tt = torch.from_numpy(T).to(dev)
    R = torch.empty((k, n), dtype=torch.float64, device=dev)
    _, stats = skmp.sketch_build(Tt[:, :n0].contiguous(), [0, n0], k, "count", 12, R=R[:, :n0])
    P = torch.full((k, n), float("nan"), dtype=torch.float64, device=dev)
    I = torch.full((k, n), -2, dtype=torch.int64, device=dev)
    skmp.mp_selfjoin(R[:, :n0], [0, n0], k, m, excl, prec="fp32", P=P, I=I)
    cur = n0
    for a in (1, 255, 744, 1000):
        skmp.sketch_append(Tt[:, cur:cur + a].contiguous(), [0, a], [cur], R, stats, k, "count", 12)
        skmp.mp_selfjoin_append(R, P, I, [0], [cur], [cur + a], k, m, excl, prec="fp32")
        cur += a
    idx, grp, score, nf = skmp.top_discords(P, [0, n], k, m, 5)
    torch.cuda.synchronize()
    R0, S, mu, sd = O.build(T[:, :n0], "count", k, 12)
    R_o = np.concatenate([R0, O.sketch_append(T[:, n0:], S, mu, sd)], axis=1)
    R_g = R.cpu().numpy()
    assert np.max(np.abs(R_g - R_o)) < 1e-11 * max(1.0, float(np.max(np.abs(R_o))))
    n_sub = n - m + 1
    P_o = np.stack([c_oracle.profile(R_g[g], m, excl)[0] for g in range(k)])
    Ph = P.cpu().numpy()[:, :n_sub]
    for g in range(k):
        ok, err = profile_close(Ph[g], P_o[g], m, mixed_tol(m))
        assert ok.all(), (g, err)
    gpu_list = [(int(idx[0, q]), int(grp[0, q]), float(score[0, q])) for q in range(int(nf[0]))]
    ora_list = O.top_discords(P_o, m, 5)
    A_o = np.max(np.where(np.isfinite(P_o), P_o, -np.inf), axis=0)
    assert len(gpu_list) == len(ora_list)
    discords_equivalent(gpu_list, ora_list, A_o, m, mixed_tol(m))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_short_appends_batched_direct_path(dev, c_oracle, prec):
    """Short appends (a few new subsequences per series, computed without
    band walks): three series in one call, one of them starting from fewer
    than m samples, flat blocks arriving among the new samples; checked
    against the oracle after every call."""
    import torch
    import paper_2311_03393_amd as skmp
    k, m, excl = 2, 24, 6
    starts, caps = [0, 3000, 6000], [2600, 2600, 2600]
    ld = 9000
    R_np = np.zeros((k, ld))
    for s in range(3):
        R_np[:, starts[s]:starts[s] + caps[s]] = _sketched(90 + s, k, caps[s])
    R_np[:, starts[1] + 2010:starts[1] + 2040] = -0.25       # flat block arriving in series 1
    R = torch.from_numpy(R_np).to(dev)
    P = torch.full((k, ld), float("nan"), dtype=torch.float64, device=dev)
    I = torch.full((k, ld), -2, dtype=torch.int64, device=dev)
    cur = [2000, 2000, 10]
    for s in (0, 1):
        a = starts[s]
        skmp.mp_selfjoin(R[:, a:a + cur[s]], [0, cur[s]], k, m, excl, prec=prec, P=P[:, a:a + cur[s]],
                         I=I[:, a:a + cur[s]])
    tol = fp64_tol(m) if prec == "fp64" else mixed_tol(m)
    # appends of at most 8 new subsequences per series use the direct kernel; the last mixes in a longer one
    for step in ([1, 7, 20], [8, 0, 3], [5, 8, 1], [0, 1, 0], [2, 30, 40]):
        new = [cur[s] + step[s] for s in range(3)]
        _say("short append", prec, cur, new)
        skmp.mp_selfjoin_append(R, P, I, starts, cur, new, k, m, excl, prec=prec)
        torch.cuda.synchronize()
        cur = new
        Ph, Ih = P.cpu().numpy(), I.cpu().numpy()
        for s in range(3):
            if cur[s] < m:
                continue
            a = starts[s]
            _check_profile(c_oracle, R_np[:, a:a + cur[s]], m, excl, Ph[:, a:a + cur[s]], Ih[:, a:a + cur[s]], tol,
                           f"series {s} at {cur[s]} samples")


def test_sketch_append_nonfinite_check(dev):
    """With the finiteness check, NaN or Inf among the new samples is rejected
    (nothing is written); finite samples pass and are sketched."""
    import torch
    import paper_2311_03393_amd as skmp
    d, n0, a, k = 6, 800, 200, 3
    T = datagen.tiny_series(95, d, n0 + a)
    Tt = torch.from_numpy(T).to(dev)
    R = torch.full((k, n0 + a), 5.0, dtype=torch.float64, device=dev)
    _, stats = skmp.sketch_build(Tt[:, :n0].contiguous(), [0, n0], k, "count", 8, R=R[:, :n0])
    bad = Tt[:, n0:].clone()
    bad[2, 17] = float("nan")
    with pytest.raises(skmp.SketchMPError) as e:
        skmp.sketch_append(bad, [0, a], [n0], R, stats, k, "count", 8, check_finite=True)
    assert e.value.code == -4
    torch.cuda.synchronize()
    assert torch.all(R[:, n0:] == 5.0)
    skmp.sketch_append(Tt[:, n0:].contiguous(), [0, a], [n0], R, stats, k, "count", 8, check_finite=True)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()[0]
    S = O.sketch_coeffs("count", k, np.arange(d), 8)
    want = O.sketch_append(T[:, n0:], S, st[:, 0], st[:, 1])
    assert np.max(np.abs(R[:, n0:].cpu().numpy() - want)) < 1e-12 * max(1.0, float(np.max(np.abs(want))))


def test_point_update_several_series(dev):
    """Point updates in a batch of two series use each series' own statistics."""
    import torch
    import paper_2311_03393_amd as skmp
    d, k, n = 5, 4, 600
    T = np.concatenate([datagen.tiny_series(96, d, n), 3.0 * datagen.tiny_series(97, d, n)], axis=1)
    Tt = torch.from_numpy(np.ascontiguousarray(T)).to(dev)
    R, stats = skmp.sketch_build(Tt, [0, n, 2 * n], k, "gauss", 21)
    torch.cuda.synchronize()
    R0 = R.cpu().numpy().copy()
    st = stats.cpu().numpy()
    S = O.sketch_coeffs("gauss", k, np.arange(d), 21)
    rng = np.random.default_rng(9)
    ser = rng.integers(0, 2, 50)
    dims = rng.integers(0, d, 50)
    cols = rng.integers(0, n, 50) + ser * n
    deltas = rng.standard_normal(50)
    skmp.sketch_point_update(R, stats, k, "gauss", 21, dims, cols, deltas, series=ser)
    torch.cuda.synchronize()
    want = R0.copy()
    for s in range(2):
        sel = ser == s
        upd = list(zip(dims[sel].tolist(), cols[sel].tolist(), deltas[sel].tolist()))
        want = O.point_update(want, S, st[s, :, 1], upd)
    got = R.cpu().numpy()
    assert np.max(np.abs(got - want)) < 1e-12 * max(1.0, float(np.max(np.abs(want))))
