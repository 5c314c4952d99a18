"""GPU parity of the discord dimension detection (Algorithm 3) through the
C-ABI against the oracle: per-dimension scores (the AB-join distance of the
test subsequence in each dimension against that dimension's train series, or
the self-join row with its exclusion zone), neighbours and the chosen
dimension; FP64 and FP32 input; constant dimensions and flat subsequences; and
the whole two-phase procedure (Algorithm 2 on the sketch, then Algorithm 3 on
the discord's group) on the small random-walk workload and the
water-treatment workload.
"""
import sys

import numpy as np
import pytest

import datagen
from oracle import sketchmp_oracle as O
from tests.helpers import fp64_tol, profile_close

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _stats(torch, skmp, T):
    _, st = skmp.sketch_build(T, [0, int(T.shape[1])], 1, "sum", 0)
    return st[0]


def _check(scores, nn, best, ref, m, tol, allow_tie=True):
    s_o, nn_o, best_o = ref
    ok, err = profile_close(scores, s_o, m, tol)
    assert ok.all(), (err, scores, s_o)
    fin = np.isfinite(s_o)
    assert np.all(nn[~fin] == -1)
    if not allow_tie:
        assert np.array_equal(nn, nn_o)
    top = np.max(s_o)
    assert s_o[best] >= top - 2 * tol   # the chosen dimension attains the largest score
    if best != best_o:
        assert abs(s_o[best] - s_o[best_o]) <= 2 * tol


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("m", [16, 64, 100])
def test_dim_detect_train_test(dtype, m):
    import torch
    import paper_2311_03393_amd as skmp
    dev = torch.device("cuda:0")
    d = 9
    Ttr = datagen.tiny_series(50 + m, d, 3000)
    Tte = datagen.tiny_series(60 + m, d, 2100)
    i_star, j0 = 777, 4
    loc = Tte[j0, i_star:i_star + m].std()
    Tte[j0, i_star:i_star + m] += 6 * loc * np.sin(np.linspace(0, 9 * np.pi, m) ** 1.3)
    Ttr[7] = 2.5                      # a constant dimension
    Tte[2, 1000:1400] = -1.0          # flat windows in the test series (not at i_star)
    Ttr[1, 200:600] = 0.25            # and in the train series
    if dtype == "f32":
        Ttr, Tte = Ttr.astype(np.float32), Tte.astype(np.float32)
    dims = [0, 1, 2, 4, 7, 8]
    _say("dim_detect", dtype, m)
    Ttr_d, Tte_d = torch.from_numpy(Ttr).to(dev), torch.from_numpy(Tte).to(dev)
    s, nn, best = skmp.dim_detect(Ttr_d, _stats(torch, skmp, Ttr_d), dims, i_star, m, T_test=Tte_d,
                                  stats_test=_stats(torch, skmp, Tte_d))
    torch.cuda.synchronize()
    ref = O.dimension_detection(Ttr.astype(np.float64), Tte.astype(np.float64), i_star, dims, m)
    _check(s.cpu().numpy(), nn.cpu().numpy(), int(best.item()), ref, m, fp64_tol(m))
    # the planted dimension wins unless the constant train dimension (every
    # window flat: distance sqrt(m) from a non-flat subsequence) scores higher
    if m > 16:
        assert dims[int(best.item())] == j0


@pytest.mark.parametrize("i_star", [0, 1500, 2936])
def test_dim_detect_self_join_setting(i_star):
    import torch
    import paper_2311_03393_amd as skmp
    dev = torch.device("cuda:0")
    d, m, excl = 6, 64, 16
    T = datagen.tiny_series(70, d, 3000)
    T[3, 2000:2300] = 1.0             # flat windows
    T[5] = 0.0                        # constant dimension
    Td = torch.from_numpy(T).to(dev)
    dims = list(range(d))
    s, nn, best = skmp.dim_detect(Td, _stats(torch, skmp, Td), dims, i_star, m, excl=excl)
    torch.cuda.synchronize()
    ref = O.dimension_detection(T, None, i_star, dims, m, excl=excl)
    _check(s.cpu().numpy(), nn.cpu().numpy(), int(best.item()), ref, m, fp64_tol(m))
    assert np.all(np.abs(nn.cpu().numpy() - i_star) >= excl)


def test_dim_detect_all_excluded_and_flat_query():
    import torch
    import paper_2311_03393_amd as skmp
    dev = torch.device("cuda:0")
    m = 32
    T = datagen.tiny_series(71, 3, 60)   # 29 windows: with excl 40 nothing is admissible
    T[1, 10:10 + m] = 3.0                 # the test subsequence of dimension 1 is flat
    Td = torch.from_numpy(T).to(dev)
    s, nn, best = skmp.dim_detect(Td, _stats(torch, skmp, Td), [0, 1, 2], 10, m, excl=40)
    torch.cuda.synchronize()
    assert np.all(np.isinf(s.cpu().numpy())) and np.all(nn.cpu().numpy() == -1) and int(best.item()) == 0
    s2, nn2, best2 = skmp.dim_detect(Td, _stats(torch, skmp, Td), [0, 1, 2], 10, m, excl=2)
    torch.cuda.synchronize()
    ref = O.dimension_detection(T, None, 10, [0, 1, 2], m, excl=2)
    _check(s2.cpu().numpy(), nn2.cpu().numpy(), int(best2.item()), ref, m, fp64_tol(m))


@pytest.mark.parametrize("workload,kind,k", [("random-walk-small", "count", 3), ("water-treatment", "gauss", 8)])
def test_two_phase_detection(workload, kind, k):
    """Algorithm 2 on the sketch finds (i*, g*); Algorithm 3 on g*'s dimensions
    (self-join setting) matches the oracle's scores at that i*."""
    import torch
    import paper_2311_03393_amd as skmp
    dev = torch.device("cuda:0")
    w = datagen.make(workload)
    T = torch.from_numpy(w.T).to(dev)
    R, stats = skmp.sketch_build(T, w.offsets, k, kind, w.sketch_seed, dim_ids=w.dim_ids)
    P, I = skmp.mp_selfjoin(R, w.offsets, k, w.m, w.excl)
    idx, grp, score, nf = skmp.top_discords(P, w.offsets, k, w.m, 1)
    torch.cuda.synchronize()
    i_star, g_star = int(idx[0, 0]), int(grp[0, 0])
    dims = skmp.group_dims(kind, k, w.sketch_seed, g_star, w.dim_ids)
    _say(workload, "i*", i_star, "g*", g_star, "dims", len(dims))
    s, nn, best = skmp.dim_detect(T, stats[0], dims, i_star, w.m, excl=w.excl)
    torch.cuda.synchronize()
    ref = O.dimension_detection(w.T, None, i_star, [int(j) for j in dims], w.m, excl=w.excl)
    _check(s.cpu().numpy(), nn.cpu().numpy(), int(best.item()), ref, w.m, fp64_tol(w.m))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_exact_multidimensional_baseline(prec, c_oracle):
    """Every dimension's own self-join profile in one batched launch (k = d,
    identity sketch) against the oracle's profile of each z-normalised dimension."""
    import torch
    import paper_2311_03393_amd as skmp
    from tests.helpers import check_neighbours, mixed_tol
    dev = torch.device("cuda:0")
    d, n, m, excl = 12, 1500, 32, 8
    T = datagen.tiny_series(77, d, n)
    T[4] = -0.5                       # constant dimension
    T[7, 300:600] = 2.0               # flat windows
    P, I = skmp.exact_profiles(torch.from_numpy(T).to(dev), m, excl, prec=prec,
                               refresh=256 if prec == "fp32" else 0)
    torch.cuda.synchronize()
    P, I = P.cpu().numpy(), I.cpu().numpy()
    Tb, _, _ = O.znorm_dims(T)
    tol = fp64_tol(m) if prec == "fp64" else mixed_tol(m)
    n_sub = n - m + 1
    for j in range(d):
        P_o, _ = c_oracle.profile(Tb[j], m, excl)
        ok, err = profile_close(P[j, :n_sub], P_o, m, tol)
        assert ok.all(), (j, err)
        check_neighbours(c_oracle, Tb[j], m, excl, np.arange(n_sub), I[j, :n_sub], P_o, tol)
