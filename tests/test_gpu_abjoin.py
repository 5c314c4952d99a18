"""GPU parity of the AB-join (the join of Algorithm 2 between a test and a
train series, Section III-B) through the C-ABI against the CPU oracle.

Both directions (A -> B and B -> A) are compared element by element with the
oracle's brute force at sizes it finishes in seconds: rectangular shapes in
both orientations, several diagonal bands and strips, one-window series, flat
subsequences in both series, a group mask.  The reported neighbour must attain
the oracle's nearest-neighbour distance (any of several equally near ones is
accepted) and the reported distance must be the exact distance to it.  At the
full water-treatment size (first and second half of the series) rows are
sampled; the top-10 discords of the test half are compared with the oracle's
greedy picks on its own AB profile at a mid size.
"""
import sys

import numpy as np
import pytest

import datagen
from oracle import sketchmp_oracle as O
from tests.helpers import discords_equivalent, fp64_tol, mixed_tol, profile_close

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _series(seed, k, n, flat=None):
    R = datagen.tiny_series(seed, k, n)
    if flat is not None:
        a, b = flat
        R[:, a:b] = 0.75
    return np.ascontiguousarray(R)


def _check_direction(c_oracle, Ra, Rb, m, P, I, tol, rows=None):
    na_sub = Ra.shape[1] - m + 1
    nb_sub = Rb.shape[1] - m + 1
    rows = np.arange(na_sub) if rows is None else np.asarray(rows)
    for g in range(Ra.shape[0]):
        P_o, I_o = c_oracle.ab_profile(Ra[g], Rb[g], m, rows=rows)
        ok, err = profile_close(P[g, rows], P_o, m, tol)
        assert ok.all(), (g, err, rows[~ok][:5])
        ii = I[g, rows]
        assert np.all((ii >= 0) & (ii < nb_sub))
        dd = c_oracle.ab_pair_dist(Ra[g], Rb[g], m, rows, ii)
        ok2, err2 = profile_close(dd, P_o, m, tol)
        assert ok2.all(), ("neighbour does not attain the NN distance", g, err2)
        assert np.max(np.abs(dd - P[g, rows])) < 1e-9, "reported distance is not the neighbour's exact distance"


AB_CASES = [  # (na, nb, m, flat windows of A, flat windows of B)
    (300, 700, 16, None, (100, 140)),
    (1500, 400, 32, (200, 260), None),
    (2600, 2600, 100, None, None),
    (777, 4100, 64, None, (3000, 3100)),   # several 1024-diagonal bands along A's rows
    (4100, 900, 8, (10, 30), (500, 520)),  # several bands along B's rows
    (4, 9, 4, None, None),                 # one window in A
    (60, 5, 5, None, None),                # one window in B
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", AB_CASES)
def test_abjoin_both_directions(case, prec, c_oracle):
    import torch
    import paper_2311_03393_amd as skmp
    na, nb, m, fa, fb = case
    _say("abjoin", prec, case)
    k = 2
    Ra = _series(na + 3, k, na, fa)
    Rb = _series(nb + 5, k, nb, fb)
    dev = torch.device("cuda:0")
    PA, IA, PB, IB = skmp.mp_abjoin(torch.from_numpy(Ra).to(dev), torch.from_numpy(Rb).to(dev), k, m, prec=prec,
                                    refresh=256 if prec == "fp32" else 0, both=True)
    torch.cuda.synchronize()
    tol = fp64_tol(m) if prec == "fp64" else mixed_tol(m)
    na_sub, nb_sub = na - m + 1, nb - m + 1
    _check_direction(c_oracle, Ra, Rb, m, PA.cpu().numpy()[:, :na_sub], IA.cpu().numpy()[:, :na_sub], tol)
    _check_direction(c_oracle, Rb, Ra, m, PB.cpu().numpy()[:, :nb_sub], IB.cpu().numpy()[:, :nb_sub], tol)


def test_abjoin_group_mask_and_one_direction(c_oracle):
    import torch
    import paper_2311_03393_amd as skmp
    dev = torch.device("cuda:0")
    k, m = 4, 24
    Ra, Rb = _series(5, k, 900), _series(6, k, 1300)
    PA, IA = skmp.mp_abjoin(torch.from_numpy(Ra).to(dev), torch.from_numpy(Rb).to(dev), k, m, group_mask=0b1010)
    torch.cuda.synchronize()
    PA, IA = PA.cpu().numpy(), IA.cpu().numpy()
    assert np.all(np.isnan(PA[[0, 2]])) and np.all(IA[[0, 2]] == -2)   # unselected groups untouched
    n_sub = 900 - m + 1
    _check_direction(c_oracle, Ra[[1, 3]], Rb[[1, 3]], m, PA[[1, 3], :n_sub], IA[[1, 3], :n_sub], fp64_tol(m))


def test_abjoin_rejects_mfma_precisions():
    import torch
    import paper_2311_03393_amd as skmp
    dev = torch.device("cuda:0")
    R = torch.zeros((1, 100), dtype=torch.float64, device=dev)
    with pytest.raises(skmp.SketchMPError):
        skmp.mp_abjoin(R, R, 1, 16, prec="bf16x3")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_abjoin_water_treatment_halves_sampled(prec, c_oracle):
    """Test half vs train half of the water-treatment workload (d = 51, k = 8, m = 100)."""
    import torch
    import paper_2311_03393_amd as skmp
    w = datagen.make("water-treatment")
    dev = torch.device("cuda:0")
    T = torch.from_numpy(w.T).to(dev)
    half = w.T.shape[1] // 2
    # each half is its own series: sketch them separately (per-series normalisation)
    Ra, _ = skmp.sketch_build(T[:, half:].contiguous(), [0, w.T.shape[1] - half], w.k, w.kind, w.sketch_seed,
                              dim_ids=w.dim_ids)
    Rb, _ = skmp.sketch_build(T[:, :half].contiguous(), [0, half], w.k, w.kind, w.sketch_seed, dim_ids=w.dim_ids)
    _say("abjoin water-treatment halves", prec)
    PA, IA = skmp.mp_abjoin(Ra, Rb, w.k, w.m, prec=prec, refresh=256 if prec == "fp32" else 0)
    torch.cuda.synchronize()
    m = w.m
    na_sub = Ra.shape[1] - m + 1
    Ra_h, Rb_h = Ra.cpu().numpy(), Rb.cpu().numpy()
    PA_h, IA_h = PA.cpu().numpy()[:, :na_sub], IA.cpu().numpy()[:, :na_sub]
    rng = np.random.default_rng(21)
    rows = np.unique(np.concatenate([rng.choice(na_sub, 48, replace=False), [0, na_sub - 1]]))
    tol = fp64_tol(m) if prec == "fp64" else mixed_tol(m)
    _check_direction(c_oracle, Ra_h, Rb_h, m, PA_h, IA_h, tol, rows=rows)
    # every reported distance is the exact distance of the reported neighbour
    for g in range(w.k):
        dd = c_oracle.ab_pair_dist(Ra_h[g], Rb_h[g], m, np.arange(na_sub), IA_h[g])
        assert np.max(np.abs(dd - PA_h[g])) < 1e-9


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_abjoin_top_discords_of_test_series(prec, c_oracle):
    """Discords of a test series against a train series (Algorithm 2 with AB-join)."""
    import torch
    import paper_2311_03393_amd as skmp
    dev = torch.device("cuda:0")
    k, m = 3, 64
    w_tr = datagen.tiny_series(91, 6, 5000)
    w_te = datagen.tiny_series(92, 6, 4000)
    loc = w_te[2, 1500:1500 + m].std()
    w_te[2, 1500:1500 + m] += 10.0 * loc * np.sin(np.arange(m) / 3.0)   # an anomaly only in the test series
    Rb, _, _, _ = O.build(w_tr, "gauss", k, 7)
    Ra, _, _, _ = O.build(w_te, "gauss", k, 7)
    PA, IA = skmp.mp_abjoin(torch.from_numpy(np.ascontiguousarray(Ra)).to(dev),
                            torch.from_numpy(np.ascontiguousarray(Rb)).to(dev), k, m, prec=prec,
                            refresh=256 if prec == "fp32" else 0)
    n_sub = Ra.shape[1] - m + 1
    idx, grp, score, nf = skmp.top_discords(PA, [0, Ra.shape[1]], k, m, 10)
    torch.cuda.synchronize()
    P_o = np.stack([c_oracle.ab_profile(Ra[g], Rb[g], m)[0] for g in range(k)])
    tol = fp64_tol(m) if prec == "fp64" else mixed_tol(m)
    for g in range(k):
        ok, err = profile_close(PA.cpu().numpy()[g, :n_sub], P_o[g], m, tol)
        assert ok.all(), (g, err)
    ref = O.top_discords(P_o, m, 10)
    got = [(int(i), int(gg), float(s)) for i, gg, s in zip(idx[0].cpu(), grp[0].cpu(), score[0].cpu())][:int(nf[0])]
    assert len(got) == len(ref)
    discords_equivalent(got, ref, P_o.max(axis=0), m, tol)
    assert any(abs(i - 1500) < m for i, _, _ in got)   # the planted anomaly is among the picks
