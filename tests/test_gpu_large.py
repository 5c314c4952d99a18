"""The large single series at full size: d = 256, n = 2^20, Gaussian k = 32,
m = 256, with the add/remove of 16 dimensions (Section III-C) and the
recomputation bench.py times.

Checked on sampled outputs: the sketch and the updated sketch element by
element against the oracle's build of the same input (R of a fresh build over
the kept and added dimensions), the changed-group mask, and 16 profile rows
of 4 groups (plus the first and last window) of the recomputed profile
against the oracle's brute-force rows, with their neighbours, for the FP64,
FP32 and FP16x3 (the workload's named precision) paths; the reported distances
are the exact distances of the reported neighbours for every window.
"""
import sys

import numpy as np
import pytest

import datagen
from oracle import sketchmp_oracle as O
from tests.helpers import check_neighbours, fp64_tol, mixed_tol, profile_close

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def large():
    import torch
    import paper_2311_03393_amd as skmp
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    w = datagen.make("large-series")
    _say("large series full size", w.T.shape)
    T = torch.from_numpy(w.T).to(dev)
    R, stats = skmp.sketch_build(T, w.offsets, w.k, w.kind, w.sketch_seed, dim_ids=w.dim_ids)
    torch.cuda.synchronize()
    R_built = R.cpu().numpy()
    rem = w.update["rem_ids"]
    add_ids = w.update["add_ids"]
    T_add = torch.from_numpy(w.update["T_add"]).to(dev)
    rem_idx = torch.from_numpy(rem).to(dev)
    _, changed = skmp.sketch_update_dims(R, w.kind, w.k, w.sketch_seed, T_add=T_add, add_ids=add_ids,
                                         T_rem=T[rem_idx].contiguous(), rem_ids=rem,
                                         rem_stats=stats[0].index_select(0, rem_idx))
    torch.cuda.synchronize()
    yield w, R, R_built, changed
    del T, R, T_add
    torch.cuda.empty_cache()


def test_c4_sketch_and_update(large):
    w, R, R_built, changed = large
    R_o, _, _, _ = O.build(w.T, w.kind, w.k, w.sketch_seed, w.dim_ids)
    assert np.max(np.abs(R_built - R_o)) <= 1e-12 * np.max(np.abs(R_o))
    keep = np.setdiff1d(w.dim_ids, w.update["rem_ids"])
    Tk = np.concatenate([w.T[keep], w.update["T_add"]])
    R_u, _, _, _ = O.build(Tk, w.kind, w.k, w.sketch_seed, np.concatenate([keep, w.update["add_ids"]]))
    Rg = R.cpu().numpy()
    assert np.max(np.abs(Rg - R_u)) <= 1e-11 * np.max(np.abs(R_u))
    assert changed == (1 << w.k) - 1   # every Gaussian row has non-zero coefficients on the changed dims


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp16x3"])
def test_c4_recomputed_profile_sampled(large, c_oracle, prec):
    import torch
    import paper_2311_03393_amd as skmp
    w, R, _, changed = large
    m, excl, k = w.m, w.excl, w.k
    _say("large series selfjoin", prec)
    P, I = skmp.mp_selfjoin(R, w.offsets, k, m, excl, prec=prec, refresh=256 if prec != "fp64" else 0,
                            group_mask=changed)
    torch.cuda.synchronize()
    n = w.T.shape[1]
    n_sub = n - m + 1
    Rh = R.cpu().numpy()
    Ph = P[:, :n_sub].cpu().numpy()
    Ih = I[:, :n_sub].cpu().numpy()
    del P, I
    tol = mixed_tol(m) if prec != "fp64" else fp64_tol(m)
    rng = np.random.default_rng(9)
    groups = rng.choice(k, 4, replace=False)
    rows = np.unique(np.concatenate([rng.choice(n_sub, 16, replace=False), [0, n_sub - 1]]))
    for g in groups:
        P_o, _ = c_oracle.profile(Rh[g], m, excl, rows=rows)
        ok, err = profile_close(Ph[g, rows], P_o, m, tol)
        assert ok.all(), (prec, int(g), err)
        check_neighbours(c_oracle, Rh[g], m, excl, rows, Ih[g, rows], P_o, tol)
    # every reported distance is the exact distance of the reported neighbour
    for g in range(k):
        assert (Ih[g] >= 0).all()
        dd = c_oracle.pair_dist(Rh[g], m, np.arange(n_sub), Ih[g])
        assert np.max(np.abs(dd - Ph[g])) < 1e-9, (prec, g)
        assert (np.abs(np.arange(n_sub) - Ih[g]) >= excl).all()
