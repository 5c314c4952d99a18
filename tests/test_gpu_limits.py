"""GPU parity at the documented limits of the C-ABI: the longest subsequences
(m = 2048 for the FP64 and FP32 paths, 1024 for the MFMA paths), the largest
group count of a join (k = 64, every precision), and appends at m = 2048 (the direct short-append kernel
stages its longest windows there).  Rows are sampled where the oracle's brute
force would take minutes; the reported neighbour must attain the oracle's
nearest-neighbour distance and the reported distance must be its exact one.
"""
import sys

import numpy as np
import pytest

import datagen
from oracle import sketchmp_oracle as O
from tests.helpers import check_neighbours, fp64_tol, mixed_tol, profile_close

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


def _check_rows(c_oracle, R_np, m, excl, P, I, rows, tol, what):
    for g in range(R_np.shape[0]):
        P_o, _ = c_oracle.profile(R_np[g], m, excl, rows=rows)
        ok, err = profile_close(P[g, rows], P_o, m, tol)
        assert ok.all(), f"{what} group {g}: {np.count_nonzero(~ok)} rows out of tolerance, max err {err}"
        check_neighbours(c_oracle, R_np[g], m, excl, rows, I[g, rows], P_o, tol)


@pytest.mark.parametrize("prec,m", [("fp64", 2048), ("fp32", 2048), ("bf16x3", 1024), ("fp16x3", 1024)])
def test_longest_subsequences(dev, c_oracle, prec, m):
    import torch
    import paper_2311_03393_amd as skmp
    n, excl, k = 6500, m // 4, 2
    _say("longest m", prec, m)
    T = datagen.tiny_series(300 + m, 4, n)
    R_np, _, _, _ = O.build(T, "gauss", k, 300 + m)
    R = torch.from_numpy(np.ascontiguousarray(R_np)).to(dev)
    P, I = skmp.mp_selfjoin(R, [0, n], k, m, excl, prec=prec)
    torch.cuda.synchronize()
    P, I = P.cpu().numpy(), I.cpu().numpy()
    n_sub = n - m + 1
    rows = np.unique(np.concatenate([np.arange(0, 40), np.arange(n_sub - 40, n_sub),
                                     np.random.default_rng(m).choice(n_sub, 120, replace=False)]))
    tol = fp64_tol(m) if prec == "fp64" else mixed_tol(m)
    _check_rows(c_oracle, R_np, m, excl, P, I, rows, tol, f"{prec} m={m}")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x3"])
def test_most_groups(dev, c_oracle, prec):
    """k = 64 sketch groups (a count sketch of 200 dimensions), every group's
    full profile against the oracle, in every precision (the 16-bit paths in
    their default blocked MFMA form)."""
    import torch
    import paper_2311_03393_amd as skmp
    n, m, excl, k = 1200, 16, 4, 64
    _say("most groups", prec, k)
    T = datagen.tiny_series(310, 200, n)
    Tt = torch.from_numpy(T).to(dev)
    R, _ = skmp.sketch_build(Tt, [0, n], k, "count", 31)
    P, I = skmp.mp_selfjoin(R, [0, n], k, m, excl, prec=prec)
    top = skmp.top_discords(P, [0, n], k, m, 5)
    torch.cuda.synchronize()
    R_np = R.cpu().numpy()
    R_o, _, _, _ = O.build(T, "count", k, 31)
    assert np.max(np.abs(R_np - R_o)) < 1e-12 * max(1.0, float(np.max(np.abs(R_o))))
    P, I = P.cpu().numpy(), I.cpu().numpy()
    n_sub = n - m + 1
    tol = fp64_tol(m) if prec == "fp64" else mixed_tol(m)
    _check_rows(c_oracle, R_np, m, excl, P, I, np.arange(n_sub), tol, f"{prec} k=64")
    assert int(top[3][0]) == 5 and int(top[1][0].max()) < k


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_appends_at_longest_subsequences(dev, c_oracle, prec):
    """Appends at m = 2048: one new subsequence (the direct kernel with its
    longest LDS staging), then three (band walks)."""
    import torch
    import paper_2311_03393_amd as skmp
    m, excl, k, n0 = 2048, 512, 2, 5000
    n = n0 + 1 + 3
    T = datagen.tiny_series(320, 4, n)
    R_np, _, _, _ = O.build(T, "gauss", k, 320)
    R = torch.from_numpy(np.ascontiguousarray(R_np)).to(dev)
    P = torch.full((k, n), float("nan"), dtype=torch.float64, device=dev)
    I = torch.full((k, n), -2, dtype=torch.int64, device=dev)
    skmp.mp_selfjoin(R[:, :n0], [0, n0], k, m, excl, prec=prec, P=P, I=I)
    cur = n0
    tol = fp64_tol(m) if prec == "fp64" else mixed_tol(m)
    for a in (1, 3):
        skmp.mp_selfjoin_append(R, P, I, [0], [cur], [cur + a], k, m, excl, prec=prec)
        cur += a
        torch.cuda.synchronize()
        n_sub = cur - m + 1
        rows = np.unique(np.concatenate([np.arange(0, 30), np.arange(n_sub - 30, n_sub),
                                         np.random.default_rng(a).choice(n_sub, 60, replace=False)]))
        _check_rows(c_oracle, R_np[:, :cur], m, excl, P.cpu().numpy()[:, :cur], I.cpu().numpy()[:, :cur], rows,
                    tol, f"{prec} append to {cur}")
