"""The allocation-free top_discords entry point against the workspace one,
through the C-ABI, on two calls in a row (the second smaller, so stale
contents of the shared scratch from the first call would show)."""
import ctypes

import numpy as np
import pytest

import paper_2311_03393_amd as skmp


def _profiles(rng, k, lengths, m):
    """k x N profile rows with the shapes discord search meets: finite values
    in [0, 2 sqrt(m)], +inf where a window has no admissible neighbour, the
    tail of every series (its last m - 1 samples) unused, and exact ties."""
    N = int(sum(lengths))
    P = rng.uniform(0.0, 2.0 * np.sqrt(m), size=(k, N))
    P[rng.random((k, N)) < 1e-3] = np.inf
    # exact ties across groups and windows: copies of the largest values
    top = np.argsort(P.max(axis=0))[-20:]
    P[:, top[:10]] = P[:, top[10:]].max()
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    return P, offs


def _call(L, fn, P, offs, k, m, top_k, halfwidth, with_ws):
    import torch
    n_series = offs.size - 1
    idx = torch.full((n_series, top_k), -7, dtype=torch.int64, device="cuda")
    grp = torch.full((n_series, top_k), -7, dtype=torch.int32, device="cuda")
    score = torch.full((n_series, top_k), -7.0, dtype=torch.float64, device="cuda")
    nf = torch.full((n_series,), -7, dtype=torch.int32, device="cuda")
    p64 = offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = [P.data_ptr(), P.stride(0), n_series, p64, k, m, top_k, halfwidth, idx.data_ptr(), grp.data_ptr(),
            score.data_ptr(), nf.data_ptr()]
    if with_ws:
        ws_n = L.top_discords_workspace(n_series, p64, k, m)
        ws = torch.empty(ws_n, dtype=torch.uint8, device="cuda")
        rc = fn(*args, ws.data_ptr(), ws.numel(), stream)
    else:
        rc = fn(*args, stream)
    assert rc == 0, L.skmp_last_error()
    torch.cuda.synchronize()
    return idx.cpu().numpy(), grp.cpu().numpy(), score.cpu().numpy(), nf.cpu().numpy()


@pytest.mark.gpu
def test_noalloc_matches_workspace_entry_point_on_two_calls():
    import torch
    L = skmp.lib()
    rng = np.random.default_rng(9001)
    cases = [
        # near the limits: 2^21 samples over 5 series (one shorter than m), k = 4
        dict(k=4, m=64, top_k=12, halfwidth=0, lengths=[700_000, 40, 500_000, 650_000, 2 ** 21 - 1_850_040]),
        # smaller second call: fewer series, fewer samples, other k / m / halfwidth
        dict(k=2, m=100, top_k=5, halfwidth=37, lengths=[30_000, 12_345, 7_655]),
    ]
    for c in cases:
        print(f"noalloc case k={c['k']} m={c['m']} lengths={c['lengths']}", flush=True)
        P_np, offs = _profiles(rng, c["k"], c["lengths"], c["m"])
        assert offs[-1] <= 2 ** 21
        P = torch.from_numpy(P_np).cuda()
        a = _call(L, L.top_discords_noalloc, P, offs, c["k"], c["m"], c["top_k"], c["halfwidth"], False)
        b = _call(L, L.top_discords, P, offs, c["k"], c["m"], c["top_k"], c["halfwidth"], True)
        for x, y in zip(a, b):
            assert np.array_equal(x, y, equal_nan=True) if x.dtype.kind == "f" else np.array_equal(x, y)
        assert np.all(a[3] >= 0)
        # a series shorter than m has no window: nothing found
        for s, n in enumerate(c["lengths"]):
            if n < c["m"]:
                assert a[3][s] == 0 and np.all(a[0][s] == -1)


@pytest.mark.gpu
def test_noalloc_binding_and_limits():
    import torch
    rng = np.random.default_rng(77)
    P_np, offs = _profiles(rng, 3, [5000, 6000], 32)
    P = torch.from_numpy(P_np).cuda()
    a = [t.cpu().numpy() for t in skmp.top_discords_noalloc(P, offs, 3, 32, 8)]
    b = [t.cpu().numpy() for t in skmp.top_discords(P, offs, 3, 32, 8)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y, equal_nan=True) if x.dtype.kind == "f" else np.array_equal(x, y)
    # beyond the limits: refused before anything is launched
    with pytest.raises(skmp.SketchMPError):
        skmp.top_discords_noalloc(P, np.arange(66, dtype=np.int64) * 10, 3, 32, 8)
