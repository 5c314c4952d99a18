"""HIP graph capture of the whole hot path (sketch, self-join, top discords),
and the autotuned launch configuration.

One eager call per argument set comes first (it creates the library's pinned
copies of the host tables); the same sequence is then captured into a graph
and replayed several times, with eager work and an in-place change of the
input between replays.  Every replay must reproduce the eager results bit for
bit (the kernels are deterministic: maxima of packed keys, FP64 polish).
The eager results themselves are held to the oracle by the parity tests.
"""
import os
import sys

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_graph_replays_match_eager(prec):
    import torch
    import paper_2311_03393_amd as skmp
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    m, excl, k, top_k = 32, 8, 4, 5
    lens = [900, 2600, 1500]
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    N = int(offsets[-1])
    _say("graph", prec, lens, m, k)
    T_a = np.concatenate([datagen.tiny_series(300 + q, 6, L) for q, L in enumerate(lens)], axis=1)
    T_b = np.concatenate([datagen.tiny_series(400 + q, 6, L) for q, L in enumerate(lens)], axis=1)
    d = T_a.shape[0]

    T = torch.from_numpy(np.ascontiguousarray(T_a)).to(dev)
    R = torch.empty((k, N), dtype=torch.float64, device=dev)
    stats = torch.empty((len(lens), d, 2), dtype=torch.float64, device=dev)
    P = torch.empty((k, N), dtype=torch.float64, device=dev)
    I = torch.empty((k, N), dtype=torch.int64, device=dev)
    ws = torch.empty(skmp.mp_selfjoin_workspace(offsets, k, m, prec), dtype=torch.uint8, device=dev)
    out = (torch.empty((len(lens), top_k), dtype=torch.int64, device=dev),
           torch.empty((len(lens), top_k), dtype=torch.int32, device=dev),
           torch.empty((len(lens), top_k), dtype=torch.float64, device=dev),
           torch.empty((len(lens),), dtype=torch.int32, device=dev))

    def step():
        skmp.sketch_build(T, offsets, k, "gauss", 11, R=R, stats=stats)
        skmp.mp_selfjoin(R, offsets, k, m, excl, prec=prec, P=P, I=I, workspace=ws)
        skmp.top_discords(P, offsets, k, m, top_k, out=out)

    # P and I are defined on the n - m + 1 window columns of every series only
    win = torch.from_numpy(np.concatenate([np.arange(offsets[s], offsets[s + 1] - m + 1)
                                           for s in range(len(lens))]))

    def snapshot():
        torch.cuda.synchronize()
        return [x.cpu().clone() for x in (R, P[:, win.to(dev)], I[:, win.to(dev)]) + out]

    def same(a, b):
        for x, y in zip(a, b):
            if x.dtype.is_floating_point:
                assert torch.equal(torch.nan_to_num(x, nan=-7.0), torch.nan_to_num(y, nan=-7.0))
            else:
                assert torch.equal(x, y)

    # eager references for both inputs
    step()
    ref_a = snapshot()
    T.copy_(torch.from_numpy(T_b).to(dev))
    step()
    ref_b = snapshot()
    T.copy_(torch.from_numpy(T_a).to(dev))
    torch.cuda.synchronize()

    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()  # eager call on the capture stream before capturing
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()

    for rep, (src, ref) in enumerate([(T_a, ref_a), (T_a, ref_a), (T_b, ref_b), (T_a, ref_a)]):
        # eager work between replays: overwrite every output, then restore the input
        P.fill_(123.0)
        I.fill_(-9)
        R.fill_(0.5)
        for x in out:
            x.fill_(3)
        T.copy_(torch.from_numpy(src).to(dev))
        torch.cuda.synchronize()
        g.replay()
        got = snapshot()
        _say("replay", rep, "top", got[3][0].tolist())
        same(got, ref)
    del g


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_autotune_choice_is_used_and_exact(prec, c_oracle):
    """The autotuner times every candidate configuration, records the fastest
    for the shape class, and later calls (which use it) still match the oracle."""
    import torch
    import paper_2311_03393_amd as skmp
    from oracle import sketchmp_oracle as O
    from tests.helpers import check_neighbours, fp64_tol, mixed_tol, profile_close
    dev = torch.device("cuda:0")
    n, m, excl, k = 6000, 64, 16, 2
    _say("autotune", prec, n, m)
    T = datagen.tiny_series(41, 5, n)
    R_np, _, _, _ = O.build(T, "gauss", k, 41)
    R = torch.from_numpy(R_np).to(dev)
    skmp.tuning_clear()
    choice = skmp.mp_selfjoin_autotune(R, [0, n], k, m, excl, prec=prec, reps=1)
    assert choice["variant"] >= 0 and choice["ms"] > 0
    assert choice["strip"] in ((1024, 2048, 4096) if prec == "fp64" else (256,))
    rows = [line.split() for line in skmp.tuning_export().splitlines()]
    assert len(rows) == 1 and int(rows[0][0]) == {"fp64": 0, "fp32": 1}[prec]
    assert rows[0][3].startswith({"fp64": "c", "fp32": "f32_c"}[prec]) and int(rows[0][4]) == choice["strip"]
    skmp.tuning_clear()
    skmp.tuning_import(" ".join(rows[0]))   # the named variant round-trips
    assert skmp.tuning_export().split() == rows[0]
    P, I = skmp.mp_selfjoin(R, [0, n], k, m, excl, prec=prec)
    torch.cuda.synchronize()
    P, I = P.cpu().numpy(), I.cpu().numpy()
    n_sub = n - m + 1
    tol = fp64_tol(m) if prec == "fp64" else mixed_tol(m)
    for g in range(k):
        P_o, _ = c_oracle.profile(R_np[g], m, excl)
        ok, err = profile_close(P[g, :n_sub], P_o, m, tol)
        assert ok.all(), err
        check_neighbours(c_oracle, R_np[g], m, excl, np.arange(n_sub), I[g, :n_sub], P_o, tol)
    skmp.tuning_clear()


def test_tuning_file_round_trip_and_stamp(tmp_path):
    """The persistent tuning cache: a saved table loads back under the same
    device and runtime stamp, a file stamped for another device or runtime
    loads nothing, and with SKMP_TUNING_FILE set an autotuning result made in
    one process is the table of the next."""
    import subprocess
    import paper_2311_03393_amd as skmp
    path = tmp_path / "tune.txt"
    skmp.tuning_clear()
    rows = "0 7 16 c8_pd2_w2_clfalse 4096 3.250000\n2 6 15 blocked_w2 256 2.000000\n"
    skmp.tuning_import(rows)
    skmp.tuning_save(str(path))
    head, body = path.read_text().split("\n", 1)
    assert head.startswith("# sketchmp-tuning v1 arch=gfx950") and " hip=" in head
    assert sorted(body.splitlines()) == sorted(rows.splitlines())
    skmp.tuning_clear()
    assert skmp.tuning_load(str(path)) == 2
    assert sorted(skmp.tuning_export().splitlines()) == sorted(rows.splitlines())
    skmp.tuning_clear()
    (tmp_path / "other.txt").write_text(head.replace("hip=", "hip=9") + "\n" + body)
    assert skmp.tuning_load(str(tmp_path / "other.txt")) == 0 and skmp.tuning_export() == ""
    (tmp_path / "bad.txt").write_text(head + "\n0 7 16 no_such_variant 4096 1.0\n")
    with pytest.raises(skmp.SketchMPError):
        skmp.tuning_load(str(tmp_path / "bad.txt"))
    (tmp_path / "foreign.txt").write_text("0 7 16 c8_pd2_w2_clfalse 4096 1.0\n")
    with pytest.raises(skmp.SketchMPError):
        skmp.tuning_load(str(tmp_path / "foreign.txt"))
    assert skmp.tuning_export() == ""
    # two child processes sharing SKMP_TUNING_FILE: the first autotunes a
    # small FP32 join, the second sees its choice without tuning
    cache = tmp_path / "cache.txt"
    child = (
        "import sys, torch, numpy as np, paper_2311_03393_amd as skmp\n"
        "if sys.argv[1] == 'tune':\n"
        "    R = torch.from_numpy(np.random.default_rng(3).standard_normal((1, 3000))).cuda()\n"
        "    c = skmp.mp_selfjoin_autotune(R, [0, 3000], 1, 32, 8, prec='fp32', reps=1)\n"
        "    print('TUNED', c['variant'], flush=True)\n"
        "print('TABLE', skmp.tuning_export().replace(chr(10), ';'), flush=True)\n")
    env = dict(os.environ, SKMP_TUNING_FILE=str(cache))
    outs = []
    for mode in ("tune", "read"):
        _say("tuning-file child", mode)
        r = subprocess.run([sys.executable, "-c", child, mode], env=env, cwd=ROOT, capture_output=True, text=True,
                           timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append([ln for ln in r.stdout.splitlines() if ln.startswith("TABLE")][0])
    assert outs[0] == outs[1] and outs[0].startswith("TABLE 1 5 12 f32_")
    assert cache.read_text().startswith(head)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x3"])
def test_every_compiled_variant_matches_oracle(prec, c_oracle):
    """Each compiled tile-kernel variant (diagonals per lane, prefetch depth,
    occupancy, column scheme; for the 16-bit split precisions the
    Hankel-direct and the blocked-recurrence forms), forced through the tuning
    table, gives the oracle's profile: the key codes of every lane width
    decode to the right diagonal."""
    import math
    import torch
    import paper_2311_03393_amd as skmp
    from oracle import sketchmp_oracle as O
    from tests.helpers import check_neighbours, fp64_tol, mixed_tol, profile_close
    dev = torch.device("cuda:0")
    n, m, excl, k = 3100, 32, 8, 2
    T = datagen.tiny_series(43, 5, n)
    R_np, _, _, _ = O.build(T, "gauss", k, 43)
    R = torch.from_numpy(R_np).to(dev)
    n_sub = n - m + 1
    mlog, nlog = math.ceil(math.log2(m)), math.ceil(math.log2(n_sub))
    strip = 2048 if prec == "fp64" else 256
    P_o = [c_oracle.profile(R_np[g], m, excl)[0] for g in range(k)]
    tol = fp64_tol(m) if prec == "fp64" else mixed_tol(m)
    tested = 0
    try:
        for v in skmp.tile_variants(prec):
            skmp.tuning_clear()
            code = {'fp64': 0, 'fp32': 1, 'bf16x3': 2, 'fp16x3': 3}[prec]
            skmp.tuning_import(f"{code} {mlog} {nlog} {v} {strip} 1.0")
            _say("variant", prec, v)
            P, I = skmp.mp_selfjoin(R, [0, n], k, m, excl, prec=prec)
            torch.cuda.synchronize()
            P, I = P.cpu().numpy(), I.cpu().numpy()
            for g in range(k):
                ok, err = profile_close(P[g, :n_sub], P_o[g], m, tol)
                assert ok.all(), f"{prec} variant {v} group {g}: max err {err}"
                check_neighbours(c_oracle, R_np[g], m, excl, np.arange(n_sub), I[g, :n_sub], P_o[g], tol)
            tested += 1
    finally:
        skmp.tuning_clear()
    assert tested == len(skmp.tile_variants(prec)) >= 3


def test_upload_past_the_pinned_cache_cap():
    """A host table larger than the library's 64 MiB pinned cache (the series
    table of 2.2 million series, 70 MB) is copied from the caller's memory, in
    stream order, and the call waits for the copy; twice in a row, the second
    also past the cap, both right."""
    import torch
    import paper_2311_03393_amd as skmp
    n_series, L, m = 2_200_000, 3, 2
    offs = np.arange(n_series + 1, dtype=np.int64) * L
    rng = np.random.default_rng(5)
    P_np = rng.uniform(0.0, 3.0, size=(1, n_series * L))
    P = torch.from_numpy(P_np).cuda()
    _say("upload past cap", n_series)
    for rep in range(2):
        idx, grp, score, nf = skmp.top_discords(P, offs, 1, m, 1)
        torch.cuda.synchronize()
        w = P_np[0].reshape(n_series, L)[:, :L - m + 1]          # the two windows of every series
        expect = np.argmax(w, axis=1)                            # first maximum on ties
        assert np.array_equal(idx.cpu().numpy()[:, 0], expect), rep
        assert np.array_equal(score.cpu().numpy()[:, 0], w[np.arange(n_series), expect])
        assert (nf.cpu().numpy() == 1).all() and (grp.cpu().numpy()[:, 0] == 0).all()
        P_np = P_np[:, ::-1].copy()                               # a different table of the same size next
        P = torch.from_numpy(P_np).cuda()
        offs = offs.copy()
