"""The C-ABI library without a GPU: it loads, exports every declared symbol,
draws the same coefficients as the oracle, and rejects bad arguments before
touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2311_03393_amd as skmp
from oracle import sketchmp_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sketchmp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(skmp.LIB_PATH):
        from paper_2311_03393_amd import build
        build.build()
    return skmp.lib()


def test_library_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 11
    assert set(names) == set(skmp.EXPORTED)
    for nm in names:
        assert hasattr(L, nm), nm
    assert "gfx950" in skmp.version()


@pytest.mark.parametrize("kind,k", [("sum", 1), ("count", 5), ("count", 64), ("count", 100), ("count", 128),
                                    ("gauss", 3), ("gauss", 16)])
def test_coefficients_match_oracle_bit_for_bit(L, kind, k):
    ids = np.array([0, 1, 2, 7, 100, 12345, 2 ** 40 + 3, 999999937])
    S_lib = skmp.sketch_coeffs(kind, k, 2001, ids)
    S_ora = O.sketch_coeffs(kind, k, ids, 2001)
    assert np.array_equal(S_lib, S_ora)


def test_coefficient_argument_errors(L):
    with pytest.raises(skmp.SketchMPError):
        skmp.sketch_coeffs("sum", 2, 0, [0, 1])
    with pytest.raises(skmp.SketchMPError):
        skmp.sketch_coeffs("count", 0, 0, [0, 1])
    with pytest.raises(skmp.SketchMPError):
        skmp.sketch_coeffs("gauss", 65, 0, [0, 1])      # Gaussian draws are keyed by id * 64 + g
    with pytest.raises(skmp.SketchMPError):
        skmp.sketch_coeffs("count", 129, 0, [0, 1])
    with pytest.raises(skmp.SketchMPError):
        skmp.sketch_coeffs("count", 4, 0, [-1])


def _offs(*xs):
    a = np.array(xs, dtype=np.int64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def test_workspace_queries(L):
    a, p = _offs(0, 1000, 5000)
    assert L.mp_selfjoin_workspace(2, p, 4, 64, 0) > 0
    assert L.mp_selfjoin_workspace(2, p, 0, 64, 0) == 0
    assert L.top_discords_workspace(2, p, 4, 64) > 0
    assert L.sketch_build_workspace(8, 2, p, 4) > 0
    assert L.sketch_update_workspace(1000, 3, 2, 4) > 0
    big, pb = _offs(0, 1 << 20)
    assert L.mp_selfjoin_workspace(1, pb, 32, 256, 0) > L.mp_selfjoin_workspace(1, p, 32, 256, 0)


def test_selfjoin_rejects_bad_arguments_before_launch(L):
    a, p = _offs(0, 100, 300)
    fake = ctypes.c_void_p(16)  # never dereferenced: validation fails first
    ws = ctypes.c_void_p(256)
    cases = [
        dict(k=0, m=16, excl=4),     # k out of range
        dict(k=129, m=16, excl=4),
        dict(k=2, m=3, excl=1),      # m < 4
        dict(k=2, m=16, excl=0),     # excl < 1
        dict(k=2, m=150, excl=4),    # first series shorter than m
    ]
    for c in cases:
        rc = L.mp_selfjoin(fake, 300, 2, p, c["k"], c["m"], c["excl"], 0, 0, ~0 & ((1 << 64) - 1), fake, fake, 300,
                           ws, 1 << 30, None)
        assert rc == -1, c
        assert L.skmp_last_error()
    # more than 64 groups are joined in blocks, all of them: a partial mask is refused
    assert L.mp_selfjoin(fake, 300, 2, p, 100, 16, 4, 0, 0, (1 << 63) - 1, fake, fake, 300, ws, 1 << 30, None) == -1
    assert b"group_mask" in L.skmp_last_error()
    bad, pbad = _offs(0, 300, 100)   # decreasing offsets
    assert L.mp_selfjoin(fake, 300, 2, pbad, 2, 16, 4, 0, 0, 1, fake, fake, 300, ws, 1 << 30, None) == -1
    assert L.mp_selfjoin(fake, 100, 2, p, 2, 16, 4, 0, 0, 1, fake, fake, 300, ws, 1 << 30, None) == -1  # ldr < N
    assert L.mp_selfjoin(fake, 300, 2, p, 2, 16, 4, 7, 0, 1, fake, fake, 300, ws, 1 << 30, None) == -1  # prec
    assert L.mp_selfjoin(fake, 300, 2, p, 2, 16, 4, 0, 0, 1, fake, fake, 300, ws, 16, None) == -2     # workspace


def test_selfjoin_rejects_more_work_units_than_the_queue_numbers(L):
    """One series of 13 million windows with k = 8 in FP32 at refresh 256 needs
    8 x 12,696 bands x 50,782 strips > 2^32 work units: refused on the host
    before anything is launched (32-bit queue entries would wrap)."""
    n = 13_000_000
    a, p = _offs(0, n)
    fake = ctypes.c_void_p(16)
    rc = L.mp_selfjoin(fake, n, 1, p, 8, 100, 25, 1, 256, 0xFF, fake, fake, n, ctypes.c_void_p(256), 1 << 40, None)
    assert rc == -1
    assert b"work units" in L.skmp_last_error()
    # a quarter of the length is fine up to the workspace check
    a, p = _offs(0, n // 4)
    assert L.mp_selfjoin(fake, n, 1, p, 8, 100, 25, 1, 256, 0xFF, fake, fake, n, ctypes.c_void_p(256), 16, None) == -2


def test_series_beyond_32bit_statistics_offsets_refused(L):
    """The tile kernels address a series' window statistics (16 bytes per
    padded window) with 32-bit byte offsets: a series longer than 2^27 - 4096
    samples is refused on the host before anything is launched, and one at
    the limit passes the check (here it then stops at the workspace size)."""
    limit = 2 ** 27 - 4096
    fake = ctypes.c_void_p(16)
    for prec in (0, 1, 2, 3):
        a, p = _offs(0, limit + 1)
        rc = L.mp_selfjoin(fake, limit + 1, 1, p, 1, 16, 4, prec, 0, 1, fake, fake, limit + 1, fake, 16, None)
        assert rc == -1 and b"32-bit offsets" in L.skmp_last_error()
    # AB-join: the long series against a short one (few diagonals, few work units)
    assert L.mp_abjoin(fake, limit + 1, limit + 1, fake, 200, 200, 1, 16, 0, 0, 1, fake, fake, limit + 1, None, None,
                       0, fake, 16, None) == -1
    assert b"32-bit offsets" in L.skmp_last_error()
    assert L.mp_abjoin(fake, limit, limit, fake, 200, 200, 1, 16, 0, 0, 1, fake, fake, limit, None, None, 0, fake, 16,
                       None) == -2    # valid up to the workspace check


def test_build_and_discords_reject_bad_arguments(L):
    a, p = _offs(0, 100)
    fake = ctypes.c_void_p(16)
    assert L.sketch_build(fake, 0, 4, 100, 1, p, None, 0, 1, 0, 0, fake, 100, fake, fake, 1 << 20, None) == -1
    assert L.sketch_build(fake, 0, 4, 100, 1, p, None, 2, 0, 0, 0, fake, 100, fake, fake, 1 << 20, None) == -1
    assert L.sketch_build(fake, 5, 4, 100, 1, p, None, 2, 1, 0, 0, fake, 100, fake, fake, 1 << 20, None) == -1
    assert L.sketch_build(fake, 0, 4, 50, 1, p, None, 2, 1, 0, 0, fake, 100, fake, fake, 1 << 20, None) == -1
    assert L.top_discords(fake, 100, 1, p, 2, 16, 0, 0, fake, fake, fake, fake, fake, 1 << 20, None) == -1
    ids = np.array([3, 3], dtype=np.int64)
    assert L.sketch_update_dims(fake, 100, 100, 2, 1, 0, 0, 100, fake, 2, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                fake, None, 0, None, None, 0, None, fake, 1 << 20, None) == -1  # duplicate id


def test_noalloc_discords_refuse_inputs_beyond_their_scratch(L):
    """The allocation-free top_discords checks its limits (64 series, 2^21
    samples) on the host before it touches the device."""
    fake = ctypes.c_void_p(16)
    a, p = _offs(*range(0, 66 * 10, 10))              # 65 series
    assert L.top_discords_noalloc(fake, 1000, 65, p, 2, 4, 3, 0, fake, fake, fake, fake, None) == -1
    assert b"64 series" in L.skmp_last_error()
    a, p = _offs(0, 2 ** 21, 2 ** 21 + 1)              # 2^21 + 1 samples
    assert L.top_discords_noalloc(fake, 2 ** 22, 2, p, 2, 4, 3, 0, fake, fake, fake, fake, None) == -1
    assert b"2^21" in L.skmp_last_error()
    a, p = _offs(0, 100)
    assert L.top_discords_noalloc(fake, 100, 1, p, 2, 16, 0, 0, fake, fake, fake, fake, None) == -1  # top_k = 0


def test_tuning_table_round_trip_and_validation(L):
    skmp.tuning_clear()
    assert skmp.tuning_export() == ""
    text = "0 7 16 c8_pd2_w2_clfalse 4096 3.25\n1 6 15 f32_c16_pd2_w4 256 2.000000\n"
    skmp.tuning_import(text)
    rows = sorted(line.split() for line in skmp.tuning_export().splitlines())
    assert rows == [["0", "7", "16", "c8_pd2_w2_clfalse", "4096", "3.250000"],
                    ["1", "6", "15", "f32_c16_pd2_w4", "256", "2.000000"]]
    skmp.tuning_import("0 7 16 c6_pd1_w3_cltrue 1024 1.0\n")  # replaces the FP64 class entry
    assert "0 7 16 c6_pd1_w3_cltrue 1024 1.000000" in skmp.tuning_export()
    for bad in ["0 7 16 c99_pd2_w2_clfalse 2048 1.0",   # no such variant
                "0 7 16 3 2048 1.0",                     # numbered, not named
                "0 7 16 f32_c16_pd2_w4 2048 1.0",        # an FP32 variant for FP64
                "2 7 16 c8_pd2_w2_clfalse 2048 1.0", "0 7 16 c8_pd2_w2_clfalse 2048",
                "0 7 16 c8_pd2_w2_clfalse 2048 1.0 x", "1 6 15 f32_c16_pd2_w4 16 1"]:
        with pytest.raises(skmp.SketchMPError):
            skmp.tuning_import(bad)
    assert len(skmp.tuning_export().splitlines()) == 2   # a rejected import changes nothing
    for prec, default in (("fp64", "c8_pd2_w2_clfalse"), ("fp32", "f32_c16_pd2_w4"), ("bf16x3", "blocked_w2"),
                          ("fp16x3", "blocked_w2")):
        names = skmp.tile_variants(prec)
        assert default in names and len(set(names)) == len(names) >= 3
        for name in names:   # every listed variant is accepted by the table
            skmp.tuning_import(f"{skmp.PRECISIONS[prec]} 5 12 {name} 1024 1.0")
    # the 16-bit split precisions list both MFMA forms
    assert {"hankel", "blocked_w2"} <= set(skmp.tile_variants("bf16x3"))
    with pytest.raises(skmp.SketchMPError):
        skmp.tuning_import("2 5 12 f32_c16_pd2_w4 1024 1.0")   # an FP32 variant for BF16x3
    skmp.tuning_clear()
    assert skmp.tuning_export() == ""


def test_tuning_file_without_device(L, tmp_path):
    """The persistent tuning cache: a missing file loads nothing; saving, or
    loading an existing file, needs a device to stamp against and says so."""
    assert L.skmp_tuning_load(str(tmp_path / "absent.txt").encode()) == 0
    assert L.skmp_tuning_load(b"") == -1 and L.skmp_tuning_save(None) == -1
    (tmp_path / "t.txt").write_text("# sketchmp-tuning v1 arch=gfx950 hip=1\n")
    assert L.skmp_tuning_load(str(tmp_path / "t.txt").encode()) == -3
    assert b"device" in L.skmp_last_error()
    assert L.skmp_tuning_save(str(tmp_path / "u.txt").encode()) == -3
    assert not (tmp_path / "u.txt").exists()


def test_autotune_rejects_bad_arguments_before_launch(L):
    a, p = _offs(0, 300)
    fake = ctypes.c_void_p(16)
    v, sp, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    args = lambda prec, reps, k=2: (fake, 300, 1, p, k, 16, 4, prec, 0, fake, fake, 300, fake, 1 << 30, None, reps,
                                    ctypes.byref(v), ctypes.byref(sp), ctypes.byref(ms))
    assert L.mp_selfjoin_autotune(*args(7, 2)) == -1   # no such precision
    assert L.mp_selfjoin_autotune(*args(0, 0)) == -1   # reps
    assert L.mp_selfjoin_autotune(*args(0, 2, k=0)) == -1
    assert L.skmp_last_error()


def test_abjoin_workspace_and_argument_checks(L):
    assert L.mp_abjoin_workspace(1000, 3000, 4, 64, 0) > 0
    assert L.mp_abjoin_workspace(1000, 3000, 4, 64, 1) > 0
    assert L.mp_abjoin_workspace(1000, 3000, 4, 64, 2) == 0   # MFMA precisions: no AB-join
    fake = ctypes.c_void_p(16)
    M = (1 << 64) - 1

    def call(na=300, nb=500, k=2, m=16, prec=0, refresh=0, PB=fake, IB=fake, lda=300, ldpa=300, ws=1 << 30):
        return L.mp_abjoin(fake, lda, na, fake, 500, nb, k, m, prec, refresh, M, fake, fake, ldpa, PB, IB, 500,
                           fake, ws, None)
    assert call(prec=2) == -1           # BF16x3
    assert call(prec=3) == -1           # FP16x3
    assert call(na=10) == -1            # A shorter than m
    assert call(nb=8) == -1             # B shorter than m
    assert call(k=0) == -1
    assert call(m=3) == -1
    assert call(PB=None) == -1          # PB without IB
    assert call(lda=100) == -1          # stride below the length
    assert call(refresh=10) == -1
    assert call(ws=16) == -2            # workspace too small
    assert L.skmp_last_error()


def test_dim_detect_argument_checks(L):
    assert L.dim_detect_workspace(5000, 8, 64) > 0
    assert L.dim_detect_workspace(10, 8, 64) == 0
    fake = ctypes.c_void_p(16)
    other = ctypes.c_void_p(32)
    dims = np.array([0, 3, 5], dtype=np.int64)
    dp = dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))

    def call(Tte=fake, ste=fake, n_tr=1000, n_te=1000, d=6, i_star=10, m=32, excl=0, dtype=0, nd=3, ws=1 << 30):
        return L.dim_detect(fake, 1000, n_tr, fake, Tte, 1000, n_te, ste, dtype, d, dp, nd, i_star, m, excl, fake,
                            fake, fake, fake, ws, None)
    assert call(m=3) == -1                  # m < 4
    assert call(n_tr=20) == -1              # train shorter than m
    assert call(i_star=1000 - 31) == -1     # the subsequence runs past the test series
    assert call(i_star=-1) == -1
    assert call(d=5) == -1                  # dimension 5 out of range
    assert call(excl=8, Tte=other) == -1    # self-join setting needs the same series
    assert call(excl=8, ste=other) == -1
    assert call(dtype=3) == -1
    assert call(nd=0) == -1
    assert call(ws=16) == -2                # workspace too small
    assert L.skmp_last_error()


def test_streaming_argument_checks(L):
    i64p = ctypes.POINTER(ctypes.c_int64)

    def arr(*xs):
        a = np.array(xs, dtype=np.int64)
        return a, a.ctypes.data_as(i64p)

    nn, nnp = arr(1000, 3000)
    assert L.mp_selfjoin_append_workspace(2, nnp, 4, 64, 0) > 0
    assert L.mp_selfjoin_append_workspace(2, nnp, 4, 64, 1) > 0
    assert L.mp_selfjoin_append_workspace(2, nnp, 4, 64, 2) == 0   # MFMA precisions: no append
    fake = ctypes.c_void_p(16)
    M = (1 << 64) - 1

    def append(starts=(0, 4000), n_old=(900, 2500), n_new=(1000, 3000), k=2, m=64, excl=16, prec=0, ld=8000,
               ws=1 << 30):
        s, sp = arr(*starts)
        o, op = arr(*n_old)
        n, np_ = arr(*n_new)
        return L.mp_selfjoin_append(fake, ld, len(starts), sp, op, np_, k, m, excl, prec, 0, M, fake, fake, ld, fake,
                                    ws, None)
    assert append(prec=2) == -1                      # BF16x3
    assert append(n_old=(1100, 2500)) == -1          # n_old > n_new
    assert append(n_old=(-1, 2500)) == -1
    assert append(n_new=(50, 3000)) == -1            # shorter than m
    assert append(starts=(0, 500)) == -1             # overlapping series
    assert append(ld=5000) == -1                     # runs past the stride
    assert append(excl=0) == -1
    assert append(ws=16) == -2                       # workspace too small
    assert append(n_old=(1000, 3000)) == 0           # nothing new: no launch at all
    assert L.skmp_last_error() == b""

    no, nop = arr(0, 300, 300)
    dst, dstp = arr(1000, 5000, 5000)
    assert L.sketch_append_workspace(6, 2, nop, 4) > 0
    bad, badp = arr(1000, 1100)                      # series 1 would overwrite series 0's columns
    assert L.sketch_append(fake, 0, 6, 300, 2, nop, badp, None, 4, 1, 7, fake, 0, fake, 8000, fake, 1 << 30,
                           None) == -1
    far, farp = arr(7800, 8100)                      # series 0 runs past ldr
    assert L.sketch_append(fake, 0, 6, 300, 2, nop, farp, None, 4, 1, 7, fake, 0, fake, 8000, fake, 1 << 30,
                           None) == -1
    assert L.sketch_append(fake, 0, 6, 300, 2, nop, dstp, None, 2, 0, 7, fake, 0, fake, 8000, fake, 1 << 30,
                           None) == -1              # sum sketch with k = 2

    dims, dimsp = arr(0, 5)
    cols, colsp = arr(3, 99)
    dl = np.array([1.0, -2.0])
    dlp = dl.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.sketch_point_update_workspace(2, 4) > 0
    assert L.sketch_point_update_workspace(0, 4) == 0
    bd, bdp = arr(0, 6)                              # dimension 6 of 6
    assert L.sketch_point_update(fake, 100, 100, 4, 1, 7, 6, None, 1, fake, 2, None, bdp, colsp, dlp, None, fake,
                                 1 << 30, None) == -1
    bc, bcp = arr(3, 100)                            # column 100 of 100
    assert L.sketch_point_update(fake, 100, 100, 4, 1, 7, 6, None, 1, fake, 2, None, dimsp, bcp, dlp, None, fake,
                                 1 << 30, None) == -1
    inf = np.array([1.0, np.inf])
    assert L.sketch_point_update(fake, 100, 100, 4, 1, 7, 6, None, 1, fake, 2, None, dimsp, colsp,
                                 inf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, fake, 1 << 30,
                                 None) == -1
    assert L.sketch_point_update(fake, 100, 100, 4, 1, 7, 6, None, 1, fake, 2, None, dimsp, colsp, dlp, None, fake,
                                 16, None) == -2     # workspace too small
    assert L.sketch_point_update(fake, 100, 100, 4, 1, 7, 6, None, 1, fake, 0, None, None, None, None, None, None,
                                 0, None) == 0       # no updates: nothing to do, nothing launched


def test_default_k_is_the_ceiling_of_sqrt_d_capped_at_128(L):
    """k = ceil(sqrt(d)) (the k of the cost analysis and of every experiment of
    Section IV), against the smallest integer whose square reaches d, found by
    counting; capped at the library's 128 groups; d < 1 is an error."""
    for d in list(range(1, 5000)) + [7_500, 10_000, 16_384, 16_385, 2**31, 2**40]:
        s = 1
        while s * s < d:
            s += 1
        assert L.sketch_default_k(d) == min(s, 128), d
    assert [L.sketch_default_k(d) for d in (1, 2, 4, 5, 9, 10, 3969, 3970)] == [1, 2, 2, 3, 3, 4, 63, 64]
    assert [L.sketch_default_k(d) for d in (5_000, 7_500, 10_000)] == [71, 87, 100]   # the paper's largest d
    assert L.sketch_default_k(0) == -1 and L.sketch_default_k(-5) == -1
    assert b"d must be" in L.skmp_last_error()
