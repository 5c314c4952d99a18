"""Python binding of libsketchmp (sketched matrix-profile discord mining on MI355X).

Argument marshalling only: every step runs in the HIP kernels of
``libsketchmp.so`` (built by ``paper_2311_03393_amd.build``).  PyTorch supplies
device memory and the current stream.  There is no fallback: if the library
is missing, or no GPU is present, every call raises.

Functions mirror the C-ABI in ``include/sketchmp.h``:

* ``sketch_build``        normalise and sketch (Section III-A, Algorithm 1)
* ``sketch_update_dims``  add / remove dimensions (Section III-C)
* ``mp_selfjoin``         self-join matrix profile of each sketched series
* ``top_discords``        Algorithm 2 plus the ordered discord list
* ``sketch_coeffs``       the coefficient matrix S (host computation)
* ``mp_abjoin``           AB-join between a test and a train series (Algorithm 2)
* ``dim_detect``          discord dimension detection (Algorithm 3)
* ``sketch_append``, ``sketch_point_update``, ``mp_selfjoin_append``
                          the streaming extension (Section III-B) and point
                          updates (Section III-C)
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsketchmp.so")

SUM, COUNT, GAUSS = 0, 1, 2
KINDS = {"sum": SUM, "count": COUNT, "gauss": GAUSS}
F64, F32 = 0, 1
FP64, FP32, BF16X3, FP16X3 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "fp16x3": FP16X3}
FLAG_CHECK_FINITE = 1

ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENONFINITE", -5: "ENOTFOUND"}

# every symbol include/sketchmp.h declares
EXPORTED = ("skmp_last_error", "skmp_version", "sketch_coeffs", "sketch_default_k", "sketch_build_workspace",
            "sketch_build",
            "sketch_update_workspace", "sketch_update_dims", "mp_selfjoin_workspace", "mp_selfjoin",
            "mp_selfjoin_autotune", "mp_abjoin_workspace", "mp_abjoin", "dim_detect_workspace", "dim_detect",
            "sketch_append_workspace", "sketch_append", "sketch_point_update_workspace", "sketch_point_update",
            "mp_selfjoin_append_workspace", "mp_selfjoin_append", "skmp_tuning_export", "skmp_tile_variants",
            "skmp_tuning_import", "skmp_tuning_clear", "skmp_tuning_save", "skmp_tuning_load",
            "top_discords_workspace", "top_discords", "top_discords_noalloc", "skmp_timing_enable",
            "skmp_timing_read")
TIMERS = {"sketch": 0, "substats": 1, "tiles": 2, "merge": 3, "discords": 4, "dimdetect": 5}


class SketchMPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None
_vp, _i32, _i64, _u32, _u64, _sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                    ctypes.c_uint64, ctypes.c_size_t)
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def lib():
    """Load libsketchmp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2311_03393_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.skmp_last_error.restype = ctypes.c_char_p
        L.skmp_version.restype = ctypes.c_char_p
        L.sketch_coeffs.argtypes = [_i32, _i32, _u64, _i64p, _i64, _dp]
        L.sketch_default_k.argtypes = [_i64]
        L.sketch_default_k.restype = _i32
        L.sketch_build_workspace.argtypes = [_i64, _i64, _i64p, _i32]
        L.sketch_build_workspace.restype = _sz
        L.sketch_build.argtypes = [_vp, _i32, _i64, _i64, _i64, _i64p, _i64p, _i32, _i32, _u64, _u32, _vp, _i64,
                                   _vp, _vp, _sz, _vp]
        L.sketch_update_workspace.argtypes = [_i64, _i64, _i64, _i32]
        L.sketch_update_workspace.restype = _sz
        L.sketch_update_dims.argtypes = [_vp, _i64, _i64, _i32, _i32, _u64, _i32, _i64, _vp, _i64, _i64p, _vp,
                                         _vp, _i64, _i64p, _vp, _u32, _u64p, _vp, _sz, _vp]
        L.mp_selfjoin_workspace.argtypes = [_i64, _i64p, _i32, _i32, _i32]
        L.mp_selfjoin_workspace.restype = _sz
        L.mp_selfjoin.argtypes = [_vp, _i64, _i64, _i64p, _i32, _i32, _i32, _i32, _i32, _u64, _vp, _vp, _i64, _vp,
                                  _sz, _vp]
        L.mp_abjoin_workspace.argtypes = [_i64, _i64, _i32, _i32, _i32]
        L.mp_abjoin_workspace.restype = _sz
        L.mp_abjoin.argtypes = [_vp, _i64, _i64, _vp, _i64, _i64, _i32, _i32, _i32, _i32, _u64, _vp, _vp, _i64, _vp,
                                _vp, _i64, _vp, _sz, _vp]
        L.dim_detect_workspace.argtypes = [_i64, _i32, _i32]
        L.dim_detect_workspace.restype = _sz
        L.dim_detect.argtypes = [_vp, _i64, _i64, _vp, _vp, _i64, _i64, _vp, _i32, _i64, _i64p, _i32, _i64, _i32,
                                 _i32, _vp, _vp, _vp, _vp, _sz, _vp]
        L.sketch_append_workspace.argtypes = [_i64, _i64, _i64p, _i32]
        L.sketch_append_workspace.restype = _sz
        L.sketch_append.argtypes = [_vp, _i32, _i64, _i64, _i64, _i64p, _i64p, _i64p, _i32, _i32, _u64, _vp, _u32,
                                    _vp, _i64, _vp, _sz, _vp]
        L.sketch_point_update_workspace.argtypes = [_i64, _i32]
        L.sketch_point_update_workspace.restype = _sz
        L.sketch_point_update.argtypes = [_vp, _i64, _i64, _i32, _i32, _u64, _i64, _i64p, _i64, _vp, _i64, _i64p,
                                          _i64p, _i64p, _dp, _u64p, _vp, _sz, _vp]
        L.mp_selfjoin_append_workspace.argtypes = [_i64, _i64p, _i32, _i32, _i32]
        L.mp_selfjoin_append_workspace.restype = _sz
        L.mp_selfjoin_append.argtypes = [_vp, _i64, _i64, _i64p, _i64p, _i64p, _i32, _i32, _i32, _i32, _i32, _u64,
                                         _vp, _vp, _i64, _vp, _sz, _vp]
        L.top_discords_workspace.argtypes = [_i64, _i64p, _i32, _i32]
        L.top_discords_workspace.restype = _sz
        L.top_discords.argtypes = [_vp, _i64, _i64, _i64p, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _sz,
                                   _vp]
        L.top_discords_noalloc.argtypes = [_vp, _i64, _i64, _i64p, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp]
        L.mp_selfjoin_autotune.argtypes = [_vp, _i64, _i64, _i64p, _i32, _i32, _i32, _i32, _i32, _vp, _vp, _i64,
                                           _vp, _sz, _vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32), _dp]
        L.skmp_tuning_export.argtypes = [ctypes.c_char_p, _sz]
        L.skmp_tuning_export.restype = _sz
        L.skmp_tuning_import.argtypes = [ctypes.c_char_p]
        L.skmp_tuning_save.argtypes = [ctypes.c_char_p]
        L.skmp_tuning_load.argtypes = [ctypes.c_char_p]
        L.skmp_tile_variants.argtypes = [_i32, ctypes.c_char_p, _sz]
        L.skmp_tile_variants.restype = _sz
        L.skmp_timing_enable.argtypes = [ctypes.c_int]
        L.skmp_timing_read.argtypes = [_i32, _i32, _dp, _i64p]
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != 0:
        raise SketchMPError(rc, lib().skmp_last_error().decode())


def _i64arr(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.int64))


def _ptr64(a: np.ndarray):
    return a.ctypes.data_as(_i64p)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("sketchmp needs a GPU (no HIP device visible)")
    return torch


def _ld(t) -> int:
    """Row stride of a 2-D tensor; a single-row tensor may carry any stride."""
    return int(t.shape[1]) if t.shape[0] == 1 else int(t.stride(0))


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_ws_cache = {}


def _workspace(torch, nbytes: int, device):
    # one cached scratch buffer per (device, stream): calls on one stream run in
    # order, calls on different streams may overlap and must not share scratch
    key = (str(device), torch.cuda.current_stream().cuda_stream)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def timing_enable(on: bool = True) -> None:
    """Record HIP events around every timed stage launch (see include/sketchmp.h)."""
    _check(lib().skmp_timing_enable(1 if on else 0))


def timing_read(stage: str, reset: bool = True):
    """(summed device milliseconds, launches) of a stage since the last reset."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().skmp_timing_read(TIMERS[stage], 1 if reset else 0, ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


def version() -> str:
    return lib().skmp_version().decode()


def sketch_coeffs(kind: str, k: int, seed: int, dim_ids: Sequence[int]) -> np.ndarray:
    """Coefficient matrix S (k x d) drawn by the library (host computation)."""
    ids = _i64arr(dim_ids)
    S = np.empty((k, ids.size), dtype=np.float64)
    _check(lib().sketch_coeffs(KINDS[kind], k, seed, _ptr64(ids), ids.size, S.ctypes.data_as(_dp)))
    return S


def sketch_default_k(d: int) -> int:
    """ceil(sqrt(d)) capped at 64 (see include/sketchmp.h)."""
    k = lib().sketch_default_k(d)
    _check(min(k, 0))
    return k


def sketch_build(T, offsets, k: int, kind: str, seed: int, dim_ids=None, check_finite: bool = False, R=None,
                 stats=None):
    """Normalise every dimension per series and sketch: returns (R k x N, dim_stats n_series x d x 2).
    k = 0 takes sketch_default_k(d)."""
    torch = _torch()
    assert T.is_cuda and T.dim() == 2 and T.stride(1) == 1
    dtype = {torch.float64: F64, torch.float32: F32}[T.dtype]
    d, N = T.shape
    if k == 0:
        k = sketch_default_k(d)
    offs = _i64arr(offsets)
    n_series = offs.size - 1
    ids = None if dim_ids is None else _i64arr(dim_ids)
    if R is None:
        R = torch.empty((k, N), dtype=torch.float64, device=T.device)
    if stats is None:
        stats = torch.empty((n_series, d, 2), dtype=torch.float64, device=T.device)
    ws_n = lib().sketch_build_workspace(d, n_series, _ptr64(offs), k)
    ws = _workspace(torch, ws_n, T.device)
    _check(lib().sketch_build(T.data_ptr(), dtype, d, _ld(T), n_series, _ptr64(offs),
                              None if ids is None else _ptr64(ids), k, KINDS[kind], seed,
                              FLAG_CHECK_FINITE if check_finite else 0, R.data_ptr(), _ld(R), stats.data_ptr(),
                              ws.data_ptr(), ws.numel(), _stream(torch)))
    return R, stats


def sketch_update_dims(R, kind: str, k: int, seed: int, T_add=None, add_ids=(), T_rem=None, rem_ids=(),
                       rem_stats=None, check_finite: bool = False):
    """Add / remove dimensions in place (Section III-C); returns (add_stats, changed_group_mask)."""
    torch = _torch()
    n = R.shape[1]
    add_ids = _i64arr(add_ids)
    rem_ids = _i64arr(rem_ids)
    d_add, d_rem = add_ids.size, rem_ids.size
    ref = T_add if d_add else T_rem
    dtype = F64 if (ref is None or ref.dtype == torch.float64) else F32
    ldt = _ld(ref) if ref is not None else n
    if d_add and d_rem:
        assert T_add.dtype == T_rem.dtype and _ld(T_add) == _ld(T_rem)
    add_stats = torch.empty((max(d_add, 1), 2), dtype=torch.float64, device=R.device)
    mask = ctypes.c_uint64(0)
    ws_n = lib().sketch_update_workspace(n, d_add, d_rem, k)
    ws = _workspace(torch, ws_n, R.device)
    _check(lib().sketch_update_dims(R.data_ptr(), _ld(R), n, k, KINDS[kind], seed, dtype, ldt,
                                    T_add.data_ptr() if d_add else None, d_add, _ptr64(add_ids),
                                    add_stats.data_ptr() if d_add else None,
                                    T_rem.data_ptr() if d_rem else None, d_rem, _ptr64(rem_ids),
                                    rem_stats.data_ptr() if d_rem else None,
                                    FLAG_CHECK_FINITE if check_finite else 0, ctypes.byref(mask), ws.data_ptr(),
                                    ws.numel(), _stream(torch)))
    return add_stats[:d_add], int(mask.value)


def mp_selfjoin_workspace(offsets, k: int, m: int, prec: str = "fp64") -> int:
    offs = _i64arr(offsets)
    return int(lib().mp_selfjoin_workspace(offs.size - 1, _ptr64(offs), k, m, PRECISIONS[prec]))


def mp_selfjoin(R, offsets, k: int, m: int, excl: int, prec: str = "fp64", refresh: int = 0,
                group_mask: Optional[int] = None, P=None, I=None, workspace=None):
    """Self-join matrix profile per sketched series: returns (P k x N float64, I k x N int64)."""
    torch = _torch()
    offs = _i64arr(offsets)
    n_series = offs.size - 1
    N = int(offs[-1])
    if P is None:
        P = torch.full((k, N), float("nan"), dtype=torch.float64, device=R.device)
    if I is None:
        I = torch.full((k, N), -2, dtype=torch.int64, device=R.device)
    assert _ld(P) == _ld(I)
    if workspace is None:
        ws_n = lib().mp_selfjoin_workspace(n_series, _ptr64(offs), k, m, PRECISIONS[prec])
        workspace = _workspace(torch, ws_n, R.device)
    mask = (1 << 64) - 1 if group_mask is None else int(group_mask)
    _check(lib().mp_selfjoin(R.data_ptr(), _ld(R), n_series, _ptr64(offs), k, m, excl, PRECISIONS[prec],
                             refresh, mask, P.data_ptr(), I.data_ptr(), _ld(P), workspace.data_ptr(),
                             workspace.numel(), _stream(torch)))
    return P, I


def mp_abjoin_workspace(na: int, nb: int, k: int, m: int, prec: str = "fp64") -> int:
    return int(lib().mp_abjoin_workspace(na, nb, k, m, PRECISIONS[prec]))


def mp_abjoin(RA, RB, k: int, m: int, prec: str = "fp64", refresh: int = 0, group_mask: Optional[int] = None,
              both: bool = False, PA=None, IA=None, PB=None, IB=None, workspace=None):
    """AB-join: nearest subsequence of RB for every subsequence of RA (and, with
    both=True, the converse).  Returns (PA, IA) or (PA, IA, PB, IB); PA/IA are
    k x na with the last m - 1 columns unused, IA indexes windows of RB."""
    torch = _torch()
    na, nb = int(RA.shape[1]), int(RB.shape[1])
    if PA is None:
        PA = torch.full((k, na), float("nan"), dtype=torch.float64, device=RA.device)
    if IA is None:
        IA = torch.full((k, na), -2, dtype=torch.int64, device=RA.device)
    assert _ld(PA) == _ld(IA)
    if both and PB is None:
        PB = torch.full((k, nb), float("nan"), dtype=torch.float64, device=RA.device)
    if both and IB is None:
        IB = torch.full((k, nb), -2, dtype=torch.int64, device=RA.device)
    if both:
        assert _ld(PB) == _ld(IB)
    if workspace is None:
        workspace = _workspace(torch, lib().mp_abjoin_workspace(na, nb, k, m, PRECISIONS[prec]), RA.device)
    mask = (1 << 64) - 1 if group_mask is None else int(group_mask)
    _check(lib().mp_abjoin(RA.data_ptr(), _ld(RA), na, RB.data_ptr(), _ld(RB), nb, k, m, PRECISIONS[prec], refresh,
                           mask, PA.data_ptr(), IA.data_ptr(), _ld(PA), PB.data_ptr() if both else None,
                           IB.data_ptr() if both else None, _ld(PB) if both else 0, workspace.data_ptr(),
                           workspace.numel(), _stream(torch)))
    return (PA, IA, PB, IB) if both else (PA, IA)


def exact_profiles(T, m: int, excl: int, prec: str = "fp64", refresh: int = 0):
    """The exact multidimensional baseline: the self-join profile of every
    dimension of one series (T: d x n contiguous device tensor), i.e. the sketch
    with k = d and the identity.  Runs as one batched launch per stage: the d
    dimensions are d one-dimensional series of the batch, each z-normalised by
    the sum sketch of one dimension.  Returns (P, I) as d x n tensors."""
    torch = _torch()
    assert T.is_contiguous() and T.dim() == 2
    d, n = int(T.shape[0]), int(T.shape[1])
    flat = T.reshape(1, d * n)
    offsets = np.arange(d + 1, dtype=np.int64) * n
    R, _ = sketch_build(flat, offsets, 1, "sum", 0)
    P, I = mp_selfjoin(R, offsets, 1, m, excl, prec=prec, refresh=refresh)
    return P.reshape(d, n), I.reshape(d, n)


def refine_discord(T, j: int, m: int, excl: int, prec: str = "fp64", refresh: int = 0):
    """The optional refinement after Algorithm 3: the self-join of the whole
    detected dimension j (z-normalised) and its top discord.  Returns
    (start, score) as host values."""
    P, _ = exact_profiles(T[j:j + 1].contiguous(), m, excl, prec=prec, refresh=refresh)
    n = int(T.shape[1])
    idx, _, score, nf = top_discords(P, [0, n], 1, m, 1)
    return int(idx[0, 0].item()), float(score[0, 0].item())


def group_dims(kind: str, k: int, seed: int, g: int, dim_ids) -> np.ndarray:
    """Rows of the dimensions that sketch group g mixes (J_g: non-zero coefficients)."""
    S = sketch_coeffs(kind, k, seed, dim_ids)
    return np.nonzero(S[g])[0].astype(np.int64)


def dim_detect(T_train, stats_train, dims, i_star: int, m: int, T_test=None, stats_test=None, excl: int = 0):
    """Discord dimension detection (Algorithm 3).  T_* are d x n device tensors
    of one series each, stats_* their (mu, sigma) per dimension (d x 2, as
    sketch_build returns for a one-series call); without T_test the test series
    is the train series (excl > 0 then excludes trivial matches of i_star).
    Returns (scores, nn, position of j* in dims) as device tensors."""
    torch = _torch()
    same = T_test is None
    if same:
        T_test, stats_test = T_train, stats_train
    assert T_train.dtype == T_test.dtype and T_train.stride(1) == 1 and T_test.stride(1) == 1
    dtype = {torch.float64: F64, torch.float32: F32}[T_train.dtype]
    st_tr = stats_train.reshape(-1, 2).contiguous()
    st_te = st_tr if same else stats_test.reshape(-1, 2).contiguous()
    dims = _i64arr(dims)
    n_tr, n_te = int(T_train.shape[1]), int(T_test.shape[1])
    scores = torch.empty(dims.size, dtype=torch.float64, device=T_train.device)
    nn = torch.empty(dims.size, dtype=torch.int64, device=T_train.device)
    best = torch.empty(1, dtype=torch.int32, device=T_train.device)
    ws = _workspace(torch, lib().dim_detect_workspace(n_tr, dims.size, m), T_train.device)
    _check(lib().dim_detect(T_train.data_ptr(), _ld(T_train), n_tr, st_tr.data_ptr(), T_test.data_ptr(), _ld(T_test),
                            n_te, st_te.data_ptr(), dtype, int(T_train.shape[0]), _ptr64(dims), dims.size, i_star, m,
                            excl, scores.data_ptr(), nn.data_ptr(), best.data_ptr(), ws.data_ptr(), ws.numel(),
                            _stream(torch)))
    return scores, nn, best


def sketch_append(T_new, new_offsets, dst_cols, R, stats, k: int, kind: str, seed: int, dim_ids=None,
                  check_finite: bool = False):
    """Sketch newly arrived samples into R with the frozen statistics the
    sketch was built with (Algorithm 1's projection, Section III-B's streaming
    extension).  T_new: d x N_new device tensor, the new samples of every
    series back to back (new_offsets, n_series + 1); series s's go to columns
    dst_cols[s], ... of R; stats: n_series x d x 2 (sketch_build's).  Returns R."""
    torch = _torch()
    assert T_new.is_cuda and T_new.dim() == 2 and T_new.stride(1) == 1
    dtype = {torch.float64: F64, torch.float32: F32}[T_new.dtype]
    d = int(T_new.shape[0])
    offs = _i64arr(new_offsets)
    dst = _i64arr(dst_cols)
    n_series = offs.size - 1
    assert dst.size == n_series
    ids = None if dim_ids is None else _i64arr(dim_ids)
    ws = _workspace(torch, lib().sketch_append_workspace(d, n_series, _ptr64(offs), k), R.device)
    _check(lib().sketch_append(T_new.data_ptr(), dtype, d, _ld(T_new), n_series, _ptr64(offs), _ptr64(dst),
                               None if ids is None else _ptr64(ids), k, KINDS[kind], seed, stats.data_ptr(),
                               FLAG_CHECK_FINITE if check_finite else 0, R.data_ptr(), _ld(R), ws.data_ptr(),
                               ws.numel(), _stream(torch)))
    return R


def sketch_point_update(R, stats, k: int, kind: str, seed: int, dims, cols, deltas, series=None, dim_ids=None,
                        n_cols: Optional[int] = None) -> int:
    """Point updates (Section III-C): sample cols[u] of dimension dims[u] (of
    series series[u]) rose by deltas[u]; R changes in place.  stats: n_series x
    d x 2.  Returns the mask of the groups that changed."""
    torch = _torch()
    st = stats.reshape(-1, stats.shape[-2], 2) if stats.dim() == 3 else stats.reshape(1, -1, 2)
    n_series, d = int(st.shape[0]), int(st.shape[1])
    dims_a, cols_a = _i64arr(dims), _i64arr(cols)
    deltas_a = np.ascontiguousarray(np.asarray(deltas, dtype=np.float64))
    ser = None if series is None else _i64arr(series)
    ids = None if dim_ids is None else _i64arr(dim_ids)
    n_upd = int(dims_a.size)
    assert cols_a.size == n_upd and deltas_a.size == n_upd and (ser is None or ser.size == n_upd)
    nc = int(R.shape[1]) if n_cols is None else int(n_cols)
    mask = ctypes.c_uint64(0)
    ws = _workspace(torch, max(lib().sketch_point_update_workspace(n_upd, k), 256), R.device)
    _check(lib().sketch_point_update(R.data_ptr(), _ld(R), nc, k, KINDS[kind], seed, d,
                                     None if ids is None else _ptr64(ids), n_series, st.data_ptr(), n_upd,
                                     None if ser is None else _ptr64(ser), _ptr64(dims_a), _ptr64(cols_a),
                                     deltas_a.ctypes.data_as(_dp), ctypes.byref(mask), ws.data_ptr(), ws.numel(),
                                     _stream(torch)))
    return int(mask.value)


def mp_selfjoin_append_workspace(n_new, k: int, m: int, prec: str = "fp64") -> int:
    nn = _i64arr(n_new)
    return int(lib().mp_selfjoin_append_workspace(nn.size, _ptr64(nn), k, m, PRECISIONS[prec]))


def mp_selfjoin_append(R, P, I, starts, n_old, n_new, k: int, m: int, excl: int, prec: str = "fp64",
                       refresh: int = 0, group_mask: Optional[int] = None, workspace=None):
    """Streaming self-join update: series s (columns starts[s] ... of R, P, I)
    grew from n_old[s] to n_new[s] samples; P, I, holding the profile of the
    first n_old[s] samples, are updated in place to that of all n_new[s]."""
    torch = _torch()
    st, no, nn = _i64arr(starts), _i64arr(n_old), _i64arr(n_new)
    n_series = st.size
    assert no.size == n_series and nn.size == n_series and _ld(P) == _ld(I)
    if workspace is None:
        workspace = _workspace(torch, lib().mp_selfjoin_append_workspace(n_series, _ptr64(nn), k, m,
                                                                         PRECISIONS[prec]), R.device)
    mask = (1 << 64) - 1 if group_mask is None else int(group_mask)
    _check(lib().mp_selfjoin_append(R.data_ptr(), _ld(R), n_series, _ptr64(st), _ptr64(no), _ptr64(nn), k, m, excl,
                                    PRECISIONS[prec], refresh, mask, P.data_ptr(), I.data_ptr(), _ld(P),
                                    workspace.data_ptr(), workspace.numel(), _stream(torch)))
    return P, I


def mp_selfjoin_autotune(R, offsets, k: int, m: int, excl: int, prec: str = "fp64", refresh: int = 0,
                         reps: int = 2, P=None, I=None, workspace=None) -> dict:
    """Time every launch configuration of the self-join on this input and keep the
    fastest for later calls of the same shape class; returns {variant, strip, ms}."""
    torch = _torch()
    offs = _i64arr(offsets)
    n_series = offs.size - 1
    N = int(offs[-1])
    if P is None:
        P = torch.empty((k, N), dtype=torch.float64, device=R.device)
    if I is None:
        I = torch.empty((k, N), dtype=torch.int64, device=R.device)
    if workspace is None:
        ws_n = lib().mp_selfjoin_workspace(n_series, _ptr64(offs), k, m, PRECISIONS[prec])
        workspace = _workspace(torch, ws_n, R.device)
    v, sp, ms = ctypes.c_int32(-1), ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(lib().mp_selfjoin_autotune(R.data_ptr(), _ld(R), n_series, _ptr64(offs), k, m, excl, PRECISIONS[prec],
                                      refresh, P.data_ptr(), I.data_ptr(), _ld(P), workspace.data_ptr(),
                                      workspace.numel(), _stream(torch), reps, ctypes.byref(v), ctypes.byref(sp),
                                      ctypes.byref(ms)))
    return {"variant": v.value, "strip": sp.value, "ms": ms.value}


def tile_variants(prec: str) -> list:
    """Names of the compiled tile-kernel variants of an FP64 or FP32 self-join."""
    n = lib().skmp_tile_variants(PRECISIONS[prec], None, 0)
    buf = ctypes.create_string_buffer(n)
    lib().skmp_tile_variants(PRECISIONS[prec], buf, n)
    return buf.value.decode().split()


def tuning_export() -> str:
    """The process's tuning table, one 'prec mlog nlog variant-name strip ms' line per shape class."""
    n = lib().skmp_tuning_export(None, 0)
    buf = ctypes.create_string_buffer(n)
    lib().skmp_tuning_export(buf, n)
    return buf.value.decode()


def tuning_import(text: str) -> None:
    _check(lib().skmp_tuning_import(text.encode()))


def tuning_clear() -> None:
    _check(lib().skmp_tuning_clear())


def tuning_save(path: str) -> None:
    """Write the tuning table to `path`, stamped with the device architecture and HIP runtime version."""
    _check(lib().skmp_tuning_save(os.fsencode(path)))


def tuning_load(path: str) -> int:
    """Add the entries of a tuning file written under the current stamp; returns how many (0: missing or stale)."""
    rc = lib().skmp_tuning_load(os.fsencode(path))
    _check(min(rc, 0))
    return rc


def top_discords(P, offsets, k: int, m: int, top_k: int, halfwidth: int = 0, out=None):
    """Ordered non-overlapping discords per series: (idx, group, score, n_found) device tensors."""
    torch = _torch()
    offs = _i64arr(offsets)
    n_series = offs.size - 1
    if out is None:
        idx = torch.empty((n_series, top_k), dtype=torch.int64, device=P.device)
        grp = torch.empty((n_series, top_k), dtype=torch.int32, device=P.device)
        score = torch.empty((n_series, top_k), dtype=torch.float64, device=P.device)
        nf = torch.empty((n_series,), dtype=torch.int32, device=P.device)
    else:
        idx, grp, score, nf = out
    ws_n = lib().top_discords_workspace(n_series, _ptr64(offs), k, m)
    ws = _workspace(torch, ws_n, P.device)
    _check(lib().top_discords(P.data_ptr(), _ld(P), n_series, _ptr64(offs), k, m, top_k, halfwidth,
                              idx.data_ptr(), grp.data_ptr(), score.data_ptr(), nf.data_ptr(), ws.data_ptr(),
                              ws.numel(), _stream(torch)))
    return idx, grp, score, nf


def top_discords_noalloc(P, offsets, k: int, m: int, top_k: int, halfwidth: int = 0, out=None):
    """top_discords through the allocation-free entry point (library-owned
    scratch; at most 64 series and 2^21 samples).  With ``out`` given, the call
    allocates nothing: (idx, group, score, n_found) device tensors."""
    torch = _torch()
    offs = _i64arr(offsets)
    n_series = offs.size - 1
    if out is None:
        idx = torch.empty((n_series, top_k), dtype=torch.int64, device=P.device)
        grp = torch.empty((n_series, top_k), dtype=torch.int32, device=P.device)
        score = torch.empty((n_series, top_k), dtype=torch.float64, device=P.device)
        nf = torch.empty((n_series,), dtype=torch.int32, device=P.device)
    else:
        idx, grp, score, nf = out
    _check(lib().top_discords_noalloc(P.data_ptr(), _ld(P), n_series, _ptr64(offs), k, m, top_k, halfwidth,
                                      idx.data_ptr(), grp.data_ptr(), score.data_ptr(), nf.data_ptr(),
                                      _stream(torch)))
    return idx, grp, score, nf
