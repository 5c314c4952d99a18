"""ctypes binding of the plain-C brute-force profile (mp_bruteforce.c).

Test infrastructure only.  ``build_c_oracle()`` compiles it with gcc and
OpenMP; ``c_oracle()`` loads the result.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mp_bruteforce.c")
_SRC_DIAG = os.path.join(_HERE, "mp_diag.c")
_LIB = os.path.join(_HERE, "libmp_oracle.so")
_lib = None


def build_c_oracle(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        # AVX2 + FMA (every x86-64 server part of the last decade); no
        # -ffast-math: the double-double arithmetic needs IEEE rounding
        # (-fno-math-errno only lets sqrt vectorise)
        subprocess.check_call(["gcc", "-O3", "-mavx2", "-mfma", "-fno-math-errno", "-fopenmp", "-fPIC", "-shared",
                               "-std=c99", "-o", tmp, _SRC, _SRC_DIAG, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _COracle:
    def __init__(self, lib):
        self.lib = lib
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_mp_rows.argtypes = [dp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ip, ctypes.c_int64, dp, ip]
        lib.oracle_mp_rows.restype = ctypes.c_int
        lib.oracle_pair_dist.argtypes = [dp, ctypes.c_int64, ctypes.c_int, ip, ip, ctypes.c_int64, dp]
        lib.oracle_pair_dist.restype = ctypes.c_int
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_ab_rows.argtypes = [dp, ctypes.c_int64, dp, ctypes.c_int64, ctypes.c_int, ip, ctypes.c_int64, dp,
                                       ip]
        lib.oracle_ab_rows.restype = ctypes.c_int
        lib.oracle_ab_pair_dist.argtypes = [dp, ctypes.c_int64, dp, ctypes.c_int64, ctypes.c_int, ip, ip,
                                            ctypes.c_int64, dp]
        lib.oracle_ab_pair_dist.restype = ctypes.c_int
        lib.oracle_mp_diag.argtypes = [dp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, dp, ip]
        lib.oracle_mp_diag.restype = ctypes.c_int

    @staticmethod
    def _d(a):
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    @staticmethod
    def _i(a):
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))

    def threads(self) -> int:
        return int(self.lib.oracle_threads())

    def profile(self, r, m: int, excl: int, rows=None):
        r = np.ascontiguousarray(r, dtype=np.float64)
        n_sub = r.size - m + 1
        if rows is None:
            P = np.empty(n_sub)
            I = np.empty(n_sub, np.int64)
            rc = self.lib.oracle_mp_rows(self._d(r), r.size, m, excl, None, 0, self._d(P), self._i(I))
        else:
            rows = np.ascontiguousarray(rows, dtype=np.int64)
            P = np.empty(rows.size)
            I = np.empty(rows.size, np.int64)
            rc = self.lib.oracle_mp_rows(self._d(r), r.size, m, excl, self._i(rows), rows.size, self._d(P), self._i(I))
        if rc != 0:
            raise RuntimeError(f"oracle_mp_rows failed ({rc})")
        return P, I

    def profile_diag(self, r, m: int, excl: int):
        """Whole self-join profile by the diagonal double-double reference (mp_diag.c)."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        n_sub = r.size - m + 1
        P = np.empty(n_sub)
        I = np.empty(n_sub, np.int64)
        rc = self.lib.oracle_mp_diag(self._d(r), r.size, m, excl, self._d(P), self._i(I))
        if rc != 0:
            raise RuntimeError(f"oracle_mp_diag failed ({rc})")
        return P, I

    def pair_dist(self, r, m: int, pi, pj):
        r = np.ascontiguousarray(r, dtype=np.float64)
        pi = np.ascontiguousarray(pi, dtype=np.int64)
        pj = np.ascontiguousarray(pj, dtype=np.int64)
        out = np.empty(pi.size)
        rc = self.lib.oracle_pair_dist(self._d(r), r.size, m, self._i(pi), self._i(pj), pi.size, self._d(out))
        if rc != 0:
            raise RuntimeError("oracle_pair_dist failed")
        return out


    def ab_profile(self, ra, rb, m: int, rows=None):
        """AB-join: nearest subsequence of rb for every (listed) subsequence of ra."""
        ra = np.ascontiguousarray(ra, dtype=np.float64)
        rb = np.ascontiguousarray(rb, dtype=np.float64)
        if rows is None:
            cnt, rp = ra.size - m + 1, None
        else:
            rows = np.ascontiguousarray(rows, dtype=np.int64)
            cnt, rp = rows.size, self._i(rows)
        P = np.empty(cnt)
        I = np.empty(cnt, np.int64)
        rc = self.lib.oracle_ab_rows(self._d(ra), ra.size, self._d(rb), rb.size, m, rp, 0 if rows is None else cnt,
                                     self._d(P), self._i(I))
        if rc != 0:
            raise RuntimeError(f"oracle_ab_rows failed ({rc})")
        return P, I

    def ab_pair_dist(self, ra, rb, m: int, pi, pj):
        ra = np.ascontiguousarray(ra, dtype=np.float64)
        rb = np.ascontiguousarray(rb, dtype=np.float64)
        pi = np.ascontiguousarray(pi, dtype=np.int64)
        pj = np.ascontiguousarray(pj, dtype=np.int64)
        out = np.empty(pi.size)
        rc = self.lib.oracle_ab_pair_dist(self._d(ra), ra.size, self._d(rb), rb.size, m, self._i(pi), self._i(pj),
                                          pi.size, self._d(out))
        if rc != 0:
            raise RuntimeError("oracle_ab_pair_dist failed")
        return out


def c_oracle() -> _COracle:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_c_oracle(force=True)
        _lib = _COracle(ctypes.CDLL(_LIB))
    return _lib
