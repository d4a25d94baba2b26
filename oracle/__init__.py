"""ACE oracle (test infrastructure only).

A plain CPU implementation of the ACE estimator (arXiv 1706.06664, Alg. 1,
Sec. 2.1, 3.2, 3.4.1, 5.3) in FP64 and exact integers, wrapped with ctypes.
Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import it; the library never does.  It shares no code with the HIP path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libace_oracle.so")
_lib = None

MODE_SCORED, MODE_CONST, MODE_TABLE = 0, 1, 2


class _Thresh(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m_scored", ctypes.c_int64),
                ("mu", ctypes.c_double), ("mu_scored", ctypes.c_double),
                ("sigma", ctypes.c_double), ("sigma_table", ctypes.c_double),
                ("tau", ctypes.c_double), ("mode", ctypes.c_int32), ("pad", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.ace_oracle_project.argtypes = [P, i64, i32, P, i32, P, P]
    lib.ace_oracle_hash.argtypes = [P, i64, i32, P, i32, i32, P, P]
    lib.ace_oracle_insert.argtypes = [P, i64, i32, i32, P, P, P, P]
    lib.ace_oracle_insert_capped.argtypes = [P, i64, i32, i32, i64, P, P, P, P]
    lib.ace_oracle_insert_capped.restype = i64
    lib.ace_oracle_delete.argtypes = [P, i64, i32, i32, P, P, P, P]
    lib.ace_oracle_delete.restype = i64
    lib.ace_oracle_score.argtypes = [P, i64, i32, i32, P, P]
    lib.ace_oracle_moments.argtypes = [P, i64, P, P, P]
    lib.ace_oracle_threshold.argtypes = [i64, i32, P, P, i64, i64, P, i32, f64, ctypes.POINTER(_Thresh)]
    lib.ace_oracle_threshold.restype = ctypes.c_int
    lib.ace_oracle_flags.argtypes = [P, i64, i32, f64, i32, P]
    lib.ace_oracle_exact_score.argtypes = [P, i64, P, i64, i32, i32, P]
    _lib = lib
    return lib


class using_library:
    """Temporarily load the oracle from another build (used by the mutation tests)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib, _LIB_PATH
        self._saved = (_lib, _LIB_PATH)
        _lib, _LIB_PATH = None, self.path
        return self

    def __exit__(self, *exc):
        global _lib, _LIB_PATH
        _lib, _LIB_PATH = self._saved
        return False


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def project(X, W):
    """FP64 projections P = X W and their rounding margins M (Sec. 2.1)."""
    X, W = _f32(X), _f32(W)
    n, d = X.shape
    ncols = W.shape[1]
    assert W.shape[0] == d
    P = np.empty((n, ncols), np.float64)
    M = np.empty((n, ncols), np.float64)
    _load().ace_oracle_project(_ptr(X), n, d, _ptr(W), ncols, _ptr(P), _ptr(M))
    return P, M


def hash_codes(X, W, K: int, L: int):
    """Codes [n][L] (uint16) and ambiguous-bit masks [n][L] (Sec. 2.1, 3.2)."""
    X, W = _f32(X), _f32(W)
    n, d = X.shape
    assert W.shape == (d, K * L)
    codes = np.empty((n, L), np.uint16)
    amb = np.empty((n, L), np.uint16)
    _load().ace_oracle_hash(_ptr(X), n, d, _ptr(W), K, L, _ptr(codes), _ptr(amb))
    return codes, amb


def exact_score(Q, X, K: int):
    """S(q, D) = sum_i p(q, x_i)^K (Sec. 3, Eq. thescore)."""
    Q, X = _f32(Q), _f32(X)
    S = np.empty(Q.shape[0], np.float64)
    _load().ace_oracle_exact_score(_ptr(Q), Q.shape[0], _ptr(X), X.shape[0], X.shape[1], K, _ptr(S))
    return S


class Sketch:
    """L count arrays of 2^K entries with the running statistics (Alg. 1, Sec. 3.4.1)."""

    def __init__(self, K: int, L: int, cap: int | None = None):
        """cap: saturating counters that stop at `cap` (Sec. 3.4's short counters use 65535
        for 16 bits); None: unbounded counts."""
        self.K, self.L, self.cap = K, L, cap
        self.dropped = 0
        self.counts = np.zeros((L, 1 << K), np.int64)
        self.S2 = np.zeros(L, np.int64)
        self.S3 = np.zeros((L, 2), np.uint64)
        self.n = np.zeros(1, np.int64)
        self.m = np.zeros(1, np.int64)
        self.sumT = np.zeros(1, np.int64)
        self.sumT2 = np.zeros(2, np.uint64)

    def insert_codes(self, codes):
        codes = np.ascontiguousarray(codes, np.uint16)
        assert codes.ndim == 2 and codes.shape[1] == self.L
        if self.cap is None:
            _load().ace_oracle_insert(_ptr(codes), codes.shape[0], self.K, self.L, _ptr(self.counts),
                                      _ptr(self.S2), _ptr(self.S3), _ptr(self.n))
        else:
            self.dropped += int(_load().ace_oracle_insert_capped(_ptr(codes), codes.shape[0], self.K, self.L,
                                                                 int(self.cap), _ptr(self.counts), _ptr(self.S2),
                                                                 _ptr(self.S3), _ptr(self.n)))

    def delete_codes(self, codes) -> int:
        codes = np.ascontiguousarray(codes, np.uint16)
        return int(_load().ace_oracle_delete(_ptr(codes), codes.shape[0], self.K, self.L,
                                             _ptr(self.counts), _ptr(self.S2), _ptr(self.S3), _ptr(self.n)))

    def score_codes(self, codes, accumulate: bool = True):
        """T per row (int64); the score is T / L.  Adds the rows to the scored set."""
        codes = np.ascontiguousarray(codes, np.uint16)
        T = np.empty(codes.shape[0], np.int64)
        _load().ace_oracle_score(_ptr(codes), codes.shape[0], self.K, self.L, _ptr(self.counts), _ptr(T))
        if accumulate:
            _load().ace_oracle_moments(_ptr(T), T.shape[0], _ptr(self.m), _ptr(self.sumT), _ptr(self.sumT2))
        return T

    def reset_scored(self):
        self.m[:] = 0
        self.sumT[:] = 0
        self.sumT2[:] = 0

    def threshold(self, mode: int = MODE_SCORED, alpha: float = 1.0):
        out = _Thresh()
        rc = _load().ace_oracle_threshold(int(self.n[0]), self.L, _ptr(self.S2), _ptr(self.S3),
                                          int(self.m[0]), int(self.sumT[0]), _ptr(self.sumT2),
                                          mode, alpha, ctypes.byref(out))
        return rc, {f: getattr(out, f) for f, _ in _Thresh._fields_ if f != "pad"}

    def flags(self, T, tau: float, mode: int = MODE_SCORED):
        T = np.ascontiguousarray(T, np.int64)
        f = np.empty(T.shape[0], np.uint8)
        _load().ace_oracle_flags(_ptr(T), T.shape[0], self.L, tau, mode, _ptr(f))
        return f

    @property
    def s3_int(self):
        return [int(lo) | (int(hi) << 64) for lo, hi in self.S3]

    @property
    def sumT2_int(self):
        return int(self.sumT2[0]) | (int(self.sumT2[1]) << 64)
