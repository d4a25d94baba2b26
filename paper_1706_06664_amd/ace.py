"""Thin Python binding of the ACE C ABI (argument marshalling only).

Every step of the path runs in the HIP library `libace_hip.so`; PyTorch is
used only to own device memory and to name streams.  There is no fallback:
if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libace_hip.so")

FP32, BF16, FP8E4M3 = 0, 1, 2
THR_SCORED, THR_CONST, THR_TABLE = 0, 1, 2
_PREC = {"fp32": FP32, "bf16": BF16, "fp8": FP8E4M3, "e4m3": FP8E4M3}
_MODES = {"scored": THR_SCORED, "const": THR_CONST, "table": THR_TABLE}
_BOUND = {"measured": 0, "generic": 1}

STATUS = {0: "ACE_OK", 1: "ACE_E_INVALID", 2: "ACE_E_NOMEM", 3: "ACE_E_OVERFLOW", 4: "ACE_E_EMPTY",
          5: "ACE_E_DEVICE", 6: "ACE_E_STATE", 7: "ACE_E_TIMEOUT"}

# Every symbol include/ace.h declares.
EXPORTS = ["ace_create", "ace_destroy", "ace_reset", "ace_reset_scored", "ace_insert", "ace_delete", "ace_score",
           "ace_threshold", "ace_flag", "ace_hash", "ace_insert_codes", "ace_score_codes", "ace_get_counts",
           "ace_get_table_stats", "ace_get_counters", "ace_set_counts", "ace_status_string", "ace_version",
           "ace_debug_fail_next", "ace_debug_set_capacity", "ace_profile_enable", "ace_get_profile",
           "ace_debug_set_refine_queue", "ace_server_create", "ace_server_submit", "ace_server_wait",
           "ace_server_drain", "ace_server_replay", "ace_server_get_stats", "ace_server_reset_stats",
           "ace_server_destroy", "ace_exact_score", "ace_create_structured", "ace_mfma_probe", "ace_hash_static", "ace_server_wait_for",
           "ace_server_cancel", "ace_get_memory", "ace_server_debug_hold", "ace_threshold_flag"]

REQ_INSERT, REQ_SCORE, REQ_DELETE = 0, 1, 2
SUBMIT_PINNED = 1
_KINDS = {"insert": REQ_INSERT, "score": REQ_SCORE, "delete": REQ_DELETE}

# Layout of ace_request (one record per request of a replayed trace).
REQUEST_DTYPE = np.dtype([("kind", "<i4"), ("pad", "<i4"), ("n", "<i8"), ("row0", "<i8"), ("out0", "<i8"),
                          ("t_arrival_s", "<f8")])


class AceError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}")


class Config(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("K", ctypes.c_int32), ("L", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("refine", ctypes.c_int32), ("device", ctypes.c_int32),
                ("max_batch_rows", ctypes.c_int64), ("mem_budget", ctypes.c_int64),
                ("bound_model", ctypes.c_int32), ("counter_bits", ctypes.c_int32)]


class Thresh(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m_scored", ctypes.c_int64), ("mu", ctypes.c_double),
                ("mu_scored", ctypes.c_double), ("sigma", ctypes.c_double), ("sigma_table", ctypes.c_double),
                ("tau", ctypes.c_double), ("mode", ctypes.c_int32), ("pad", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("hash_ms", ctypes.c_double), ("hash_launches", ctypes.c_int64), ("hash_rows", ctypes.c_int64),
                ("update_ms", ctypes.c_double), ("update_launches", ctypes.c_int64),
                ("score_ms", ctypes.c_double), ("score_launches", ctypes.c_int64),
                ("other_ms", ctypes.c_double), ("other_launches", ctypes.c_int64),
                ("refine_ms", ctypes.c_double), ("refine_launches", ctypes.c_int64),
                ("convert_ms", ctypes.c_double), ("convert_launches", ctypes.c_int64)]


class Counters(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m_scored", ctypes.c_int64), ("sum_T", ctypes.c_int64),
                ("sum_T2_lo", ctypes.c_uint64), ("sum_T2_hi", ctypes.c_uint64), ("bits_hashed", ctypes.c_uint64),
                ("bits_refined", ctypes.c_uint64), ("bits_flipped", ctypes.c_uint64),
                ("bits_in_bound_unrefined", ctypes.c_uint64), ("saturated_increments", ctypes.c_uint64)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("batch_rows", ctypes.c_int32), ("max_rows", ctypes.c_int64),
                ("gather_max_bytes", ctypes.c_int64), ("use_graphs", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_int64), ("inserts", ctypes.c_int64), ("scores", ctypes.c_int64),
                ("rows", ctypes.c_int64), ("insert_rows", ctypes.c_int64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("p99_insert_ms", ctypes.c_double), ("p99_score_ms", ctypes.c_double), ("wall_ms", ctypes.c_double),
                ("batches", ctypes.c_int64), ("mean_batch_requests", ctypes.c_double),
                ("gathered_requests", ctypes.c_int64), ("p50_queue_ms", ctypes.c_double),
                ("p99_queue_ms", ctypes.c_double), ("graph_launches", ctypes.c_int64),
                ("graph_captures", ctypes.c_int64), ("slots", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("deletes", ctypes.c_int64), ("delete_rows", ctypes.c_int64), ("p99_delete_ms", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"ACE HIP library not built: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    P, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sigs = {
        "ace_create": [ctypes.POINTER(Config), P, ctypes.POINTER(P)],
        "ace_destroy": [P],
        "ace_reset": [P, P],
        "ace_reset_scored": [P, P],
        "ace_insert": [P, P, i64, P],
        "ace_delete": [P, P, i64, P],
        "ace_score": [P, P, i64, P, P, P],
        "ace_threshold": [P, i32, f64, P, ctypes.POINTER(Thresh)],
        "ace_flag": [P, P, i64, f64, i32, P, P],
        "ace_threshold_flag": [P, i32, f64, P, i64, P, P, ctypes.POINTER(Thresh)],
        "ace_hash": [P, P, i64, P, P, P],
        "ace_hash_static": [P, P, i64, P, P, P],
        "ace_insert_codes": [P, P, i64, P],
        "ace_score_codes": [P, P, i64, P, P, P],
        "ace_get_counts": [P, P],
        "ace_get_table_stats": [P, P, P],
        "ace_get_counters": [P, ctypes.POINTER(Counters)],
        "ace_set_counts": [P, P, i64],
        "ace_debug_fail_next": [P],
        "ace_debug_set_capacity": [P, i64],
        "ace_profile_enable": [P, i32],
        "ace_debug_set_refine_queue": [P, i64],
        "ace_get_profile": [P, ctypes.POINTER(Profile)],
        "ace_server_create": [P, ctypes.POINTER(ServerConfig), ctypes.POINTER(P)],
        "ace_server_submit": [P, i32, P, i64, P, P, i32, ctypes.POINTER(ctypes.c_uint64)],
        "ace_server_wait": [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)],
        "ace_server_wait_for": [P, ctypes.c_uint64, f64, ctypes.POINTER(ctypes.c_double)],
        "ace_server_cancel": [P, ctypes.c_uint64],
        "ace_server_debug_hold": [P, i32],
        "ace_get_memory": [P, ctypes.POINTER(ctypes.c_int64)],
        "ace_server_drain": [P],
        "ace_server_replay": [P, P, i64, P, i64, i32, P, P, P],
        "ace_server_get_stats": [P, ctypes.POINTER(ServerStats)],
        "ace_server_reset_stats": [P],
        "ace_server_destroy": [P],
        "ace_exact_score": [P, i64, P, i64, i32, i32, P, P, i32, P],
        "ace_create_structured": [ctypes.POINTER(Config), P, ctypes.POINTER(P)],
        "ace_mfma_probe": [i32, P, P, P, P, i32],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.ace_status_string.argtypes = [ctypes.c_int]
    lib.ace_status_string.restype = ctypes.c_char_p
    lib.ace_version.argtypes = []
    lib.ace_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != 0:
        raise AceError(rc, where)


def _stream_ptr(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev_ptr(t, dtype, what: str):
    import torch
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous {dtype} CUDA tensor")
    return t.data_ptr()


class ACE:
    """L count arrays of 2^K counters on one GPU, filled and queried through the C ABI."""

    def __init__(self, W: Optional[np.ndarray], K: int, L: int, precision: str = "fp32", refine: bool = True,
                 device: int = 0, max_batch_rows: int = 0, mem_budget: int = 0, bound: str = "measured",
                 counter_bits: int = 32, signs: Optional[np.ndarray] = None, d: Optional[int] = None):
        """W: dense projections float32 [d][K*L]; or W=None with `signs` (uint8 [B][3][dp])
        and `d` for the structured projection H D3 H D2 H D1."""
        import torch
        self.lib = load_library()
        if W is not None:
            W = np.ascontiguousarray(W, dtype=np.float32)
            if W.ndim != 2 or W.shape[1] != K * L:
                raise ValueError("W must be float32 [d][K*L]")
            d = int(W.shape[0])
        elif signs is None or d is None:
            raise ValueError("give W, or signs and d")
        self.d, self.K, self.L = int(d), int(K), int(L)
        self.device = torch.device("cuda", device)
        rmode = int(refine) if not isinstance(refine, bool) else (1 if refine else 0)
        cfg = Config(self.d, self.K, self.L, _PREC[precision], rmode, device, max_batch_rows,
                     mem_budget, _BOUND[bound], int(counter_bits))
        h = ctypes.c_void_p()
        if W is not None:
            _check(self.lib.ace_create(ctypes.byref(cfg), W.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)),
                   "ace_create")
        else:
            sg = np.ascontiguousarray(signs, dtype=np.uint8)
            _check(self.lib.ace_create_structured(ctypes.byref(cfg), sg.ctypes.data_as(ctypes.c_void_p),
                                                  ctypes.byref(h)), "ace_create_structured")
        self.h = h

    def close(self):
        srv = getattr(self, "_server", None)
        if srv is not None:
            srv.close()
        if getattr(self, "h", None):
            _check(self.lib.ace_destroy(self.h), "ace_destroy")
            self.h = None

    def server(self, slots: int = 4, max_rows: int = 65536, gather_max_bytes: int = 0,
               batch_rows: int = 0, graphs: bool = False) -> "Server":
        """Attach a serving loop (request queue, `slots` batches in flight)."""
        return Server(self, slots, max_rows, gather_max_bytes, batch_rows, graphs)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- stream-ordered calls ---
    def reset(self, stream=None):
        _check(self.lib.ace_reset(self.h, _stream_ptr(stream)), "ace_reset")

    def reset_scored(self, stream=None):
        _check(self.lib.ace_reset_scored(self.h, _stream_ptr(stream)), "ace_reset_scored")

    def _rows(self, X):
        import torch
        if X.dim() != 2 or X.shape[1] != self.d:
            raise ValueError(f"X must be [n][{self.d}]")
        return _dev_ptr(X, torch.float32, "X"), X.shape[0]

    def insert(self, X, stream=None):
        p, n = self._rows(X)
        _check(self.lib.ace_insert(self.h, p, n, _stream_ptr(stream)), "ace_insert")

    def delete(self, X, stream=None):
        p, n = self._rows(X)
        _check(self.lib.ace_delete(self.h, p, n, _stream_ptr(stream)), "ace_delete")

    def score(self, X, s=None, T=None, want_s: bool = True, want_T: bool = True, stream=None):
        import torch
        p, n = self._rows(X)
        if want_s and s is None:
            s = torch.empty(n, dtype=torch.float32, device=X.device)
        if want_T and T is None:
            T = torch.empty(n, dtype=torch.int32, device=X.device)
        _check(self.lib.ace_score(self.h, p, n, _dev_ptr(s, torch.float32, "s"), _dev_ptr(T, torch.int32, "T"),
                                  _stream_ptr(stream)), "ace_score")
        return s, T

    def hash(self, X, want_refined: bool = False, stream=None):
        """Codes as an int16 tensor [L][n] holding the uint16 bit patterns."""
        import torch
        p, n = self._rows(X)
        codes = torch.empty((self.L, n), dtype=torch.int16, device=X.device)
        ref = torch.empty((self.L, n), dtype=torch.int16, device=X.device) if want_refined else None
        _check(self.lib.ace_hash(self.h, p, n, codes.data_ptr(), ref.data_ptr() if ref is not None else None,
                                 _stream_ptr(stream)), "ace_hash")
        return (codes, ref) if want_refined else codes

    def hash_static(self, X, want_refined: bool = False, stream=None):
        """As hash(), through ace_hash_static (no device allocation inside the call)."""
        import torch
        p, n = self._rows(X)
        codes = torch.empty((self.L, n), dtype=torch.int16, device=X.device)
        ref = torch.empty((self.L, n), dtype=torch.int16, device=X.device) if want_refined else None
        _check(self.lib.ace_hash_static(self.h, p, n, codes.data_ptr(), ref.data_ptr() if ref is not None else None,
                                        _stream_ptr(stream)), "ace_hash_static")
        return (codes, ref) if want_refined else codes

    def insert_codes(self, codes, stream=None):
        import torch
        assert codes.dim() == 2 and codes.shape[0] == self.L
        _check(self.lib.ace_insert_codes(self.h, _dev_ptr(codes, torch.int16, "codes"), codes.shape[1],
                                         _stream_ptr(stream)), "ace_insert_codes")

    def score_codes(self, codes, stream=None):
        import torch
        n = codes.shape[1]
        s = torch.empty(n, dtype=torch.float32, device=codes.device)
        T = torch.empty(n, dtype=torch.int32, device=codes.device)
        _check(self.lib.ace_score_codes(self.h, _dev_ptr(codes, torch.int16, "codes"), n, s.data_ptr(),
                                        T.data_ptr(), _stream_ptr(stream)), "ace_score_codes")
        return s, T

    def threshold(self, mode="scored", alpha: float = 1.0, stream=None) -> dict:
        m = _MODES[mode] if isinstance(mode, str) else int(mode)
        out = Thresh()
        _check(self.lib.ace_threshold(self.h, m, float(alpha), _stream_ptr(stream), ctypes.byref(out)),
               "ace_threshold")
        return {f: getattr(out, f) for f, _ in Thresh._fields_ if f != "pad"}

    def threshold_flag(self, T, mode="scored", alpha: float = 1.0, stream=None):
        """threshold() then flag() with its tau, enqueued together (one wait).  Returns
        (flags, threshold dict)."""
        import torch
        m = _MODES[mode] if isinstance(mode, str) else int(mode)
        flags = torch.empty(T.shape[0], dtype=torch.uint8, device=T.device)
        out = Thresh()
        _check(self.lib.ace_threshold_flag(self.h, m, float(alpha), _dev_ptr(T, torch.int32, "T"), T.shape[0],
                                           flags.data_ptr(), _stream_ptr(stream), ctypes.byref(out)),
               "ace_threshold_flag")
        return flags, {f: getattr(out, f) for f, _ in Thresh._fields_ if f != "pad"}

    def flag(self, T, tau: float, mode="scored", stream=None):
        import torch
        m = _MODES[mode] if isinstance(mode, str) else int(mode)
        flags = torch.empty(T.shape[0], dtype=torch.uint8, device=T.device)
        _check(self.lib.ace_flag(self.h, _dev_ptr(T, torch.int32, "T"), T.shape[0], float(tau), m,
                                 flags.data_ptr(), _stream_ptr(stream)), "ace_flag")
        return flags

    # --- synchronising getters ---
    def counts(self) -> np.ndarray:
        out = np.empty((self.L, 1 << self.K), np.int32)
        _check(self.lib.ace_get_counts(self.h, out.ctypes.data_as(ctypes.c_void_p)), "ace_get_counts")
        return out

    def table_stats(self):
        S2 = np.empty(self.L, np.int64)
        S3 = np.empty((self.L, 2), np.uint64)
        _check(self.lib.ace_get_table_stats(self.h, S2.ctypes.data_as(ctypes.c_void_p),
                                            S3.ctypes.data_as(ctypes.c_void_p)), "ace_get_table_stats")
        return S2, S3

    def counters(self) -> dict:
        out = Counters()
        _check(self.lib.ace_get_counters(self.h, ctypes.byref(out)), "ace_get_counters")
        return {f: getattr(out, f) for f, _ in Counters._fields_}

    def memory(self) -> int:
        """Device bytes the context (and an attached server) holds."""
        out = ctypes.c_int64()
        _check(self.lib.ace_get_memory(self.h, ctypes.byref(out)), "ace_get_memory")
        return out.value

    def profile_enable(self, on: bool = True):
        _check(self.lib.ace_profile_enable(self.h, 1 if on else 0), "ace_profile_enable")

    def profile(self) -> dict:
        out = Profile()
        _check(self.lib.ace_get_profile(self.h, ctypes.byref(out)), "ace_get_profile")
        return {f: getattr(out, f) for f, _ in Profile._fields_}

    def set_counts(self, counts: np.ndarray, n: int):
        counts = np.ascontiguousarray(counts, np.int32)
        _check(self.lib.ace_set_counts(self.h, counts.ctypes.data_as(ctypes.c_void_p), int(n)), "ace_set_counts")


def exact_score(Q, X, K: int, want_S2: bool = False, stream=None):
    """S(q, D) = sum_x p(q, x)^K for every row q of Q against the rows of X (Eq. thescore),
    on the GPU.  Q, X: contiguous float32 CUDA tensors [m][d], [n][d].  Returns FP64 S
    (and sum p^{2K} when want_S2)."""
    import torch
    lib = load_library()
    if Q.dim() != 2 or X.dim() != 2 or Q.shape[1] != X.shape[1]:
        raise ValueError("Q and X must be [m][d] and [n][d]")
    m, d = Q.shape
    S = torch.empty(m, dtype=torch.float64, device=Q.device)
    S2 = torch.empty(m, dtype=torch.float64, device=Q.device) if want_S2 else None
    _check(lib.ace_exact_score(_dev_ptr(Q, torch.float32, "Q"), m, _dev_ptr(X, torch.float32, "X"), X.shape[0], d,
                               int(K), S.data_ptr(), S2.data_ptr() if S2 is not None else None,
                               Q.device.index or 0, _stream_ptr(stream)), "ace_exact_score")
    return (S, S2) if want_S2 else S


_PROBE = {"fp32": (0, np.float32, (16, 4), (4, 16)), "bf16": (1, np.uint16, (16, 32), (32, 16)),
          "e4m3": (2, np.uint8, (16, 128), (128, 16))}


def mfma_probe(kind: str, A: np.ndarray, B: np.ndarray, C: np.ndarray, device: int = 0) -> np.ndarray:
    """One matrix instruction D = C + A B on the GPU (ace_mfma_probe): kind "fp32" (A, B
    float32 [16][4], [4][16]), "bf16" (uint16 bf16 bits [16][32], [32][16]) or "e4m3"
    (uint8 codes [16][128], [128][16]); C float32 [16][16].  Returns D float32 [16][16]."""
    k, dt, sa, sb = _PROBE[kind]
    A = np.ascontiguousarray(A, dt)
    B = np.ascontiguousarray(B, dt)
    C = np.ascontiguousarray(C, np.float32)
    if A.shape != sa or B.shape != sb or C.shape != (16, 16):
        raise ValueError(f"{kind}: A {sa}, B {sb}, C (16, 16) expected")
    D = np.empty((16, 16), np.float32)
    _check(load_library().ace_mfma_probe(k, A.ctypes.data, B.ctypes.data, C.ctypes.data, D.ctypes.data, device),
           "ace_mfma_probe")
    return D


def _host_ptr(a, dtype, what: str):
    """Address of a host buffer: a C-contiguous numpy array or a CPU torch tensor."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        if a.dtype != dtype or not a.flags["C_CONTIGUOUS"]:
            raise ValueError(f"{what} must be a C-contiguous {np.dtype(dtype)} array")
        return a.ctypes.data
    if a.device.type != "cpu" or not a.is_contiguous():
        raise ValueError(f"{what} must be a contiguous CPU tensor")
    return a.data_ptr()


class Server:
    """Serving loop of one ACE context: requests are admitted in order onto `slots`
    streams; a score sees exactly the inserts and deletes admitted before it.  Kinds:
    "insert", "score" and "delete" (rows inserted earlier leaving a sliding window)."""

    def __init__(self, ace: ACE, slots: int = 4, max_rows: int = 65536, gather_max_bytes: int = 0,
                 batch_rows: int = 0, graphs: bool = False):
        if getattr(ace, "_server", None) is not None:
            raise AceError(6, "ace_server_create")
        self.ace, self.lib, self.d = ace, ace.lib, ace.d
        cfg = ServerConfig(int(slots), int(batch_rows), int(max_rows), int(gather_max_bytes), 1 if graphs else 0, 0)
        h = ctypes.c_void_p()
        _check(self.lib.ace_server_create(ace.h, ctypes.byref(cfg), ctypes.byref(h)), "ace_server_create")
        self.h = h
        self._keep = {}
        ace._server = self

    def close(self):
        if getattr(self, "h", None):
            _check(self.lib.ace_server_destroy(self.h), "ace_server_destroy")
            self.h = None
            self._keep.clear()
            self.ace._server = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, kind, X, s=None, T=None, pinned: bool = False) -> int:
        """Queue one request.  X: host float32 [n][d].  For scores, s (float32 [n]) and T
        (uint32 [n]) are host buffers filled when the request completes.  X, s and T are
        held until wait/drain.  pinned=True: X is pinned memory, copied to the device directly."""
        k = _KINDS[kind] if isinstance(kind, str) else int(kind)
        n = int(X.shape[0])
        if X.shape[1] != self.d:
            raise ValueError(f"X must be [n][{self.d}]")
        t = ctypes.c_uint64()
        _check(self.lib.ace_server_submit(self.h, k, _host_ptr(X, np.float32, "X"), n,
                                          _host_ptr(s, np.float32, "s"), _host_ptr(T, np.uint32, "T"),
                                          SUBMIT_PINNED if pinned else 0, ctypes.byref(t)), "ace_server_submit")
        self._keep[t.value] = (X, s, T)
        return t.value

    def wait(self, ticket: int, timeout_ms: Optional[float] = None) -> float:
        """Latency of the request in ms.  With timeout_ms, raises AceError (ACE_E_TIMEOUT) if
        it has not completed in time (it stays admitted)."""
        lat = ctypes.c_double()
        if timeout_ms is None:
            _check(self.lib.ace_server_wait(self.h, int(ticket), ctypes.byref(lat)), "ace_server_wait")
        else:
            _check(self.lib.ace_server_wait_for(self.h, int(ticket), float(timeout_ms), ctypes.byref(lat)),
                   "ace_server_wait_for")
        self._keep.pop(int(ticket), None)
        return lat.value

    def hold(self, on: bool = True):
        """Test hook: stop (or resume) forming new batches."""
        _check(self.lib.ace_server_debug_hold(self.h, 1 if on else 0), "ace_server_debug_hold")

    def cancel(self, ticket: int) -> bool:
        """Withdraw a request still in the queue: True if withdrawn, False if it already
        runs or ran (it then completes as usual), or if it is an insert whose rows the
        deletes admitted since still need."""
        rc = self.lib.ace_server_cancel(self.h, int(ticket))
        if rc == 6:
            return False
        _check(rc, "ace_server_cancel")
        self._keep.pop(int(ticket), None)
        return True

    def drain(self):
        _check(self.lib.ace_server_drain(self.h), "ace_server_drain")
        self._keep.clear()

    def replay(self, reqs: np.ndarray, pool, s_out=None, T_out=None, pinned: bool = False) -> np.ndarray:
        """Replay a trace (REQUEST_DTYPE records) against host rows `pool` [rows][d];
        returns each request's latency in ms."""
        reqs = np.ascontiguousarray(reqs, REQUEST_DTYPE)
        lat = np.empty(len(reqs), np.float64)
        _check(self.lib.ace_server_replay(self.h, reqs.ctypes.data, len(reqs), _host_ptr(pool, np.float32, "pool"),
                                          int(pool.shape[0]), SUBMIT_PINNED if pinned else 0,
                                          _host_ptr(s_out, np.float32, "s_out"), _host_ptr(T_out, np.uint32, "T_out"),
                                          lat.ctypes.data), "ace_server_replay")
        return lat

    def stats(self) -> dict:
        out = ServerStats()
        _check(self.lib.ace_server_get_stats(self.h, ctypes.byref(out)), "ace_server_get_stats")
        return {f: getattr(out, f) for f, _ in ServerStats._fields_}

    def reset_stats(self):
        _check(self.lib.ace_server_reset_stats(self.h), "ace_server_reset_stats")


def codes_as_uint16(codes_t) -> np.ndarray:
    """Device int16 codes [L][n] -> host uint16 [n][L] (the row-major layout the oracle uses)."""
    return codes_t.cpu().numpy().view(np.uint16).T.copy()
