"""ACE (arXiv 1706.06664) hot path for AMD Instinct MI355X (gfx950).

SRP hashing on MFMA with a sign-packing epilogue, LDS-privatised count-array
insertion, gather-sum scoring and exact threshold statistics, behind the C ABI
declared in include/ace.h.  `ACE` is a thin ctypes binding over that library.
"""
from .ace import (ACE, AceError, Server, load_library, codes_as_uint16, EXPORTS, LIB_PATH,  # noqa: F401
                  REQUEST_DTYPE, REQ_INSERT, REQ_SCORE, REQ_DELETE, exact_score, mfma_probe)
