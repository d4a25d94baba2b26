"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
symbol the header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "ace.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:ace_status|const char\*)\s+(ace_\w+)\s*\(", text, re.M)))


def _lib():
    from paper_1706_06664_amd import load_library
    return load_library()


def test_exports_every_declared_symbol():
    lib = _lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    from paper_1706_06664_amd import EXPORTS
    assert sorted(EXPORTS) == names


def test_status_strings_and_version():
    lib = _lib()
    assert lib.ace_status_string(0) == b"ACE_OK"
    assert lib.ace_status_string(3) == b"ACE_E_OVERFLOW"
    assert b"gfx950" in lib.ace_version()


@pytest.mark.parametrize("field,value", [("d", 0), ("K", 0), ("K", 17), ("L", 0), ("L", 5000),
                                         ("precision", 7), ("refine", 3), ("refine", -1), ("max_batch_rows", -1),
                                         ("mem_budget", -5), ("device", -1), ("bound_model", 2), ("counter_bits", 1),
                                         ("counter_bits", 8), ("counter_bits", 64)])
def test_create_rejects_bad_config(field, value):
    from paper_1706_06664_amd.ace import Config
    lib = _lib()
    cfg = Config(8, 6, 4, 0, 1, 0, 0, 0, 0, 0)
    setattr(cfg, field, value)
    W = np.zeros((8, 24), np.float32)
    h = ctypes.c_void_p()
    assert lib.ace_create(ctypes.byref(cfg), W.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)) == 1
    assert h.value is None


def test_create_rejects_e4m3_with_generic_bound():
    """The generic error model's premise (2^-23 per addition) does not cover the e4m3
    instruction's in-group loss, so that pair is refused before any device is touched."""
    from paper_1706_06664_amd.ace import Config
    lib = _lib()
    cfg = Config(8, 6, 4, 2, 1, 0, 0, 0, 1, 0)
    W = np.zeros((8, 24), np.float32)
    h = ctypes.c_void_p()
    assert lib.ace_create(ctypes.byref(cfg), W.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)) == 1
    assert h.value is None


def test_null_arguments_rejected():
    lib = _lib()
    from paper_1706_06664_amd.ace import Config
    cfg = Config(8, 6, 4, 0, 1, 0, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    assert lib.ace_create(None, None, ctypes.byref(h)) == 1
    assert lib.ace_create(ctypes.byref(cfg), None, ctypes.byref(h)) == 1
    assert lib.ace_insert(None, None, 10, None) == 1
    assert lib.ace_score(None, None, 10, None, None, None) == 1
    assert lib.ace_destroy(None) == 0


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1706_06664_amd import ace as m
    saved = m._lib
    m._lib = None
    try:
        with pytest.raises(RuntimeError):
            m.load_library(str(tmp_path / "missing.so"))
    finally:
        m._lib = saved


def test_server_calls_reject_null_handles():
    lib = _lib()
    from paper_1706_06664_amd.ace import ServerConfig, ServerStats
    h = ctypes.c_void_p()
    cfg = ServerConfig(2, 0, 16, 0, 0, 0)
    assert lib.ace_server_create(None, ctypes.byref(cfg), ctypes.byref(h)) == 1
    assert h.value is None
    X = np.zeros((4, 8), np.float32)
    t = ctypes.c_uint64()
    assert lib.ace_server_submit(None, 0, X.ctypes.data, 4, None, None, 0, ctypes.byref(t)) == 1
    assert lib.ace_server_wait(None, 0, None) == 1
    assert lib.ace_server_drain(None) == 1
    assert lib.ace_server_replay(None, None, 0, None, 0, 0, None, None, None) == 1
    st = ServerStats()
    assert lib.ace_server_get_stats(None, ctypes.byref(st)) == 1
    assert lib.ace_server_reset_stats(None) == 1
    assert lib.ace_server_destroy(None) == 1


def test_request_record_layout_matches_header():
    from paper_1706_06664_amd import REQUEST_DTYPE
    from paper_1706_06664_amd.ace import ServerConfig, ServerStats
    assert REQUEST_DTYPE.itemsize == 40
    assert [REQUEST_DTYPE.fields[f][1] for f in ("kind", "pad", "n", "row0", "out0", "t_arrival_s")] == \
        [0, 4, 8, 16, 24, 32]
    assert ctypes.sizeof(ServerConfig) == 32
    assert ctypes.sizeof(ServerStats) == 5 * 8 + 7 * 8 + 8 + 8 + 8 + 16 + 16 + 16 + 16 + 8


def test_server_structs_match_header_offsets(tmp_path):
    """The ctypes mirrors of ace_server_stats and ace_server_config against the header as a
    C compiler lays it out (every field's offset, and the size)."""
    import shutil
    import subprocess
    from paper_1706_06664_amd.ace import ServerConfig, ServerStats
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = {"ace_server_stats": ServerStats, "ace_server_config": ServerConfig}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "ace.h"', "int main(void) {"]
    for cname, cls in fields.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-std=c11", "-I", inc, "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in fields.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_exact_score_rejects_bad_arguments():
    lib = _lib()
    S = ctypes.c_double()
    assert lib.ace_exact_score(None, 1, None, 1, 4, 3, ctypes.byref(S), None, 0, None) == 1   # NULL Q
    assert lib.ace_exact_score(None, 0, None, 0, 4, 3, None, None, 0, None) == 0              # m = 0: no-op
    assert lib.ace_exact_score(None, 0, None, 0, 4, 65, None, None, 0, None) == 1             # K > 64
    assert lib.ace_exact_score(None, 0, None, 0, 0, 3, None, None, 0, None) == 1              # d = 0
    assert lib.ace_exact_score(None, -1, None, 0, 4, 3, None, None, 0, None) == 1             # m < 0


def test_create_structured_rejects_bad_arguments():
    from paper_1706_06664_amd.ace import Config
    lib = _lib()
    h = ctypes.c_void_p()
    signs = np.zeros((1, 3, 64), np.uint8)
    cfg = Config(8, 6, 4, 1, 1, 0, 0, 0, 0, 0)          # BF16: structured projections are FP32 only
    assert lib.ace_create_structured(ctypes.byref(cfg), signs.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)) == 1
    cfg = Config(5000, 6, 4, 0, 1, 0, 0, 0, 0, 0)       # dp would exceed 4096
    assert lib.ace_create_structured(ctypes.byref(cfg), signs.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)) == 1
    cfg = Config(8, 6, 4, 0, 1, 0, 0, 0, 0, 0)
    bad = signs.copy()
    bad[0, 1, 3] = 2                                    # a sign byte other than 0 / 1
    assert lib.ace_create_structured(ctypes.byref(cfg), bad.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)) == 1
    assert lib.ace_create_structured(ctypes.byref(cfg), None, ctypes.byref(h)) == 1
    assert h.value is None
