"""ace_hash_static (the allocation-free variant of ace_hash) against ace_hash (needs the GPU).

Codes and refined masks are integers, so the bar is bit-exact equality with ace_hash's
output for the same context and rows.  Each case makes two calls in a row through the C ABI,
the second with fewer rows, so the second call runs on whatever the first left in the shared
static scratch; the BF16 and e4m3 cases span several scratch-sized chunks.
"""
import ctypes

import numpy as np
import pytest

import oracle
from ace_inputs import c1_points, heavy_tail_points_torch, low_rank_points_torch, projection_matrix

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _static(ace, X, refined):
    """Codes (and masks) through the raw C entry point."""
    import torch
    n = X.shape[0]
    codes = torch.full((ace.L, n), -1, dtype=torch.int16, device=X.device)
    ref = torch.full((ace.L, n), -1, dtype=torch.int16, device=X.device) if refined else None
    st = torch.cuda.current_stream().cuda_stream
    rc = ace.lib.ace_hash_static(ace.h, ctypes.c_void_p(X.data_ptr()), n, ctypes.c_void_p(codes.data_ptr()),
                                 ctypes.c_void_p(ref.data_ptr()) if refined else None, ctypes.c_void_p(st))
    assert rc == 0, f"ace_hash_static returned {rc}"
    return codes, ref


def _compare(ace, X, refined):
    import torch
    print(dict(n=X.shape[0], d=X.shape[1], L=ace.L, refined=refined), flush=True)
    c_s, r_s = _static(ace, X, refined)
    got = ace.hash(X, want_refined=refined)
    c_h, r_h = got if refined else (got, None)
    torch.cuda.synchronize()
    assert torch.equal(c_s, c_h), "codes differ from ace_hash"
    if refined:
        assert torch.equal(r_s, r_h), "refined masks differ from ace_hash"
    return c_s


@pytest.mark.parametrize("precision,n1,n2", [("fp32", 50_000, 7_331), ("bf16", 40_000, 15_001),
                                             ("fp8", 33_000, 1_000)])
def test_static_equals_hash_two_calls(precision, n1, n2):
    import torch
    from paper_1706_06664_amd import ACE
    if precision == "fp32":
        K, L, d = 15, 50, 120
        X = torch.from_numpy(c1_points(n=n1, seed=11)[0].repeat(4, axis=1)[:, :d].copy()).to("cuda:0")
    elif precision == "bf16":
        K, L, d = 15, 64, 1024
        X, _ = low_rank_points_torch(n1, d, seed=12, device="cuda:0")
    else:
        K, L, d = 16, 100, 512
        X, _ = heavy_tail_points_torch(n1, d, seed=13, device="cuda:0")
    W = projection_matrix(d, K, L, 1706066660)
    ace = ACE(W, K, L, precision=precision, refine=True)
    c1 = _compare(ace, X, refined=True)
    # second call, fewer rows (a ragged count), on what the first left in the scratch
    _compare(ace, X[:n2].contiguous(), refined=False)
    if precision == "fp32":   # the oracle's FP64 signs on a sample of the first call's rows
        idx = np.arange(0, n1, 97)
        co, amb = oracle.hash_codes(X.cpu().numpy()[idx], W, K, L)
        cg = c1.cpu().numpy().view(np.uint16).T[idx]
        assert int(amb.sum()) == 0 and np.array_equal(cg, co)
    ace.close()


def test_static_two_contexts_share_the_scratch():
    """Calls from two contexts in a row use the same array; each still equals its ace_hash."""
    import torch
    from paper_1706_06664_amd import ACE
    X, _ = low_rank_points_torch(20_000, 256, seed=14, device="cuda:0")
    a = ACE(projection_matrix(256, 10, 20, 5), 10, 20, precision="bf16")
    b = ACE(projection_matrix(256, 16, 30, 6), 16, 30, precision="fp32")
    _compare(a, X, refined=True)
    _compare(b, X[:3000].contiguous(), refined=True)
    _compare(a, X[:999].contiguous(), refined=False)
    a.close()
    b.close()


def test_static_rejects_rows_that_do_not_fit():
    """A BF16 context whose 256-row chunk exceeds the 64 MiB array is refused before anything
    is enqueued; empty input is a no-op."""
    import torch
    from paper_1706_06664_amd import ACE
    d = 80_000
    ace = ACE(np.ones((d, 4), np.float32), 4, 1, precision="bf16", max_batch_rows=256)
    X = torch.zeros((4, d), dtype=torch.float32, device="cuda:0")
    codes = torch.empty((1, 4), dtype=torch.int16, device="cuda:0")
    rc = ace.lib.ace_hash_static(ace.h, ctypes.c_void_p(X.data_ptr()), 4, ctypes.c_void_p(codes.data_ptr()), None,
                                 None)
    assert rc == 1
    ace.close()
    small = ACE(projection_matrix(16, 8, 4, 7), 8, 4)
    assert small.lib.ace_hash_static(small.h, None, 0, None, None, None) == 0
    assert small.lib.ace_hash_static(small.h, None, 5, None, None, None) == 1
    small.close()
