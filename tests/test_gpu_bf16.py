"""Split-BF16 projection mode vs the oracle (needs the GPU).

With refinement on, every bit must equal the FP64 sign outside the oracle's margin,
exactly as in FP32 mode; with refinement off, a raw bit may differ from the FP64
sign only inside the bound the library states for its split-BF16 sums.
"""
import math

import numpy as np
import pytest

import oracle
from ace_inputs import c2_points, gaussian_clusters, projection_matrix
from tests.parity import compare_codes, full_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(m):
    print(m, flush=True)


@pytest.mark.parametrize("n,d,K,L", [
    (1, 5, 1, 1), (127, 33, 15, 3), (129, 120, 15, 50), (300, 7, 16, 4), (1000, 64, 10, 64),
    (777, 1, 4, 100), (515, 130, 16, 13), (2000, 256, 15, 50),
])
def test_bf16_parity_shapes(n, d, K, L):
    X, _ = gaussian_clusters(n, d, 3, 0.05, seed=n + 3 * d)
    W = projection_matrix(d, K, L, 70 + n)
    r = full_parity(X, W, K, L, precision="bf16")
    _say((n, d, K, L, r))


def test_bf16_tiny_chunks_long_rows():
    """Chunks of 16 rows (one row tile each, the last chunk a single row) and rows whose
    padded width is an odd number of 32-wide k-steps (d = 4100: 129 steps)."""
    X, _ = gaussian_clusters(17, 4100, 2, 0.05, seed=4117)
    W = projection_matrix(4100, 16, 20, 4118)
    r = full_parity(X, W, 16, 20, precision="bf16", max_batch_rows=16)
    _say(r)


def test_bf16_connection_log_sample():
    X, _ = c2_points(n=30_000, seed=12)
    W = projection_matrix(120, 15, 50, 1706066642)
    r = full_parity(X, W, 15, 50, precision="bf16")
    _say(r)


def test_bf16_low_rank_sample():
    """1024-dimensional low-rank-plus-noise rows (20,000 of them), K=15, L=64."""
    import torch
    from ace_inputs import low_rank_points_torch
    Xd, _ = low_rank_points_torch(20_000, 1024, seed=3, device="cuda")
    X = Xd.cpu().numpy()
    W = projection_matrix(1024, 15, 64, 1706066643)
    r = full_parity(X, W, 15, 64, precision="bf16")
    _say(r)


def test_bf16_degenerate_rows():
    rng = np.random.default_rng(5)
    d, K, L = 24, 15, 8
    W = projection_matrix(d, K, L, 99)
    zero = np.zeros((200, d), np.float32)
    same = np.repeat(rng.standard_normal((1, d)).astype(np.float32), 3000, axis=0)
    near = []
    for i in range(500):
        y = rng.standard_normal(d)
        c = rng.integers(0, K * L)
        w = W[:, c].astype(np.float64)
        near.append((y - (y @ w) / (w @ w) * w).astype(np.float32))
    X = np.concatenate([zero, same, np.array(near)], axis=0)
    r = full_parity(X, W, K, L, precision="bf16")
    _say(r)
    assert r["bits_refined"] >= 200 * K * L


def _bf16_split(a):
    """Round-to-nearest-even split of float32 values into hi + lo + rest (exact)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, np.float32))
    hi = t.to(torch.bfloat16).to(torch.float32)
    r1 = t - hi
    lo = r1.to(torch.bfloat16).to(torch.float32)
    return hi.numpy().astype(np.float64), lo.numpy().astype(np.float64), (r1 - lo).numpy().astype(np.float64)


def bf16_bound(X, W, model):
    """The split-BF16 refinement bound A cA + B cB + C cC the library states."""
    d = X.shape[1]
    xh, xl, xr = _bf16_split(X)
    wh, wl, wr = _bf16_split(W)
    A, B, C = (np.linalg.norm(v, axis=1) for v in (xh, xl, xr))
    nh, nl, nr, nw = (np.linalg.norm(v, axis=0) for v in (wh, wl, wr, W.astype(np.float64)))
    u = 2.0 ** -23
    I = math.ceil(d / 32)
    hm, hc = (34 * I, 68 * I) if model == "generic" else (4 + 2 * I, 4 + 4 * I)
    cA = nr + hm * u * nh + hc * u * nl + 2 * u * (nh + nl)
    cB = nl + nr + hc * u * nh + 2 * u * nh
    return A[:, None] * cA[None, :] + B[:, None] * cB[None, :] + C[:, None] * nw[None, :]


@pytest.mark.parametrize("model", ["measured", "generic"])
@pytest.mark.parametrize("shape", ["connection_log", "low_rank_1024"])
def test_bf16_raw_signs_stay_inside_stated_bound(model, shape):
    """Refinement off: raw split-BF16 bits may differ from the FP64 signs only where
    |p64| is inside the bound stated for the error model (adversarial rows included)."""
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16
    from tests.parity import adversarial_rows, raw_flip_report
    if shape == "connection_log":
        K, L = 15, 50
        X0, _ = c2_points(n=3000, seed=9)
    else:
        from ace_inputs import low_rank_points_torch
        K, L = 15, 64
        X0 = low_rank_points_torch(3000, 1024, seed=19, device="cuda")[0].cpu().numpy()
    W = projection_matrix(X0.shape[1], K, L, 5)
    X = adversarial_rows(X0, W, 2000, 2000, seed=9)
    ace = ACE(W, K, L, precision="bf16", refine=False, bound=model)
    cg = codes_as_uint16(ace.hash(torch.from_numpy(X).cuda()))
    P, _ = oracle.project(X, W)
    rep = raw_flip_report(cg, P, bf16_bound(X, W, model), K, L)
    _say(rep)
    assert rep["violations"] == 0


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
def test_chunked_conversion(precision):
    """Several chunks (max_batch_rows = 1000, ragged last chunk), each converted and hashed in
    turn.  Hash, insert, score and flags must match the oracle as for one chunk, for aligned
    rows and for an unaligned view (scalar loads)."""
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16
    X, _ = gaussian_clusters(3500, 96, 4, 0.05, seed=21)
    W = projection_matrix(96, 15, 20, 22)
    r = full_parity(X, W, 15, 20, precision=precision, max_batch_rows=1000)
    _say(r)
    big = torch.from_numpy(np.concatenate([np.zeros(1, np.float32), X.ravel()])).cuda()
    Xoff = big[1:].view(3500, 96)
    assert Xoff.data_ptr() % 16 != 0
    ace = ACE(W, 15, 20, precision=precision, max_batch_rows=1000)
    cg = codes_as_uint16(ace.hash(Xoff))
    co, amb = oracle.hash_codes(X, W, 15, 20)
    bad, _, _ = compare_codes(cg, co, amb)
    assert bad == 0
    # the same context again: its buffers are reused across calls
    cg2 = codes_as_uint16(ace.hash(torch.from_numpy(X).cuda()))
    assert np.array_equal(cg, cg2)
    ace.close()
