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


def test_bf16_raw_signs_stay_inside_stated_bound():
    """Refinement off: raw split-BF16 bits may differ from the FP64 signs only where
    |p64| is inside the bound A cA + B cB + C cC stated for the kernel."""
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16
    rng = np.random.default_rng(9)
    K, L = 15, 50
    X, _ = c2_points(n=3000, seed=9)
    d = X.shape[1]
    W = projection_matrix(d, K, L, 5)
    near = []
    for i in range(3000):
        y = X[rng.integers(0, 3000)].astype(np.float64)
        c = rng.integers(0, K * L)
        w = W[:, c].astype(np.float64)
        near.append((y - (y @ w) / (w @ w) * w).astype(np.float32))
    X = np.concatenate([X, np.array(near)], axis=0)
    ace = ACE(W, K, L, precision="bf16", refine=False)
    cg = codes_as_uint16(ace.hash(torch.from_numpy(X).cuda()))
    P, _ = oracle.project(X, W)
    xh, xl, xr = _bf16_split(X)
    wh, wl, wr = _bf16_split(W)
    A, B, C = (np.linalg.norm(v, axis=1) for v in (xh, xl, xr))
    nh, nl, nr, nw = (np.linalg.norm(v, axis=0) for v in (wh, wl, wr, W.astype(np.float64)))
    u = 2.0 ** -23
    I = math.ceil(d / 32)
    cA = nr + 34 * I * u * nh + 68 * I * u * nl + 2 * u * (nh + nl)
    cB = nl + nr + 68 * I * u * nh + 2 * u * nh
    bound = A[:, None] * cA[None, :] + B[:, None] * cB[None, :] + C[:, None] * nw[None, :]
    bits_ref = P > 0
    flips = viol = 0
    worst = 0.0
    for j in range(L):
        for k in range(K):
            c = j * K + k
            gbit = ((cg[:, j] >> k) & 1).astype(bool)
            diff = gbit != bits_ref[:, c]
            flips += int(diff.sum())
            if diff.any():
                ratio = np.abs(P[diff, c]) / bound[diff, c]
                worst = max(worst, float(ratio.max()))
                viol += int((ratio > 1).sum())
    _say({"raw_flips": flips, "raw_flip_rate": flips / (X.shape[0] * K * L), "worst_ratio": worst})
    assert viol == 0
