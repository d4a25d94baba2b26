"""Structured projections (H D3 H D2 H D1, fast Walsh-Hadamard on the GPU) vs the oracle's
dense equivalent (needs the GPU).

With refinement on, every code bit must equal the FP64 sign of sum_t x_t M[c][t] outside
the oracle's margin; with refinement off, a raw bit may differ only inside the bound the
library states for its FP32 transforms: g dp^1.5 |x|_2 (3 + 4g), g = m u (1 + 2u)^m.
"""
import math

import numpy as np
import pytest

import oracle
from ace_inputs import c2_points, gaussian_clusters, heavy_tail_points_torch, structured_signs
from oracle.structured import structured_matrix
from tests.parity import compare_codes, full_parity, raw_flip_report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(m):
    print(m, flush=True)


def struct_bound(X, dp):
    u, m = 2.0 ** -24, math.log2(dp)
    g = m * u * (1 + 2 * u) ** m
    return g * dp ** 1.5 * (3 + 4 * g) * np.linalg.norm(X.astype(np.float64), axis=1) + 2.0 ** -90


@pytest.mark.parametrize("n,d,K,L", [(1, 1, 1, 1), (300, 7, 10, 20), (129, 64, 16, 4), (1000, 120, 15, 50),
                                     (777, 1000, 16, 13), (50, 2048, 16, 300), (400, 4096, 16, 100)])
def test_structured_parity_shapes(n, d, K, L):
    X, _ = gaussian_clusters(n, d, 3, 0.05, seed=n + d)
    signs, dp = structured_signs(d, K, L, 50 + d)
    W = structured_matrix(signs, d, K, L)
    r = full_parity(X, W, K, L, signs=signs)
    _say((n, d, K, L, dp, r))


def test_structured_connection_log_sample():
    X, _ = c2_points(n=20_000, seed=15)
    signs, _ = structured_signs(120, 15, 50, 1706066646)
    W = structured_matrix(signs, 120, 15, 50)
    _say(full_parity(X, W, 15, 50, signs=signs))


def test_structured_degenerate_rows():
    rng = np.random.default_rng(4)
    d, K, L = 100, 15, 10
    signs, _ = structured_signs(d, K, L, 9)
    W = structured_matrix(signs, d, K, L)
    base = rng.standard_normal((50, d)).astype(np.float32)
    X = np.concatenate([np.zeros((20, d), np.float32), np.repeat(base[:1], 100, axis=0), base * 1e30,
                        base * 1e-30, base]).astype(np.float32)
    r = full_parity(X, W, K, L, signs=signs)
    _say(r)
    assert r["bits_refined"] >= 20 * K * L     # zero rows: every bit is inside the bound


def test_structured_queue_full_path():
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16
    X, _ = gaussian_clusters(2000, 256, 3, 0.05, seed=2)
    X[:200] = 0.0
    signs, _ = structured_signs(256, 16, 20, 3)
    W = structured_matrix(signs, 256, 16, 20)
    ace = ACE(None, 16, 20, signs=signs, d=256)
    ace.lib.ace_debug_set_refine_queue(ace.h, 100)
    cg = codes_as_uint16(ace.hash(torch.from_numpy(X).cuda()))
    co, amb = oracle.hash_codes(X, W, 16, 20)
    bad, _, _ = compare_codes(cg, co, amb)
    assert bad == 0
    assert ace.counters()["bits_refined"] >= 200 * 16 * 20 - 100
    ace.close()


@pytest.mark.parametrize("d,K,L", [(120, 15, 50), (4096, 16, 100)])
def test_structured_raw_signs_inside_bound(d, K, L):
    """Refinement off, rows built near the sign boundary of chosen outputs: every raw bit
    that differs from the FP64 sign lies inside the stated bound."""
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16
    signs, dp = structured_signs(d, K, L, 21)
    W = structured_matrix(signs, d, K, L).astype(np.float64)
    if d == 4096:
        X0 = heavy_tail_points_torch(1500, d, seed=6, device="cuda")[0].cpu().numpy()
    else:
        X0, _ = c2_points(n=1500, seed=16)
    rng = np.random.default_rng(8)
    near = []
    for _ in range(1500):
        y = X0[rng.integers(0, X0.shape[0])].astype(np.float64)
        w = W[:, rng.integers(0, K * L)]
        near.append(y - (y @ w) / (w @ w) * w)
    X = np.concatenate([X0, np.array(near, np.float32)]).astype(np.float32)
    ace = ACE(None, K, L, signs=signs, d=d, refine=False)
    cg = codes_as_uint16(ace.hash(torch.from_numpy(X).cuda()))
    P, _ = oracle.project(X, W.astype(np.float32))
    bound = np.repeat(struct_bound(X, dp)[:, None], K * L, axis=1)
    rep = raw_flip_report(cg, P, bound, K, L)
    _say(rep)
    assert rep["violations"] == 0
    ace.close()
