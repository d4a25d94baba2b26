"""FP8 (e4m3, power-of-two row/column scales) projection mode (needs the GPU).

Refinement on: every bit equals the FP64 sign outside the oracle's margin.
Refinement off: a raw bit may differ from the FP64 sign only inside the bound the
library states for e4m3 (quantisation + measured in-group accumulation loss).
Count-only mode: the bits it counts inside the bound cover every raw flip.
"""
import math

import numpy as np
import pytest

import oracle
from ace_inputs import c2_points, gaussian_clusters, projection_matrix
from tests.parity import adversarial_rows, compare_codes, full_parity, raw_flip_report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(m):
    print(m, flush=True)


def _pow2_scale(m):
    """Smallest power of two s with m / s <= 448 (1 for m == 0)."""
    e = np.zeros_like(m, dtype=np.int64)
    nz = m > 0
    e[nz] = np.floor(np.log2(m[nz] / 448.0)).astype(np.int64)
    for _ in range(3):
        e = np.where(np.ldexp(m, -e) > 448.0, e + 1, e)
    return e


def _e4m3(v):
    import torch
    return torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(torch.float8_e4m3fn).to(torch.float32).numpy()


def fp8_bound(X, W):
    """Bound in scaled units and the scales: (bound [n][ncols], row exponents, column exponents)."""
    d = X.shape[1]
    ex = _pow2_scale(np.abs(X).max(axis=1).astype(np.float64))
    ew = _pow2_scale(np.abs(W).max(axis=0).astype(np.float64))
    xs = np.ldexp(X.astype(np.float64), -ex[:, None]).astype(np.float32)
    ws = np.ldexp(W.astype(np.float64), -ew[None, :]).astype(np.float32)
    xq, wq = _e4m3(xs), _e4m3(ws)
    A = np.linalg.norm(xq.astype(np.float64), axis=1)
    B = np.linalg.norm((xs - xq).astype(np.float64), axis=1)
    nq = np.linalg.norm(wq.astype(np.float64), axis=0)
    nd = np.linalg.norm((ws - wq).astype(np.float64), axis=0)
    I = math.ceil(d / 128)
    hacc = 2.0 ** -9 + 8 * I * 2.0 ** -24
    cA = nd + hacc * nq
    cB = nq + nd
    return A[:, None] * cA[None, :] + B[:, None] * cB[None, :], ex, ew


@pytest.mark.parametrize("n,d,K,L", [(1, 5, 1, 1), (127, 33, 15, 3), (300, 7, 16, 4), (515, 130, 16, 13),
                                     (1000, 64, 10, 20)])
def test_fp8_parity_shapes(n, d, K, L):
    X, _ = gaussian_clusters(n, d, 3, 0.05, seed=n + 5 * d)
    W = projection_matrix(d, K, L, 90 + n)
    r = full_parity(X, W, K, L, precision="fp8")
    _say((n, d, K, L, r))


def test_fp8_tiny_chunks_long_rows():
    """Chunks of 16 rows (the last a single row) and rows of 33 k-steps of 128 (d = 4100)."""
    X, _ = gaussian_clusters(17, 4100, 2, 0.05, seed=4127)
    W = projection_matrix(4100, 16, 20, 4128)
    r = full_parity(X, W, 16, 20, precision="fp8", max_batch_rows=16)
    _say(r)


@pytest.mark.parametrize("shape", ["connection_log", "heavy_tail_512"])
def test_fp8_raw_signs_stay_inside_stated_bound(shape):
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16
    if shape == "connection_log":
        K, L = 15, 50
        X0, _ = c2_points(n=2000, seed=10)
    else:
        from ace_inputs import heavy_tail_points_torch
        K, L = 16, 20
        X0 = heavy_tail_points_torch(2000, 512, seed=4, device="cuda")[0].cpu().numpy()
    W = projection_matrix(X0.shape[1], K, L, 6)
    X = adversarial_rows(X0, W, 1000, 1000, seed=10)
    # rows whose largest value is below 2^-119: their scale 2^-e is beyond FP32 (e < -127),
    # so the conversion must scale each value in one exact step
    rng = np.random.default_rng(12)
    tiny = (np.sign(rng.standard_normal((20, X.shape[1]))) * 2.0 ** -123 *
            (1 + rng.random((20, X.shape[1])))).astype(np.float32)
    X = np.concatenate([X, tiny], axis=0)
    ace = ACE(W, K, L, precision="fp8", refine=False)
    cg = codes_as_uint16(ace.hash(torch.from_numpy(X).cuda()))
    P, _ = oracle.project(X, W)
    bnd, ex, ew = fp8_bound(X, W)
    Ps = np.ldexp(P, -(ex[:, None] + ew[None, :]))   # FP64 projection in scaled units
    rep = raw_flip_report(cg, Ps, bnd, K, L)
    _say(rep)
    assert rep["violations"] == 0
    assert rep["raw_flips"] > 0


def test_fp8_count_mode_covers_flips():
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16
    K, L = 15, 50
    X, _ = c2_points(n=5000, seed=11)
    W = projection_matrix(X.shape[1], K, L, 7)
    a = ACE(W, K, L, precision="fp8", refine=2)
    cg = codes_as_uint16(a.hash(torch.from_numpy(X).cuda()))
    cnt = a.counters()
    co, amb = oracle.hash_codes(X, W, K, L)
    _, _, ndiff = compare_codes(cg, co, amb)
    _say({"in_bound": cnt["bits_in_bound_unrefined"], "raw_flips": ndiff, "bits": cnt["bits_hashed"]})
    assert cnt["bits_in_bound_unrefined"] >= ndiff > 0
    assert cnt["bits_refined"] == 0
