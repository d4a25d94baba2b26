"""Exact S(q, D) of Eq. thescore on the GPU vs the oracle (needs the GPU).

Tolerance.  Both sides form c = q.x / (|q||x|) from FP64 sums of exact products, in
different orders (the GPU multiplies by inverse norms, the oracle divides by their
product), so their c differ by at most delta = 4 gamma_d + 16u (u = 2^-53).  arccos
amplifies that near c = +-1: |d theta| <= delta / sqrt(1 - (|c| + 2 delta)^2) away from
the ends and <= (pi / sqrt 2) sqrt(delta) everywhere, and |d p^K| <= K |d theta| / pi.  The
per-query tolerance is the sum of these per-point bounds (c taken from an FP64 evaluation
here) plus 64u per point for the arccos / power implementations and 4 n u S for the order
of the additions.
"""
import math

import numpy as np
import pytest

import oracle
from ace_inputs import c2_points, gaussian_clusters

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(m):
    print(m, flush=True)


def tolerance(Q, X, K, S_ref):
    d = Q.shape[1]
    gam = d * U / (1 - d * U)
    delta = 4 * gam + 16 * U
    q = Q.astype(np.float64)
    x = X.astype(np.float64)
    nq = np.linalg.norm(q, axis=1)
    nx = np.linalg.norm(x, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        C = (q @ x.T) / np.outer(nq, nx)
    C = np.nan_to_num(C, nan=0.0)
    zero = (nq[:, None] == 0) | (nx[None, :] == 0)
    a = np.minimum(np.abs(C) + 2 * delta, 1.0)
    with np.errstate(divide="ignore"):
        far = delta / np.sqrt(np.maximum(1.0 - a * a, 0.0))
    dth = np.minimum(far, math.pi / math.sqrt(2.0) * math.sqrt(delta))
    dth[zero] = 0.0
    per = K * dth / math.pi + 64 * U
    return per.sum(axis=1) + 4 * X.shape[0] * U * np.abs(S_ref)


def _check(Q, X, K):
    import torch
    from paper_1706_06664_amd import exact_score
    S_o = oracle.exact_score(Q, X, K)
    S2_o = oracle.exact_score(Q, X, 2 * K)
    S, S2 = exact_score(torch.from_numpy(Q).cuda(), torch.from_numpy(X).cuda(), K, want_S2=True)
    S, S2 = S.cpu().numpy(), S2.cpu().numpy()
    tol = tolerance(Q, X, K, S_o)
    tol2 = tolerance(Q, X, 2 * K, S2_o)
    err = np.abs(S - S_o)
    assert (err <= tol).all(), (err.max(), tol[np.argmax(err / tol)])
    assert (np.abs(S2 - S2_o) <= tol2).all()
    return {"m": Q.shape[0], "n": X.shape[0], "d": Q.shape[1], "K": K, "max_err": float(err.max()),
            "max_err_over_tol": float((err / tol).max()), "S_mean": float(S_o.mean())}


@pytest.mark.parametrize("m,n,d,K", [(1, 1, 1, 1), (37, 529, 33, 15), (130, 1000, 120, 15), (64, 777, 7, 3),
                                     (200, 300, 256, 16), (5, 2000, 4, 64)])
def test_exact_score_shapes(m, n, d, K):
    X, _ = gaussian_clusters(n, d, 3, 0.05, seed=m + d)
    Q, _ = gaussian_clusters(m, d, 3, 0.05, seed=m + d + 1)
    _say(_check(Q, X, K))


def test_exact_score_degenerate_rows():
    """Zero rows on either side, queries equal to points (c = 1) and their negations (c = -1)."""
    rng = np.random.default_rng(3)
    d, K = 24, 15
    X = rng.standard_normal((300, d)).astype(np.float32)
    X[:7] = 0.0
    Q = np.concatenate([np.zeros((3, d), np.float32), X[10:40], -X[40:60], 2.0 * X[60:70],
                        rng.standard_normal((20, d)).astype(np.float32)])
    r = _check(Q, X, K)
    _say(r)
    # a zero query: 7 zero points give p = 1, the rest p = 1/2
    from paper_1706_06664_amd import exact_score
    import torch
    S = exact_score(torch.from_numpy(Q[:1]).cuda(), torch.from_numpy(X).cuda(), K).cpu().numpy()
    assert S[0] == 7 + 293 * 0.5 ** K


def test_exact_score_connection_log_sample():
    X, _ = c2_points(n=40_000, seed=21)
    Q = X[::157][:256].copy()
    _say(_check(Q, X, 15))


def test_theorem1_ace_mean_matches_exact_score():
    """Theorem 1: each table's count at the query's bucket has mean S(q, D).  With many
    tables the ACE score T / L must lie within 5 standard errors of the exact S, where the
    per-table variance is at most n S (a count is at most n)."""
    import torch
    from ace_inputs import projection_matrix
    from paper_1706_06664_amd import ACE, exact_score
    n, d, K, L = 40, 3, 3, 4096
    X, _ = gaussian_clusters(n, d, 2, 0.1, seed=8)
    Q, _ = gaussian_clusters(30, d, 2, 0.1, seed=9)
    W = projection_matrix(d, K, L, 123)
    ace = ACE(W, K, L)
    ace.insert(torch.from_numpy(X).cuda())
    s, _ = ace.score(torch.from_numpy(Q).cuda())
    S = exact_score(torch.from_numpy(Q).cuda(), torch.from_numpy(X).cuda(), K).cpu().numpy()
    s = s.cpu().numpy().astype(np.float64)
    se = np.sqrt(n * S / L)
    z = np.abs(s - S) / se
    _say({"max_z": float(z.max()), "mean_S": float(S.mean())})
    assert (z <= 5).all()
    ace.close()
