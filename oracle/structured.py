"""Structured SRP projections (test infrastructure only, like the rest of `oracle/`).

The paper costs a hash at O(d log d + KL) by computing the projections with a fast
transform (Sec. 2.1, Sec. 3.4) but gives no construction.  The one taken here: the row x
is zero-padded to dp (a power of two) and multiplied by M_b = H D3_b H D2_b H D1_b for
blocks b = 0 .. B-1, where H is the dp x dp Sylvester Hadamard matrix (entries +-1,
unnormalised) and each D is a diagonal of random signs; output i of block b is bit
c = b dp + i (c < K L; bit k of table j is c = j K + k, as for a dense W).

M is an integer matrix (|entries| <= dp^2 <= 2^24 for dp <= 4096, so it is exact in
FP32), and its first d columns give a dense projection matrix W [d][K L] with which the
dense oracle computes the same bits: bit c = [sum_t x_t M[c][t] > 0] in FP64.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import hadamard


def structured_matrix(signs: np.ndarray, d: int, K: int, L: int) -> np.ndarray:
    """W = first d columns of the stacked block matrices M_b, transposed: float32 [d][K L].

    The products run in FP64 (a library matmul): every entry of every partial product is
    an integer of magnitude <= dp^2 <= 2^24 and every partial sum stays below 2^53, so the
    result is exact whatever the order of the additions."""
    B, three, dp = signs.shape
    assert three == 3 and dp >= d and B * dp >= K * L
    if dp > 4096:
        raise ValueError("entries of M reach dp^2 and must stay exact in FP32 (dp <= 4096)")
    H = hadamard(dp).astype(np.float64)
    KL = K * L
    rows = []
    for b in range(B):
        D = [np.where(signs[b, r] == 1, -1.0, 1.0) for r in range(3)]
        need = min(dp, KL - b * dp)                # outputs of this block that are bits
        # M_b[:need, :d] = H[:need] D3 H D2 H D1[:, :d]  (diagonal D as a scaling)
        M = H[:, :d] * D[0][None, :d]
        M = H @ (D[1][:, None] * M)
        M = H[:need] @ (D[2][:, None] * M)
        rows.append(M)
    M = np.concatenate(rows, axis=0)
    assert np.abs(M).max() <= 1 << 24 and np.array_equal(M, np.round(M))
    return np.ascontiguousarray(M.T.astype(np.float32))


def structured_hash(X: np.ndarray, signs: np.ndarray, K: int, L: int):
    """Codes [n][L] and ambiguity masks of the structured projection (via the dense oracle)."""
    import oracle
    W = structured_matrix(signs, X.shape[1], K, L)
    return oracle.hash_codes(X, W, K, L)
