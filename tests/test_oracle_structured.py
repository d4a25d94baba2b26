"""Pins of the structured projection in `oracle/structured.py` (CPU only).

  orthogonality  - M M^T = dp^3 I exactly (each H D factor is sqrt(dp) times orthogonal)
  definition     - M built entry by entry from H[i][j] = (-1)^popcount(i & j) (Sylvester),
                   without the library Hadamard routine, on small sizes
  collision_law  - bits of two unit vectors at angle theta agree at rate 1 - theta/pi
                   (Eq. srp) within 0.015 over 25,600 bits
Plausible mistakes planted in copies of the builder must each fail one of them.
"""
import math

import numpy as np
import pytest

from ace_inputs import structured_signs
from oracle import structured


def _sylvester(dp):
    return np.array([[(-1) ** bin(i & j).count("1") for j in range(dp)] for i in range(dp)], dtype=np.int64)


def pin_orthogonality(build):
    signs, dp = structured_signs(64, 8, 8, 5)           # one block of 64 outputs
    M = build(signs, 64, 8, 8).astype(np.int64).T      # [64][64]
    assert np.array_equal(M @ M.T, dp ** 3 * np.eye(dp, dtype=np.int64))


def pin_definition(build):
    rng = np.random.default_rng(7)
    dp, B, d, K, L = 8, 2, 5, 3, 4
    signs = (rng.random((B, 3, dp)) < 0.5).astype(np.uint8)
    H = _sylvester(dp)
    want = np.zeros((K * L, d), np.int64)
    for c in range(K * L):
        b, i = divmod(c, dp)
        s = [[-1 if signs[b, r, t] else 1 for t in range(dp)] for r in range(3)]
        for t in range(d):
            # entry (i, t) of H D3 H D2 H D1: sum over u, v of H[i][u] s3[u] H[u][v] s2[v] H[v][t] s1[t]
            want[c, t] = sum(H[i, u] * s[2][u] * H[u, v] * s[1][v] * H[v, t] * s[0][t]
                             for u in range(dp) for v in range(dp))
    assert np.array_equal(build(signs, d, K, L).astype(np.int64).T, want)


def pin_collision_law(build):
    rng = np.random.default_rng(11)
    d = 128
    signs, _ = structured_signs(d, 16, 1600, 3)        # 200 blocks
    W = build(signs, d, 16, 1600).astype(np.float64)
    for th in (math.pi / 6, math.pi / 3, math.pi / 2, 2 * math.pi / 3):
        x = rng.standard_normal(d)
        u = rng.standard_normal(d)
        u -= (u @ x) / (x @ x) * x
        x /= np.linalg.norm(x)
        u /= np.linalg.norm(u)
        y = math.cos(th) * x + math.sin(th) * u
        rate = float((((x @ W) > 0) == ((y @ W) > 0)).mean())
        assert abs(rate - (1 - th / math.pi)) < 0.015, (th, rate)


PINS = [pin_orthogonality, pin_definition, pin_collision_law]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_structured_pin(pin):
    pin(structured.structured_matrix)


def _mutant(kind):
    """A copy of the builder with one plausible mistake."""
    from scipy.linalg import hadamard

    def build(signs, d, K, L):
        B, _, dp = signs.shape
        H = hadamard(dp).astype(np.int64)
        rows = []
        for b in range(B):
            D = [np.where(signs[b, r] == 1, -1, 1).astype(np.int64) for r in range(3)]
            if kind == "missing_middle_diagonal":
                D[1] = np.ones(dp, np.int64)
            if kind == "sign_rows_not_columns":
                M = D[0][:, None] * H
            else:
                M = H * D[0][None, :]
            M = H @ (D[1][:, None] * M)
            if kind != "two_rounds":
                M = H @ (D[2][:, None] * M)
            rows.append(M[:, :d])
        M = np.concatenate(rows, axis=0)
        if kind == "blocks_interleaved":
            M = M.reshape(B, dp, -1).transpose(1, 0, 2).reshape(B * dp, -1)
        return np.ascontiguousarray(M[: K * L].T.astype(np.float32))
    return build


@pytest.mark.parametrize("kind", ["missing_middle_diagonal", "sign_rows_not_columns", "two_rounds",
                                  "blocks_interleaved"])
def test_structured_mutant_is_caught(kind):
    build = _mutant(kind)
    failed = []
    for pin in PINS:
        try:
            pin(build)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin caught {kind}"
