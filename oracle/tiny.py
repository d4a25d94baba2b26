"""Exact pure-Python ACE for tiny inputs (test infrastructure only).

Written from the paper (arXiv 1706.06664) independently of the C oracle:
every projection is summed exactly as a rational number, so its sign is the
true sign of w^T x (Sec. 2.1); counts, scores and the running mean are Python
integers and Fractions (Alg. 1, Sec. 3.4.1 Eq. dynadd).  Only for a few
hundred points at most.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Dict, List, Sequence


def exact_projection(x: Sequence[float], w_col: Sequence[float]) -> Fraction:
    return sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, w_col)), Fraction(0))


def exact_codes(X, W, K: int, L: int) -> List[List[int]]:
    """codes[i][j] = sum_k [w_{jK+k}^T x_i > 0] 2^k, from exact rational projections."""
    d = len(X[0])
    out = []
    for x in X:
        row = []
        for j in range(L):
            code = 0
            for k in range(K):
                c = j * K + k
                p = exact_projection(x, [W[t][c] for t in range(d)])
                if p > 0:
                    code |= 1 << k
            row.append(code)
        out.append(row)
    return out


class TinyACE:
    """Alg. 1 with a dictionary per table and the mean kept by Eq. dynadd."""

    def __init__(self, L: int):
        self.L = L
        self.tables: List[Dict[int, int]] = [dict() for _ in range(L)]
        self.n = 0
        self.mu = Fraction(0)

    def insert(self, codes_row: Sequence[int]):
        # Eq. dynadd: mu' = (n mu + sum_j (2 A_j[H_j(x)] + 1) / L) / (n + 1), A_j before the increment
        incr = Fraction(0)
        for j, b in enumerate(codes_row):
            a = self.tables[j].get(b, 0)
            incr += Fraction(2 * a + 1, self.L)
            self.tables[j][b] = a + 1
        self.mu = (self.n * self.mu + incr) / (self.n + 1)
        self.n += 1

    def delete(self, codes_row: Sequence[int]):
        # Eq. dynsub: mu' = (n mu - sum_j (2 A_j[H_j(x)] - 1) / L) / (n - 1), A_j before the decrement
        decr = Fraction(0)
        for j, b in enumerate(codes_row):
            a = self.tables[j][b]
            decr += Fraction(2 * a - 1, self.L)
            self.tables[j][b] = a - 1
        self.mu = (self.n * self.mu - decr) / (self.n - 1) if self.n > 1 else Fraction(0)
        self.n -= 1

    def score(self, codes_row: Sequence[int]) -> Fraction:
        return sum((Fraction(self.tables[j].get(b, 0)) for j, b in enumerate(codes_row)), Fraction(0)) / self.L

