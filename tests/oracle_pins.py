"""Checks that pin the oracle to facts outside itself.

Each function raises AssertionError on failure.  They are run against the real
oracle (test_oracle_pins.py) and against deliberately broken builds of it
(test_oracle_mutants.py), which must fail at least one of them.

What pins what (arXiv 1706.06664):
  hand examples        - golden values worked by hand from Sec. 2.1, 3.2, Alg. 1, Sec. 5.3
  exact_signs          - FP64 projection vs exact rational sum, inside the stated margin
  scale_negation       - exact invariances of the SRP sign under x -> 2^k x and x -> -x
  recount              - counts equal a dictionary recount of the codes; sum_b A_j[b] = n
  identical_points     - n identical points: every score is n, mu = n, sigma = 0
  mean_closed_form     - sum_j S2_j = sum_i T_i after the last insert, and equals the
                         running mean of Eq. dynadd (kept with exact fractions)
  order_invariance     - any insertion order gives the same counts and S2/S3
  sigma_two_pass       - exact-integer sigma vs a two-pass FP64 std
  deletion             - insert then delete equals never inserting (Eq. dynsub)
  collision_law        - Monte Carlo SRP collision rate vs 1 - theta/pi (Eq. srp, Eq. metasrp)
  unbiased             - mean over many tables of A_j[H_j(q)] vs sum_i p_i^K (Theorem 1)
  zero_vectors         - S(q, D) with zero rows: p = 1 for two zero vectors and 1/2 for a
                         zero and a nonzero one (Eq. srp under the sign(0) -> 0 reading),
                         against the closed form and a Monte Carlo over the oracle's hash
  table_sigma_bound    - the per-table sigma bounds the inserted points' sigma
  saturating_counters  - short counters (Sec. 3.4) with a cap: stored counts equal
                         min(true count, cap) in any insertion order, S2/S3 follow
                         them, dropped increments = sum of the excess
"""
from __future__ import annotations

import json
import math
import os
from collections import Counter
from fractions import Fraction

import numpy as np

import oracle
from oracle import tiny

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_examples.json")


def hand_examples():
    with open(GOLDEN) as f:
        ex = json.load(f)["examples"]
    for e in ex:
        K, L = e["K"], e["L"]
        X = np.array(e["X"], np.float32)
        W = np.array(e["W"], np.float32)
        codes, amb = oracle.hash_codes(X, W, K, L)
        assert codes.tolist() == e["codes"], (e["name"], codes.tolist())
        sk = oracle.Sketch(K, L)
        sk.insert_codes(codes)
        assert sk.counts.tolist() == e["counts"], (e["name"], sk.counts.tolist())
        assert sk.S2.tolist() == e["S2"]
        assert sk.s3_int == e["S3"]
        T = sk.score_codes(codes)
        assert T.tolist() == e["T"]
        rc, th = sk.threshold(oracle.MODE_SCORED, 1.0)
        assert rc == 0
        mu = e["mu_num"] / e["mu_den"]
        sig = math.sqrt(e["sigma2_num"] / e["sigma2_den"])
        assert abs(th["mu"] - mu) <= 1e-15 * mu
        assert abs(th["mu_scored"] - mu) <= 1e-15 * mu
        assert abs(th["sigma"] - sig) <= 1e-14 * sig
        assert abs(th["sigma_table"] - e["sigma_table"]) <= 1e-14 * e["sigma_table"]
        assert sk.flags(T, th["tau"], oracle.MODE_SCORED).tolist() == e["flags_scored_alpha1"]
        rc, thc = sk.threshold(oracle.MODE_CONST, 1.0)
        assert rc == 0 and abs(thc["tau"] - (mu - 1.0)) <= 1e-15
        assert sk.flags(T, thc["tau"], oracle.MODE_CONST).tolist() == e["flags_const_alpha1"]


def const_mode_is_non_strict():
    """Alg. 1 reports s <= mu - alpha: a score exactly at the threshold is flagged."""
    with open(GOLDEN) as f:
        e = json.load(f)["examples"][1]
    K, L = e["K"], e["L"]
    codes, _ = oracle.hash_codes(np.array(e["X"], np.float32), np.array(e["W"], np.float32), K, L)
    sk = oracle.Sketch(K, L)
    sk.insert_codes(codes)
    T = sk.score_codes(codes)
    # mu = 1.8 = s of none; choose alpha so that tau = 1.0 exactly (= s of the last two points)
    rc, th = sk.threshold(oracle.MODE_CONST, 0.8)
    assert rc == 0
    f = sk.flags(T, 1.0, oracle.MODE_CONST)
    assert f.tolist() == [0, 0, 0, 1, 1]
    f = sk.flags(T, 1.0, oracle.MODE_SCORED)
    assert f.tolist() == [0, 0, 0, 0, 0]


def exact_signs(seed: int = 11):
    """FP64 projections vs exact rational sums: |p64 - p| <= margin, and the sign
    of p64 is the exact sign wherever |p64| > margin.  Includes near-orthogonal
    rows built to make projections tiny."""
    rng = np.random.default_rng(seed)
    d, ncols = 9, 7
    W = rng.standard_normal((d, ncols)).astype(np.float32)
    X = rng.standard_normal((12, d)).astype(np.float32)
    near = []
    for c in range(ncols):
        y = rng.standard_normal(d)
        w = W[:, c].astype(np.float64)
        y = y - (y @ w) / (w @ w) * w                 # orthogonal to column c before rounding
        near.append(y.astype(np.float32))
    X = np.concatenate([X, np.array(near)], axis=0)
    P, M = oracle.project(X, W)
    n_near_zero = 0
    for i in range(X.shape[0]):
        for c in range(ncols):
            ex = tiny.exact_projection(X[i], W[:, c])
            err = abs(Fraction(float(P[i, c])) - ex)
            assert err <= Fraction(float(M[i, c])), (i, c, float(err), M[i, c])
            if abs(P[i, c]) > M[i, c]:
                assert (P[i, c] > 0) == (ex > 0), (i, c)
            if abs(P[i, c]) < 1e-5:
                n_near_zero += 1
    assert n_near_zero >= ncols // 2    # the near-orthogonal rows did land near zero


def scale_negation(seed: int = 12):
    rng = np.random.default_rng(seed)
    K, L, d = 6, 5, 17
    W = rng.standard_normal((d, K * L)).astype(np.float32)
    X = rng.standard_normal((40, d)).astype(np.float32)
    c0, a0 = oracle.hash_codes(X, W, K, L)
    for k in (-7, -1, 3, 20):
        ck, ak = oracle.hash_codes(np.ldexp(X, k), W, K, L)
        assert np.array_equal(ck, c0) and np.array_equal(ak, a0)
    P, _ = oracle.project(X, W)
    assert np.all(P != 0.0)
    cn, _ = oracle.hash_codes(-X, W, K, L)
    assert np.array_equal(cn, (~c0) & np.uint16((1 << K) - 1))
    # a zero row projects to exactly 0 everywhere: every bit 0, every bit ambiguous
    cz, az = oracle.hash_codes(np.zeros((1, d), np.float32), W, K, L)
    assert np.all(cz == 0) and np.all(az == (1 << K) - 1)


def recount(seed: int = 13):
    rng = np.random.default_rng(seed)
    K, L, d, n = 5, 7, 6, 300
    W = rng.standard_normal((d, K * L)).astype(np.float32)
    X = rng.standard_normal((n, d)).astype(np.float32)
    codes, _ = oracle.hash_codes(X, W, K, L)
    # the codes themselves against exact rational signs on a few rows
    ex = tiny.exact_codes(X[:8].tolist(), W.tolist(), K, L)
    assert codes[:8].tolist() == ex
    sk = oracle.Sketch(K, L)
    sk.insert_codes(codes)
    assert int(sk.n[0]) == n
    for j in range(L):
        cnt = Counter(codes[:, j].tolist())
        dense = np.zeros(1 << K, np.int64)
        for b, v in cnt.items():
            dense[b] = v
        assert np.array_equal(sk.counts[j], dense)
        assert int(sk.counts[j].sum()) == n
        assert int(sk.S2[j]) == sum(v * v for v in cnt.values())
        assert sk.s3_int[j] == sum(v ** 3 for v in cnt.values())
    T = sk.score_codes(codes)
    for i in range(0, n, 37):
        assert int(T[i]) == sum(int(sk.counts[j, codes[i, j]]) for j in range(L))


def identical_points():
    """n copies of one point: every table puts all n in one bucket, so every score is n,
    mu = n and sigma = 0 (a point identical to every inserted one scores n)."""
    rng = np.random.default_rng(14)
    K, L, d, n = 8, 6, 5, 257
    W = rng.standard_normal((d, K * L)).astype(np.float32)
    X = np.repeat(rng.standard_normal((1, d)).astype(np.float32), n, axis=0)
    codes, _ = oracle.hash_codes(X, W, K, L)
    sk = oracle.Sketch(K, L)
    sk.insert_codes(codes)
    T = sk.score_codes(codes)
    assert np.all(T == n * L)
    rc, th = sk.threshold()
    assert rc == 0 and th["mu"] == n and th["mu_scored"] == n and th["sigma"] == 0.0
    assert th["sigma_table"] == 0.0


def mean_closed_form(seed: int = 15):
    """After the last insert, sum_j S2_j equals the sum of the inserted points' T
    (so mu = sum S2 / (n L) is the mean score, Sec. 3.4.1), and it equals the mean
    kept step by step with Eq. dynadd in exact fractions."""
    rng = np.random.default_rng(seed)
    K, L, d, n = 3, 4, 4, 120
    W = rng.standard_normal((d, K * L)).astype(np.float32)
    X, _ = _clusters(rng, n, d)
    codes, _ = oracle.hash_codes(X, W, K, L)
    sk = oracle.Sketch(K, L)
    run = tiny.TinyACE(L)
    for i in range(n):
        sk.insert_codes(codes[i:i + 1])
        run.insert(codes[i].tolist())
        assert Fraction(int(sk.S2.sum()), (i + 1) * L) == run.mu
    T = sk.score_codes(codes)
    assert int(T.sum()) == int(sk.S2.sum())
    rc, th = sk.threshold()
    assert th["mu"] == float(run.mu)
    assert th["mu"] == th["mu_scored"]


def order_invariance(seed: int = 16):
    rng = np.random.default_rng(seed)
    K, L, d, n = 4, 5, 3, 200
    W = rng.standard_normal((d, K * L)).astype(np.float32)
    X, _ = _clusters(rng, n, d)
    codes, _ = oracle.hash_codes(X, W, K, L)
    a = oracle.Sketch(K, L)
    a.insert_codes(codes)
    b = oracle.Sketch(K, L)
    b.insert_codes(codes[rng.permutation(n)])
    assert np.array_equal(a.counts, b.counts)
    assert np.array_equal(a.S2, b.S2) and np.array_equal(a.S3, b.S3)


def sigma_two_pass(seed: int = 17):
    rng = np.random.default_rng(seed)
    K, L, d, n = 6, 9, 8, 2000
    W = rng.standard_normal((d, K * L)).astype(np.float32)
    X, _ = _clusters(rng, n, d)
    codes, _ = oracle.hash_codes(X, W, K, L)
    sk = oracle.Sketch(K, L)
    sk.insert_codes(codes)
    T = sk.score_codes(codes)
    rc, th = sk.threshold()
    s = T.astype(np.float64) / L
    assert abs(th["mu_scored"] - s.mean()) <= 1e-13 * s.mean()
    assert abs(th["sigma"] - s.std(ddof=0)) <= 1e-12 * s.std(ddof=0)
    m = len(T)
    assert sk.sumT2_int == sum(int(t) * int(t) for t in T) and int(sk.m[0]) == m


def deletion(seed: int = 18):
    """Inserting everything and then deleting a subset gives the same state as
    inserting only the rest; the running mean of Eq. dynsub matches."""
    rng = np.random.default_rng(seed)
    K, L, d, n = 4, 6, 5, 150
    W = rng.standard_normal((d, K * L)).astype(np.float32)
    X, _ = _clusters(rng, n, d)
    codes, _ = oracle.hash_codes(X, W, K, L)
    drop = rng.permutation(n)[:60]
    keep = np.setdiff1d(np.arange(n), drop)
    a = oracle.Sketch(K, L)
    a.insert_codes(codes)
    run = tiny.TinyACE(L)
    for i in range(n):
        run.insert(codes[i].tolist())
    assert a.delete_codes(codes[drop]) == 0
    for i in drop:
        run.delete(codes[i].tolist())
    b = oracle.Sketch(K, L)
    b.insert_codes(codes[keep])
    assert np.array_equal(a.counts, b.counts)
    assert np.array_equal(a.S2, b.S2) and np.array_equal(a.S3, b.S3) and a.n[0] == b.n[0]
    assert Fraction(int(a.S2.sum()), int(a.n[0]) * L) == run.mu
    # a point whose bucket is empty in some table was never inserted: rejected whole
    empty = oracle.Sketch(K, L)
    assert empty.delete_codes(codes[:3]) == 3 and empty.n[0] == 0


def collision_law(seed: int = 19, R: int = 400_000):
    """Eq. srp and Eq. metasrp by Monte Carlo: with R independent N(0,1) columns the
    fraction of equal bits of two points is 1 - theta/pi, and of equal K-bit codes
    (1 - theta/pi)^K, each within 5 binomial standard errors."""
    rng = np.random.default_rng(seed)
    d = 5
    pairs = [(rng.standard_normal(d), rng.standard_normal(d)) for _ in range(3)]
    x0 = rng.standard_normal(d)
    pairs.append((x0, x0 + 0.3 * rng.standard_normal(d)))      # a close pair
    for x, y in pairs:
        x32, y32 = x.astype(np.float32), y.astype(np.float32)
        xd, yd = x32.astype(np.float64), y32.astype(np.float64)
        theta = math.acos(float(np.clip(xd @ yd / (np.linalg.norm(xd) * np.linalg.norm(yd)), -1, 1)))
        p = 1.0 - theta / math.pi
        W = rng.standard_normal((d, R)).astype(np.float32)
        codes, _ = oracle.hash_codes(np.stack([x32, y32]), W, 1, R)
        rate = float(np.mean(codes[0] == codes[1]))
        assert abs(rate - p) <= 5 * math.sqrt(p * (1 - p) / R), (rate, p)
        K = 4
        codes, _ = oracle.hash_codes(np.stack([x32, y32]), W, K, R // K)
        rate = float(np.mean(codes[0] == codes[1]))
        pk = p ** K
        assert abs(rate - pk) <= 5 * math.sqrt(pk * (1 - pk) / (R // K)), (rate, pk)


def unbiased(seed: int = 20, L: int = 60_000):
    """Theorem 1: A_j[H_j(q)] is an unbiased estimate of S(q, D) = sum_i p_i^K.  With
    L independent tables the mean lies within 5 standard errors of the exact S
    computed from brute-force angles."""
    rng = np.random.default_rng(seed)
    n, d, K = 20, 3, 3
    X, _ = _clusters(rng, n, d)
    Q = np.concatenate([X[:2], rng.uniform(-20, 20, (2, d)).astype(np.float32)])
    W = rng.standard_normal((d, K * L)).astype(np.float32)
    cx, _ = oracle.hash_codes(X, W, K, L)
    cq, _ = oracle.hash_codes(Q, W, K, L)
    sk = oracle.Sketch(K, L)
    sk.insert_codes(cx)
    S = oracle.exact_score(Q, X, K)
    for a in range(Q.shape[0]):
        per_table = sk.counts[np.arange(L), cq[a].astype(np.int64)].astype(np.float64)
        # brute-force S from angles, independent of the oracle's exact_score
        brute = 0.0
        for x in X.astype(np.float64):
            q = Q[a].astype(np.float64)
            cs = float(np.clip(q @ x / (np.linalg.norm(q) * np.linalg.norm(x)), -1, 1))
            brute += (1.0 - math.acos(cs) / math.pi) ** K
        assert abs(S[a] - brute) <= 1e-9 * max(1.0, brute)
        se = per_table.std(ddof=1) / math.sqrt(L)
        assert abs(per_table.mean() - S[a]) <= 5 * se + 1e-12, (a, per_table.mean(), S[a], se)
        T = sk.score_codes(cq[a:a + 1], accumulate=False)
        assert int(T[0]) == int(per_table.sum())


def zero_vectors(seed: int = 23, R: int = 200_000):
    """Eq. thescore with zero vectors.  A zero vector projects to 0 on every column, so under
    the sign(0) -> 0 reading all its bits are 0: it collides with another zero vector on every
    bit (p = 1) and with a nonzero vector on half of the bits on average (p = 1/2, the
    nonzero vector's bit being a fair coin over W ~ N(0, I)).  Checked two ways that do not go
    through the exact-score routine: the closed form sum of p^K with those p and brute-force
    angles for the nonzero pairs, and a Monte Carlo of bit collisions over R columns of the
    oracle's own hash."""
    rng = np.random.default_rng(seed)
    d, K = 5, 3
    X = rng.standard_normal((7, d)).astype(np.float32)
    X[[1, 4]] = 0.0
    Q = np.stack([np.zeros(d, np.float32), X[0], rng.standard_normal(d).astype(np.float32)])
    S = oracle.exact_score(Q, X, K)
    for a in range(Q.shape[0]):
        q = Q[a].astype(np.float64)
        want = 0.0
        for x in X.astype(np.float64):
            qz, xz = not q.any(), not x.any()
            if qz and xz:
                p = 1.0
            elif qz or xz:
                p = 0.5
            else:
                cs = float(np.clip(q @ x / (np.linalg.norm(q) * np.linalg.norm(x)), -1, 1))
                p = 1.0 - math.acos(cs) / math.pi
            want += p ** K
        assert abs(S[a] - want) <= 1e-12 * max(1.0, want), (a, S[a], want)
    # zero query against only zero rows: every pair collides surely, S = n
    assert oracle.exact_score(Q[:1], X[[1, 4]], K)[0] == 2.0
    # Monte Carlo over the hash: zero rows give all-zero codes; a zero and a nonzero row agree
    # on a bit with rate 1/2
    W = rng.standard_normal((d, R)).astype(np.float32)
    codes, _ = oracle.hash_codes(np.stack([X[1], X[4], X[0]]), W, 1, R)
    assert not codes[0].any() and not codes[1].any()
    rate = float(np.mean(codes[0] == codes[2]))
    assert abs(rate - 0.5) <= 5 * math.sqrt(0.25 / R), rate


def table_sigma_bound(seed: int = 21):
    rng = np.random.default_rng(seed)
    K, L, d, n = 5, 8, 6, 700
    W = rng.standard_normal((d, K * L)).astype(np.float32)
    X, _ = _clusters(rng, n, d)
    codes, _ = oracle.hash_codes(X, W, K, L)
    sk = oracle.Sketch(K, L)
    sk.insert_codes(codes)
    sk.score_codes(codes)
    rc, th = sk.threshold(oracle.MODE_TABLE, 1.0)
    assert rc == 0
    assert th["sigma"] <= th["sigma_table"] * (1 + 1e-12)
    assert th["tau"] == th["mu"] - th["sigma_table"]
    # per-table sigma from the counts directly: var_j = sum_b A^3 / n - (sum_b A^2 / n)^2
    per = []
    for j in range(L):
        a = sk.counts[j].astype(np.float64)
        per.append(math.sqrt(max(0.0, (a ** 3).sum() / n - ((a ** 2).sum() / n) ** 2)))
    assert abs(np.mean(per) - th["sigma_table"]) <= 1e-9 * th["sigma_table"]


def saturating_counters(seed: int = 22):
    rng = np.random.default_rng(seed)
    K, L, n, cap = 3, 4, 300, 7
    # skewed codes so that several buckets pass the cap
    codes = np.minimum(rng.geometric(0.35, size=(n, L)) - 1, (1 << K) - 1).astype(np.uint16)
    sk = oracle.Sketch(K, L, cap=cap)
    sk.insert_codes(codes[:120])
    sk.insert_codes(codes[120:])
    true = np.stack([np.bincount(codes[:, j].astype(np.int64), minlength=1 << K) for j in range(L)])
    want = np.minimum(true, cap)
    assert (true > cap).any()
    assert np.array_equal(sk.counts, want)
    assert sk.dropped == int(np.maximum(true - cap, 0).sum())
    assert int(sk.n[0]) == n
    assert np.array_equal(sk.S2, (want ** 2).sum(axis=1))
    assert sk.s3_int == [int((want[j].astype(object) ** 3).sum()) for j in range(L)]
    # another order gives the same state
    sk2 = oracle.Sketch(K, L, cap=cap)
    sk2.insert_codes(codes[rng.permutation(n)])
    assert np.array_equal(sk2.counts, sk.counts) and np.array_equal(sk2.S2, sk.S2) and sk2.dropped == sk.dropped
    # a cap that is never reached changes nothing
    big = oracle.Sketch(K, L, cap=10 ** 9)
    big.insert_codes(codes)
    ref = oracle.Sketch(K, L)
    ref.insert_codes(codes)
    assert np.array_equal(big.counts, ref.counts) and np.array_equal(big.S2, ref.S2) and big.dropped == 0
    assert big.s3_int == ref.s3_int
    # scores read the stored counts
    T = sk.score_codes(codes[:5], accumulate=False)
    assert list(T) == [int(sum(want[j, codes[i, j]] for j in range(L))) for i in range(5)]


def _clusters(rng, n, d):
    means = rng.standard_normal((3, d)) * 5
    X = means[rng.integers(0, 3, n)] + rng.standard_normal((n, d))
    return X.astype(np.float32), None


ALL = [saturating_counters, hand_examples, const_mode_is_non_strict, exact_signs, scale_negation, recount,
       identical_points, mean_closed_form, order_invariance, sigma_two_pass, deletion,
       collision_law, unbiased, zero_vectors, table_sigma_bound]
