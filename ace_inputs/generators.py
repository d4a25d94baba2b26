"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and arranges them into arrays.  It holds
none of the ACE arithmetic (no projections, signs, codes, counts or scores), so
both the CPU oracle and the HIP path can take their inputs from here without
sharing any of the method.

The paper evaluates on Statlog Shuttle, ALOI and KDD-Cup99 HTTP (Section 5.1,
Table 1).  Those datasets are not available here; every workload below is a
synthetic stand-in with the shape, value distribution and anomaly structure of
the workload it replaces, built from the recipe in its docstring.

The projection matrix follows Section 2.1: every entry of every SRP vector w is
an independent N(0, 1) draw; W has shape [d][K*L] and column c = j*K + k holds
bit k of table j.
"""
from __future__ import annotations

import dataclasses
import numpy as np

SEED_W_BASE = 1706066640


def projection_matrix(d: int, K: int, L: int, seed: int) -> np.ndarray:
    """W ~ N(0,1), float32, shape [d][K*L]; drawn in float64 from PCG64(seed), then rounded."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((d, K * L)).astype(np.float32)


def gaussian_clusters(n: int, d: int, n_clusters: int, anomaly_frac: float, seed: int,
                      mean_std: float = 5.0, anomaly_box: float = 20.0):
    """Isotropic Gaussian clusters plus uniform anomalies.

    Cluster means ~ N(0, mean_std^2 I), points ~ N(mean, I); a fraction
    `anomaly_frac` of the rows is replaced by uniform draws in
    [-anomaly_box, anomaly_box]^d.  Rows are shuffled.  Returns (X float32
    [n][d], is_anomaly bool [n]).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n_anom = int(round(n * anomaly_frac))
    n_in = n - n_anom
    means = rng.standard_normal((n_clusters, d)) * mean_std
    which = rng.integers(0, n_clusters, size=n_in)
    inl = means[which] + rng.standard_normal((n_in, d))
    anom = rng.uniform(-anomaly_box, anomaly_box, size=(n_anom, d))
    X = np.concatenate([inl, anom], axis=0)
    lab = np.concatenate([np.zeros(n_in, bool), np.ones(n_anom, bool)])
    perm = rng.permutation(n)
    return X[perm].astype(np.float32), lab[perm]


def c1_points(n: int = 10_000, seed: int = 1):
    """Small clustered workload: d=32, 4 clusters with means ~N(0,25 I), unit variance,
    1% anomalies uniform in [-20,20]^32."""
    return gaussian_clusters(n, 32, 4, 0.01, seed)


# Cardinalities of the three categorical fields of the connection-log stand-in;
# they sum to 82 one-hot columns.
C2_CARDS = (3, 68, 11)
C2_N_CONT = 38


def _zipf_probs(card: int, s: float, reverse: bool = False) -> np.ndarray:
    k = np.arange(1, card + 1, dtype=np.float64)
    p = k ** (-s)
    p /= p.sum()
    return p[::-1].copy() if reverse else p


def c2_points(n: int = 494_021, seed: int = 2, anomaly_frac: float = 0.2):
    """Connection-log shaped workload: d = 38 + 82 = 120.

    Inliers: 38 lognormal(0,1) columns; 3 categorical fields of cardinality
    (3, 68, 11) one-hot encoded, category k drawn with probability ~ k^-1.2.
    Anomalies (20% of rows) come from 5 rare clusters: each cluster shifts the
    lognormal log-means by N(0, 1.5^2) per feature and draws categories from
    the reversed Zipf order.  The continuous columns are z-scored over all rows
    at the end.  Returns (X float32 [n][120], is_anomaly bool [n]).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n_anom = int(round(n * anomaly_frac))
    is_anom = np.zeros(n, bool)
    is_anom[rng.permutation(n)[:n_anom]] = True
    cluster = rng.integers(0, 5, size=n)
    offsets = rng.normal(0.0, 1.5, size=(5, C2_N_CONT))
    logmean = np.where(is_anom[:, None], offsets[cluster], 0.0)
    cont = np.exp(logmean + rng.standard_normal((n, C2_N_CONT)))
    cont = (cont - cont.mean(axis=0)) / cont.std(axis=0)
    d = C2_N_CONT + sum(C2_CARDS)
    X = np.zeros((n, d), np.float32)
    X[:, :C2_N_CONT] = cont
    col = C2_N_CONT
    for card in C2_CARDS:
        cat_in = rng.choice(card, size=n, p=_zipf_probs(card, 1.2))
        cat_out = rng.choice(card, size=n, p=_zipf_probs(card, 1.2, reverse=True))
        cat = np.where(is_anom, cat_out, cat_in)
        X[np.arange(n), col + cat] = 1.0
        col += card
    return X, is_anom


def low_rank_points_torch(n: int, d: int, seed: int, device, rank: int = 32,
                          noise: float = 0.1, anomaly_frac: float = 0.005, chunk: int = 1 << 18):
    """Dense low-rank-plus-noise workload, generated on `device` with a seeded torch.Generator.

    Inliers: X = Z F + noise*E with Z ~ N(0,1) [n][rank], F ~ N(0, 1/rank) [rank][d].
    Anomalies: g ~ N(0, I) projected off row-space(F) (QR of F^T), rescaled to the
    median inlier norm, plus noise*E.  Returns (X float32 [n][d] on device,
    is_anomaly bool [n] on device).
    """
    import torch
    gcpu = torch.Generator().manual_seed(seed)
    F = torch.randn(rank, d, generator=gcpu, dtype=torch.float64) / np.sqrt(rank)
    Q, _ = torch.linalg.qr(F.T)  # d x rank, orthonormal basis of row-space(F)
    n_anom = int(round(n * anomaly_frac))
    perm = torch.randperm(n, generator=gcpu)
    is_anom = torch.zeros(n, dtype=torch.bool)
    is_anom[perm[:n_anom]] = True
    F32 = F.to(device=device, dtype=torch.float32)
    Q32 = Q.to(device=device, dtype=torch.float32)
    is_anom_d = is_anom.to(device)
    g = torch.Generator(device=device).manual_seed(seed + 1)
    X = torch.empty((n, d), dtype=torch.float32, device=device)
    med = None
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        m = e - s
        Z = torch.randn((m, rank), generator=g, device=device)
        blk = Z @ F32
        if med is None:
            med = blk.norm(dim=1).median()
        G = torch.randn((m, d), generator=g, device=device)
        Goff = G - (G @ Q32) @ Q32.T
        Goff = Goff * (med / Goff.norm(dim=1, keepdim=True).clamp_min(1e-30))
        blk = torch.where(is_anom_d[s:e, None], Goff, blk)
        blk += noise * torch.randn((m, d), generator=g, device=device)
        X[s:e] = blk
    return X, is_anom_d


def heavy_tail_points_torch(n: int, d: int, seed: int, device, dof: float = 3.0,
                            anomaly_frac: float = 0.01, coord_frac: float = 0.05,
                            scale: float = 10.0, chunk: int = 1 << 16):
    """Student-t(dof) features; anomalies have `coord_frac` of their coordinates
    (chosen per row) multiplied by `scale`.  Generated on `device`."""
    import torch
    gcpu = torch.Generator().manual_seed(seed)
    n_anom = int(round(n * anomaly_frac))
    perm = torch.randperm(n, generator=gcpu)
    is_anom = torch.zeros(n, dtype=torch.bool)
    is_anom[perm[:n_anom]] = True
    is_anom_d = is_anom.to(device)
    n_coord = int(round(d * coord_frac))
    g = torch.Generator(device=device).manual_seed(seed + 1)
    X = torch.empty((n, d), dtype=torch.float32, device=device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        m = e - s
        # Student-t as N(0,1) / sqrt(chi2_dof / dof); chi2 from a sum of squared normals
        z = torch.randn((m, d), generator=g, device=device)
        chi = torch.zeros((m, d), device=device)
        for _ in range(int(dof)):
            chi += torch.randn((m, d), generator=g, device=device) ** 2
        t = z / torch.sqrt(chi / dof)
        sel = torch.rand((m, d), generator=g, device=device).argsort(dim=1)[:, :n_coord]
        mult = torch.ones((m, d), device=device)
        mult.scatter_(1, sel, scale)
        t = torch.where(is_anom_d[s:e, None], t * mult, t)
        X[s:e] = t
    return X, is_anom_d


@dataclasses.dataclass
class Request:
    rid: int
    kind: str          # "insert" or "score"
    n: int
    arrival_s: float


def serving_requests(n_requests: int, seed: int = 5, insert_frac: float = 0.7,
                     median_batch: int = 256, sigma_log: float = 1.0,
                     max_batch: int = 65_536, rate_per_s: float = 1000.0):
    """Poisson stream of insert/score requests with lognormal batch sizes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kinds = np.where(rng.random(n_requests) < insert_frac, "insert", "score")
    sizes = np.clip(np.round(rng.lognormal(np.log(median_batch), sigma_log, n_requests)), 1, max_batch)
    gaps = rng.exponential(1.0 / rate_per_s, n_requests)
    t = np.cumsum(gaps)
    return [Request(i, str(kinds[i]), int(sizes[i]), float(t[i])) for i in range(n_requests)]


def drifting_mixture_rows(rid: int, n: int, d: int, seed: int = 5, n_means: int = 8,
                          drift_per_1000: float = 0.01, anomaly_frac: float = 0.01):
    """Rows of request `rid`: 8 Gaussian-mixture means ~N(0,25 I) that drift by
    0.01 per coordinate per 1,000 requests along a fixed random sign vector,
    unit variance, 1% anomalies uniform in [-20,20]^d.  Each request has its
    own counter-keyed stream (seed, rid), so any request can be regenerated."""
    base = np.random.Generator(np.random.PCG64(seed))
    means = base.standard_normal((n_means, d)) * 5.0
    signs = np.where(base.random((n_means, d)) < 0.5, -1.0, 1.0)
    rng = np.random.Generator(np.random.PCG64([seed, rid]))
    shift = drift_per_1000 * (rid / 1000.0)
    which = rng.integers(0, n_means, size=n)
    X = means[which] + shift * signs[which] + rng.standard_normal((n, d))
    anom = rng.random(n) < anomaly_frac
    X[anom] = rng.uniform(-20.0, 20.0, size=(int(anom.sum()), d))
    return X.astype(np.float32), anom


def serving_trace(n_requests: int, d: int, seed: int = 5, median_batch: int = 256, sigma_log: float = 1.0,
                  max_batch: int = 65_536, rate_per_s: float = 1000.0, insert_frac: float = 0.7,
                  pool_rows: int | None = None, n_override: dict | None = None):
    """Request log and host rows of the serving workload.

    Returns (kind int32 [R] with 0 = insert and 1 = score, n int64 [R], row0 int64 [R],
    out0 int64 [R], t_arrival float64 [R] in seconds, pool float32 [rows][d]).  Score
    outputs are packed: request r writes [out0, out0 + n).  With pool_rows=None every
    request has its own rows, drifting_mixture_rows(r, n), laid out in request order.
    Otherwise the pool holds pool_rows drifting rows (blocks of 16,384 rows, block b drawn as
    request id 1000*b) and request r reads the window starting at a seeded offset.
    n_override {rid: rows} replaces the drawn sizes of the named requests."""
    reqs = serving_requests(n_requests, seed=seed, insert_frac=insert_frac, median_batch=median_batch,
                            sigma_log=sigma_log, max_batch=max_batch, rate_per_s=rate_per_s)
    kind = np.array([0 if q.kind == "insert" else 1 for q in reqs], np.int32)
    n = np.array([q.n for q in reqs], np.int64)
    for rid, rows in (n_override or {}).items():
        n[rid] = rows
    t = np.array([q.arrival_s for q in reqs], np.float64)
    out0 = np.zeros(n_requests, np.int64)
    sc = kind == 1
    out0[sc] = np.concatenate([[0], np.cumsum(n[sc])[:-1]]) if sc.any() else []
    if pool_rows is None:
        row0 = np.concatenate([[0], np.cumsum(n)[:-1]]).astype(np.int64)
        pool = np.concatenate([drifting_mixture_rows(r, int(n[r]), d, seed=seed)[0] for r in range(n_requests)])
    else:
        blk = 16_384
        nb = -(-pool_rows // blk)
        pool = np.concatenate([drifting_mixture_rows(1000 * b, blk, d, seed=seed)[0] for b in range(nb)])[:pool_rows]
        if n.max() > pool_rows:
            raise ValueError("pool smaller than the largest request")
        rng = np.random.Generator(np.random.PCG64([seed, 7]))
        row0 = (rng.random(n_requests) * (pool_rows - n + 1)).astype(np.int64)
    return kind, n, row0, out0, t, np.ascontiguousarray(pool, np.float32)


def structured_signs(d: int, K: int, L: int, seed: int):
    """Random sign diagonals of the structured projection: returns (signs uint8 [B][3][dp]
    holding 0 for +1 and 1 for -1, dp), with dp = max(64, next power of two >= d) and
    B = ceil(K*L / dp) independent blocks of three diagonals each."""
    dp = 64
    while dp < d:
        dp *= 2
    B = -(-(K * L) // dp)
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.random((B, 3, dp)) < 0.5).astype(np.uint8), dp


def serving_rows_torch(n: np.ndarray, d: int, out, seed: int = 5, n_means: int = 8,
                       drift_per_1000: float = 0.01, anomaly_frac: float = 0.01,
                       block_rows: int = 1 << 20, device="cuda"):
    """Rows of a whole request log, written into `out` (float32 [sum n][d], host pinned or
    device) in request order: request r holds rows [cumsum(n)[r-1], cumsum(n)[r]).  The
    recipe is drifting_mixture_rows': 8 mixture means ~N(0, 25 I) (the same means and drift
    signs as drifting_mixture_rows for this seed), mean g shifted by 0.01 (r / 1000) per
    coordinate along its sign vector, so the drift follows the request id r; unit variance;
    1% anomalies uniform in [-20, 20]^d.  Rows are drawn on the GPU in blocks of whole
    requests (about block_rows rows), block b from its own torch Philox stream seeded by
    (seed, b), so the log is reproducible block by block."""
    import torch
    base = np.random.Generator(np.random.PCG64(seed))
    means = torch.from_numpy(base.standard_normal((n_means, d)) * 5.0).to(device=device, dtype=torch.float32)
    signs = torch.from_numpy(np.where(base.random((n_means, d)) < 0.5, -1.0, 1.0)).to(device=device,
                                                                                         dtype=torch.float32)
    n = np.asarray(n, np.int64)
    ends = np.cumsum(n)
    r, row, b = 0, 0, 0
    while r < len(n):
        r1 = r
        while r1 < len(n) and (r1 == r or ends[r1] - row <= block_rows):
            r1 += 1
        m = int(ends[r1 - 1] - row)
        g = torch.Generator(device=device)
        g.manual_seed(int(seed) * 1_000_003 + b)
        rid = torch.from_numpy(np.repeat(np.arange(r, r1), n[r:r1])).to(device=device, dtype=torch.float32)
        which = torch.randint(0, n_means, (m,), generator=g, device=device)
        X = torch.randn((m, d), generator=g, device=device)
        X += means[which] + (drift_per_1000 * rid / 1000.0)[:, None] * signs[which]
        anom = torch.rand((m,), generator=g, device=device) < anomaly_frac
        U = torch.rand((m, d), generator=g, device=device) * 40.0 - 20.0
        X = torch.where(anom[:, None], U, X)
        out[row:row + m].copy_(X, non_blocking=False)
        row += m
        r = r1
        b += 1
    return out
