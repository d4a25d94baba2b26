"""GPU-vs-oracle comparison helpers (used by the gpu-marked tests, smoke() and bench.py).

The bar, per quantity:
  codes   bit-exact wherever the oracle's FP64 projection is outside its rounding
          margin (|p64| > gamma_d(2^-53) sum|x w|); bits inside it are counted.
  counts  exact: against the oracle when no code differs, and always against a
          recount of the GPU's own codes.
  T       exact integers; s = T / L within 1e-6 relative (FP32 output).
  mu, sigma, sigma_table  within 1e-12 relative (exact integer sums, FP64 finish).
  flags   exact outside the band |T - L tau| <= 1e-9 max(1, L tau).
"""
from __future__ import annotations

import math

import numpy as np

import oracle

REL_STAT = 1e-12
REL_S = 1e-6
FLAG_BAND = 1e-9


def popcount16(a: np.ndarray) -> int:
    return int(np.unpackbits(np.ascontiguousarray(a, np.uint16).view(np.uint8)).sum())


def compare_codes(codes_gpu: np.ndarray, codes_ref: np.ndarray, amb: np.ndarray):
    """Both [n][L] uint16.  Returns (mismatches outside the margin, ambiguous bits, differing bits)."""
    diff = np.bitwise_xor(codes_gpu, codes_ref)
    outside = np.bitwise_and(diff, np.bitwise_not(amb))
    return popcount16(outside), popcount16(amb), popcount16(diff)


def recount(codes: np.ndarray, K: int) -> np.ndarray:
    """Counts [L][2^K] from codes [n][L] by bincount (independent of both implementations)."""
    n, L = codes.shape
    return np.stack([np.bincount(codes[:, j].astype(np.int64), minlength=1 << K) for j in range(L)])


def rel(a: float, b: float) -> float:
    return abs(a - b) / max(abs(b), 1e-300)


def check_thresh(gpu: dict, ref: dict, keys=("mu", "mu_scored", "sigma", "sigma_table", "tau")):
    for k in keys:
        if ref[k] == 0.0:
            assert abs(gpu[k]) <= 1e-300, (k, gpu[k], ref[k])
        else:
            assert rel(gpu[k], ref[k]) <= REL_STAT, (k, gpu[k], ref[k])
    assert gpu["n"] == ref["n"] and gpu["m_scored"] == ref["m_scored"]


def check_flags(flags_gpu: np.ndarray, flags_ref: np.ndarray, T: np.ndarray, L: int, tau: float):
    lim = L * tau
    band = np.abs(T.astype(np.float64) - lim) <= FLAG_BAND * max(1.0, abs(lim))
    bad = (flags_gpu != flags_ref) & ~band
    assert not bad.any(), f"{int(bad.sum())} flags differ outside the band"
    return int(band.sum())


def full_parity(X: np.ndarray, W: np.ndarray, K: int, L: int, device="cuda", signs=None, **ace_kwargs) -> dict:
    """Insert all rows, score all rows, threshold and flag, on both sides; assert the bar.
    With `signs`, the GPU context uses the structured projection and W is its dense
    equivalent (what the oracle hashes with)."""
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16

    n = X.shape[0]
    codes_o, amb = oracle.hash_codes(X, W, K, L)
    sk = oracle.Sketch(K, L)
    sk.insert_codes(codes_o)
    T_o = sk.score_codes(codes_o)
    rc, th_o = sk.threshold(oracle.MODE_SCORED, 1.0)
    flags_o = sk.flags(T_o, th_o["tau"], oracle.MODE_SCORED)

    if signs is None:
        ace = ACE(W, K, L, **ace_kwargs)
    else:
        ace = ACE(None, K, L, signs=signs, d=X.shape[1], **ace_kwargs)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(device)
    codes_g = codes_as_uint16(ace.hash(Xd))
    bad, n_amb, n_diff = compare_codes(codes_g, codes_o, amb)
    assert bad == 0, f"{bad} code bits differ outside the FP64 margin"

    ace.insert(Xd)
    s_g, T_g = ace.score(Xd)
    th_g = ace.threshold("scored", 1.0)
    flags_g = ace.flag(T_g, th_g["tau"], "scored").cpu().numpy()
    counts_g = ace.counts()
    T_gn = T_g.cpu().numpy().view(np.uint32).astype(np.int64)
    s_gn = s_g.cpu().numpy()

    assert np.array_equal(counts_g.astype(np.int64), recount(codes_g, K)), "counts != recount of GPU codes"
    # T is the sum of the GPU's counts at the GPU's codes, whichever kernel gathered them
    T_own = counts_g.astype(np.int64)[np.arange(L)[None, :], codes_g.astype(np.int64) & ((1 << K) - 1)].sum(axis=1)
    assert np.array_equal(T_gn, T_own), "T != gather of the GPU's counts at its codes"
    S2_g, S3_g = ace.table_stats()
    if n_diff == 0:
        assert np.array_equal(counts_g.astype(np.int64), sk.counts)
        assert np.array_equal(S2_g, sk.S2) and np.array_equal(S3_g, sk.S3)
        assert np.array_equal(T_gn, T_o)
        check_thresh(th_g, th_o)
        band = check_flags(flags_g, flags_o, T_o, L, th_o["tau"])
    else:
        band = -1
    np.testing.assert_allclose(s_gn, T_gn / L, rtol=REL_S, atol=0)
    cnt = ace.counters()
    ace.close()
    return {"n": n, "ambiguous_bits": n_amb, "differing_bits": n_diff, "flag_band": band,
            "bits_refined": cnt["bits_refined"], "bits_flipped": cnt["bits_flipped"],
            "bits_hashed": cnt["bits_hashed"], "flagged": int(flags_g.sum()), "mu": th_g["mu"],
            "sigma": th_g["sigma"], "tau": th_g["tau"]}


def adversarial_rows(X: np.ndarray, W: np.ndarray, n_near: int, n_cancel: int, seed: int) -> np.ndarray:
    """Rows built to sit near the sign boundary of chosen projection columns:
    - near-orthogonal: a data row with its component along column c removed (in FP64,
      then rounded to FP32), so w_c^T x is tiny;
    - cancelling: two large terms x_i w_ic = 1 and x_j w_jc = -1 plus noise of 1e-3 on the
      other coordinates, so the running sum passes through magnitudes far above |w_c^T x|.
    Returns the rows appended to X (float32)."""
    rng = np.random.default_rng(seed)
    n, d = X.shape
    ncol = W.shape[1]
    out = [X]
    near = []
    for _ in range(n_near):
        y = X[rng.integers(0, n)].astype(np.float64)
        c = rng.integers(0, ncol)
        w = W[:, c].astype(np.float64)
        near.append(y - (y @ w) / (w @ w) * w)
    if near:
        out.append(np.array(near, np.float32))
    canc = []
    if d >= 2:
        for _ in range(n_cancel):
            c = rng.integers(0, ncol)
            w = W[:, c].astype(np.float64)
            i, j = rng.choice(d, 2, replace=False)
            x = rng.standard_normal(d) * 1e-3
            x[i] = 1.0 / w[i]
            x[j] = -1.0 / w[j]
            canc.append(x)
        out.append(np.array(canc, np.float32))
    return np.concatenate(out, axis=0).astype(np.float32)


def fp32_bound(X: np.ndarray, W: np.ndarray, model: str) -> np.ndarray:
    """The FP32-mode refinement bound gamma_h(u) ||x|| ||w|| the library states.  Rows of
    2048 or more values (128 or more 16-wide k blocks) are hashed with k split four ways:
    chains of at most P = 16 ceil(nfull/4) + 16 products plus two roundings to add the
    four partial sums."""
    d = X.shape[1]
    DP = -(-d // 32) * 32
    nfull = d // 16
    if nfull >= 128:
        P = 16 * (-(-nfull // 4)) + 16
        h, u = (2 * P + 10, 2.0 ** -23) if model == "generic" else (P + 6, 2.0 ** -24)
    else:
        h, u = (2 * DP + 8, 2.0 ** -23) if model == "generic" else (DP + 4, 2.0 ** -24)
    gam = h * u / (1 - h * u)
    return gam * np.linalg.norm(X.astype(np.float64), axis=1)[:, None] * \
        np.linalg.norm(W.astype(np.float64), axis=0)[None, :]


def raw_flip_report(codes_gpu: np.ndarray, P: np.ndarray, bound: np.ndarray, K: int, L: int) -> dict:
    """Compare raw GPU bits with FP64 signs; every differing bit must lie inside `bound`."""
    ref = P > 0
    flips = viol = 0
    worst = 0.0
    for j in range(L):
        for k in range(K):
            c = j * K + k
            gbit = ((codes_gpu[:, j] >> k) & 1).astype(bool)
            diff = gbit != ref[:, c]
            flips += int(diff.sum())
            if diff.any():
                ratio = np.abs(P[diff, c]) / bound[diff, c]
                worst = max(worst, float(ratio.max()))
                viol += int((ratio > 1).sum())
    return {"raw_flips": flips, "violations": viol, "worst_ratio": worst,
            "raw_flip_rate": flips / (codes_gpu.shape[0] * K * L)}
