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


def full_parity(X: np.ndarray, W: np.ndarray, K: int, L: int, device="cuda", **ace_kwargs) -> dict:
    """Insert all rows, score all rows, threshold and flag, on both sides; assert the bar."""
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16

    n = X.shape[0]
    codes_o, amb = oracle.hash_codes(X, W, K, L)
    sk = oracle.Sketch(K, L)
    sk.insert_codes(codes_o)
    T_o = sk.score_codes(codes_o)
    rc, th_o = sk.threshold(oracle.MODE_SCORED, 1.0)
    flags_o = sk.flags(T_o, th_o["tau"], oracle.MODE_SCORED)

    ace = ACE(W, K, L, **ace_kwargs)
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
