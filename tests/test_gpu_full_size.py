"""Parity at the full benchmark sizes, in the launch configuration the benchmark times
(needs the GPU; large: about a minute in all).

The oracle cannot hash millions of rows in seconds, so at these sizes the checks are:
  - codes of sampled rows (the first, the last and a seeded random set) equal the
    oracle's outside its FP64 margin;
  - the counts equal a recount of the GPU's own codes (per-table bincount);
  - T of sampled rows equals the sum of the counts at their codes;
  - mu and sigma equal their definitions, evaluated here from the counts and all T with
    exact integers.
"""
import math

import numpy as np
import pytest

import oracle
from tests.parity import compare_codes

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(m):
    print(m, flush=True)


def _sample(n, m, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([np.arange(64), np.arange(n - 64, n), rng.integers(0, n, m)]))


def _full_check(Xd, W, K, L, W_oracle=None, sample=1500, **ace_kwargs):
    import torch
    from paper_1706_06664_amd import ACE
    n = Xd.shape[0]
    ace = ACE(W, K, L, **ace_kwargs) if W is not None else ACE(None, K, L, d=Xd.shape[1], **ace_kwargs)
    codes = ace.hash(Xd)                                      # int16 [L][n] on the device
    idx = _sample(n, sample, seed=n % 1000)
    idx_t = torch.from_numpy(idx).to(Xd.device)
    Xs = Xd[idx_t].cpu().numpy()
    co, amb = oracle.hash_codes(Xs, W if W is not None else W_oracle, K, L)
    cg = codes[:, idx_t].cpu().numpy().view(np.uint16).T
    bad, n_amb, n_diff = compare_codes(cg, co, amb)
    assert bad == 0, f"{bad} sampled code bits differ outside the FP64 margin"

    ace.insert(Xd)
    s, T = ace.score(Xd)
    th = ace.threshold("scored", 1.0)
    counts = torch.from_numpy(ace.counts()).to(Xd.device).long()
    cu = codes.long() & 0xFFFF
    for j in range(L):
        rc = torch.bincount(cu[j], minlength=1 << K)
        assert torch.equal(rc, counts[j]), f"table {j}: counts != recount of the GPU codes"
    Tsum = counts.gather(1, cu[:, idx_t]).sum(dim=0)
    Tg = T[idx_t].long() & 0xFFFFFFFF
    assert torch.equal(Tsum, Tg), "sampled T != sum of the counts at their codes"
    # mu = sum_j sum_b A_j[b]^2 / (n L); sigma of the scored set from exact integer moments
    S2 = int((counts * counts).sum().item())
    assert abs(th["mu"] - S2 / (n * L)) <= 1e-12 * th["mu"]
    Tall = (T.long() & 0xFFFFFFFF).cpu().numpy()
    sT = int(Tall.sum())
    sq = Tall.astype(np.uint64) ** 2                          # each < 2^63
    sq = np.concatenate([sq, np.zeros((-sq.size) % 64, np.uint64)])
    sT2 = sum(int(v) for v in sq.reshape(-1, 64).sum(axis=1, dtype=np.uint64))   # chunk sums < 2^64
    sigma = math.sqrt(n * sT2 - sT * sT) / (n * L)
    assert abs(th["sigma"] - sigma) <= 1e-12 * sigma
    np.testing.assert_allclose(s[idx_t].cpu().numpy(), Tg.cpu().numpy() / L, rtol=1e-6, atol=0)
    cnt = ace.counters()
    ace.close()
    return {"n": n, "sampled_rows": int(idx.size), "ambiguous_bits": n_amb, "differing_bits": n_diff,
            "refined_frac": cnt["bits_refined"] / max(1, cnt["bits_hashed"]), "mu": th["mu"], "sigma": th["sigma"]}


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_low_rank_4m_x_1024(prec):
    import torch
    from ace_inputs import low_rank_points_torch, projection_matrix
    Xd, _ = low_rank_points_torch(4_000_000, 1024, seed=3, device="cuda")
    W = projection_matrix(1024, 15, 64, 1706066643)
    r = _full_check(Xd, W, 15, 64, precision=prec)
    _say((prec, r))
    del Xd
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "structured"])
def test_heavy_tail_1m_x_4096(prec):
    import torch
    from ace_inputs import heavy_tail_points_torch, projection_matrix, structured_signs
    Xd, _ = heavy_tail_points_torch(1_000_000, 4096, seed=4, device="cuda")
    if prec == "structured":
        from oracle.structured import structured_matrix
        signs, _ = structured_signs(4096, 16, 100, 1706066647)
        r = _full_check(Xd, None, 16, 100, W_oracle=structured_matrix(signs, 4096, 16, 100), sample=600,
                        signs=signs)
    else:
        W = projection_matrix(4096, 16, 100, 1706066644)
        r = _full_check(Xd, W, 16, 100, sample=600, precision=prec)
    _say((prec, r))
    del Xd
    torch.cuda.empty_cache()
