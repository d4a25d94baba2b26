"""16-bit saturating counters (the short counters of Sec. 3.4) vs the oracle (needs the GPU).

Below 65535 points per bucket the 16-bit context must equal the 32-bit one exactly.  Past
it, every count must equal the oracle's saturating count min(true count, 65535), with S2,
S3, the dropped increments, the scores and the thresholds following the stored counts.
"""
import numpy as np
import pytest

import oracle
from ace_inputs import c2_points, gaussian_clusters, projection_matrix
from tests.parity import check_thresh, full_parity, recount

pytestmark = pytest.mark.gpu

CAP = 65535


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(m):
    print(m, flush=True)


@pytest.mark.parametrize("n,d,K,L,prec", [(1000, 16, 10, 20, "fp32"), (3000, 120, 15, 50, "fp32"),
                                          (777, 33, 16, 7, "bf16"), (5, 8, 12, 3, "fp32")])
def test_c16_parity_below_cap(n, d, K, L, prec):
    X, _ = gaussian_clusters(n, d, 3, 0.05, seed=n + d)
    W = projection_matrix(d, K, L, 40 + n)
    r = full_parity(X, W, K, L, precision=prec, counter_bits=16)
    _say((n, d, K, L, r))


def test_c16_connection_log_sample():
    X, _ = c2_points(n=30_000, seed=14)
    W = projection_matrix(120, 15, 50, 1706066642)
    _say(full_parity(X, W, 15, 50, counter_bits=16))


def _saturating_workload():
    """200,000 rows in 3 tight clusters: at K = 4 the cluster buckets pass 65535."""
    rng = np.random.default_rng(31)
    d, K, L = 8, 4, 8
    centers = rng.standard_normal((3, d)) * 4.0
    which = rng.choice(3, size=200_000, p=[0.6, 0.3, 0.1])
    X = (centers[which] + 0.05 * rng.standard_normal((200_000, d))).astype(np.float32)
    W = projection_matrix(d, K, L, 77)
    return X, W, K, L


def test_c16_saturation_matches_capped_oracle():
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16
    X, W, K, L = _saturating_workload()
    codes_o, amb = oracle.hash_codes(X, W, K, L)
    assert not amb.any()
    sk = oracle.Sketch(K, L, cap=CAP)
    ace = ACE(W, K, L, counter_bits=16)
    Xd = torch.from_numpy(X).cuda()
    # one large insert (LDS histogram path), then small ones (one atomic per row and table)
    parts = [(0, 199_000)] + [(199_000 + 5 * i, 199_000 + 5 * i + 5) for i in range(200)]
    for a, b in parts:
        ace.insert(Xd[a:b])
        sk.insert_codes(codes_o[a:b])
    cg = codes_as_uint16(ace.hash(Xd))
    assert np.array_equal(cg, codes_o)
    true = recount(codes_o, K)
    assert (true > CAP).any(), "workload must saturate"
    counts = ace.counts().astype(np.int64)
    assert np.array_equal(counts, np.minimum(true, CAP))
    assert np.array_equal(counts, sk.counts)
    S2, S3 = ace.table_stats()
    assert np.array_equal(S2, sk.S2) and np.array_equal(S3, sk.S3)
    cnt = ace.counters()
    assert cnt["saturated_increments"] == sk.dropped == int(np.maximum(true - CAP, 0).sum())
    _, T = ace.score(Xd[::97].contiguous())
    T_o = sk.score_codes(codes_o[::97])
    assert np.array_equal(T.cpu().numpy().view(np.uint32).astype(np.int64), T_o)
    check_thresh(ace.threshold("scored", 1.0), sk.threshold(oracle.MODE_SCORED, 1.0)[1])
    check_thresh(ace.threshold("const", 1.0), sk.threshold(oracle.MODE_CONST, 1.0)[1],
                 keys=("mu", "sigma_table", "tau"))
    _say({"dropped": cnt["saturated_increments"], "max_true": int(true.max())})
    ace.reset()
    assert ace.counters()["saturated_increments"] == 0 and ace.counts().max() == 0
    ace.close()


def test_c16_delete_and_underflow():
    import torch
    from paper_1706_06664_amd import ACE, AceError
    X, _ = gaussian_clusters(4000, 16, 3, 0.05, seed=5)
    W = projection_matrix(16, 12, 10, 6)
    codes_o, _ = oracle.hash_codes(X, W, 12, 10)
    ace = ACE(W, 12, 10, counter_bits=16)
    Xd = torch.from_numpy(X).cuda()
    ace.insert(Xd)
    ace.delete(Xd[:1500])
    sk = oracle.Sketch(12, 10, cap=CAP)
    sk.insert_codes(codes_o)
    assert sk.delete_codes(codes_o[:1500]) == 0
    assert np.array_equal(ace.counts().astype(np.int64), sk.counts)
    S2, S3 = ace.table_stats()
    assert np.array_equal(S2, sk.S2) and np.array_equal(S3, sk.S3)
    ace.close()
    # deleting a row whose bucket is empty in some table drives a count below zero: the
    # count is clamped at zero and the context reports ACE_E_STATE from then on
    ace = ACE(W, 12, 10, counter_bits=16)
    ace.insert(Xd[:10])
    neg = -Xd[:1]
    c_neg, _ = oracle.hash_codes(-X[:1], W, 12, 10)
    occupied = [set(codes_o[:10, j].tolist()) for j in range(10)]
    assert any(int(c_neg[0, j]) not in occupied[j] for j in range(10))
    ace.delete(neg.contiguous())
    with pytest.raises(AceError) as e:
        ace.counts()
    assert e.value.status == 6
    ace.close()


def test_c16_checkpoint_roundtrip():
    import torch
    from paper_1706_06664_amd import ACE, AceError
    X, W, K, L = _saturating_workload()
    a = ACE(W, K, L, counter_bits=16)
    a.insert(torch.from_numpy(X).cuda())
    counts = a.counts()
    S2, S3 = a.table_stats()
    b = ACE(W, K, L, counter_bits=16)
    b.set_counts(counts, X.shape[0])
    S2b, S3b = b.table_stats()
    assert np.array_equal(b.counts(), counts) and np.array_equal(S2b, S2) and np.array_equal(S3b, S3)
    bad = counts.copy()
    bad[0, 0] = CAP + 1
    with pytest.raises(AceError):
        b.set_counts(bad, X.shape[0])
    with pytest.raises(AceError):   # a table summing to more than n
        b.set_counts(counts, int(counts[0].sum()) - 1)
    a.close()
    b.close()
