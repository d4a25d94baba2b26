"""HIP path vs the oracle, element by element, through the C ABI (needs the GPU)."""
import numpy as np
import pytest

import oracle
from ace_inputs import c1_points, c2_points, projection_matrix, gaussian_clusters
from tests.parity import compare_codes, full_parity, recount

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1706_06664_amd import load_library
    load_library()


def _say(msg):
    print(msg, flush=True)


def test_mfma_layout_small():
    """One row tile, one table, FP32: tiny case checks operand and output lane layout."""
    rng = np.random.default_rng(100)
    X = rng.standard_normal((16, 4)).astype(np.float32)
    W = rng.standard_normal((4, 16)).astype(np.float32)
    r = full_parity(X, W, 16, 1)
    _say(r)


def test_parity_small_clusters():
    """Clustered workload at 10,000 x 32, K=10, L=20, FP32 (all rows, all stats)."""
    X, _ = c1_points()
    W = projection_matrix(32, 10, 20, 1706066641)
    r = full_parity(X, W, 10, 20)
    _say(r)
    assert r["differing_bits"] == 0


@pytest.mark.parametrize("n,d,K,L", [
    (1, 5, 1, 1), (127, 33, 15, 3), (129, 120, 15, 50), (300, 7, 16, 4), (1000, 64, 10, 64),
    (777, 1, 4, 100), (2048, 32, 12, 9), (515, 130, 16, 13),
    # d % 4 == 0 with every remainder of d mod 16 (last k block of 4, 8 or 12 values, d < 16)
    (300, 4, 8, 5), (257, 8, 15, 21), (130, 12, 16, 3), (333, 100, 15, 10), (200, 24, 13, 30),
    (64, 44, 16, 7), (1100, 16, 15, 50),
    # 128+ k blocks: k split four ways over a workgroup's waves (every d mod 16 remainder)
    (300, 2048, 15, 11), (257, 2052, 16, 9), (129, 2056, 12, 13), (200, 2060, 16, 5), (70, 4100, 16, 20),
])
def test_parity_shapes(n, d, K, L):
    X, _ = gaussian_clusters(n, d, 3, 0.05, seed=n + d)
    W = projection_matrix(d, K, L, 7 + n)
    r = full_parity(X, W, K, L)
    _say((n, d, K, L, r))


def test_parity_chunked_and_unaligned():
    """max_batch_rows forces several chunks; an offset view makes rows unaligned (scalar loads)."""
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16
    X, _ = gaussian_clusters(2501, 36, 4, 0.02, seed=3)
    W = projection_matrix(36, 15, 50, 11)
    r = full_parity(X, W, 15, 50, max_batch_rows=1000)
    _say(r)
    big = torch.from_numpy(np.concatenate([np.zeros(1, np.float32), X.ravel()])).cuda()
    Xoff = big[1:].view(2501, 36)
    assert Xoff.data_ptr() % 16 != 0
    ace = ACE(W, 15, 50, max_batch_rows=1000)
    cg = codes_as_uint16(ace.hash(Xoff))
    co, amb = oracle.hash_codes(X, W, 15, 50)
    bad, _, _ = compare_codes(cg, co, amb)
    assert bad == 0


def test_zero_rows_identical_rows_near_orthogonal():
    """Degenerate inputs: zero rows (every projection exactly 0, all refined, code 0);
    identical rows (one hot bucket per table); rows orthogonal to chosen columns
    before rounding (tiny projections decided by the FP64 tier)."""
    rng = np.random.default_rng(5)
    d, K, L = 24, 15, 8
    W = projection_matrix(d, K, L, 99)
    zero = np.zeros((200, d), np.float32)
    same = np.repeat(rng.standard_normal((1, d)).astype(np.float32), 3000, axis=0)
    near = []
    for i in range(500):
        y = rng.standard_normal(d)
        c = rng.integers(0, K * L)
        w = W[:, c].astype(np.float64)
        near.append((y - (y @ w) / (w @ w) * w).astype(np.float32))
    X = np.concatenate([zero, same, np.array(near)], axis=0)
    r = full_parity(X, W, K, L)
    _say(r)
    assert r["bits_refined"] >= 200 * K * L


@pytest.mark.parametrize("model", ["measured", "generic"])
@pytest.mark.parametrize("long_rows", [False, True], ids=["d120", "d2056_split_k"])
def test_refine_off_respects_bound(model, long_rows):
    """Raw FP32 MFMA signs (refine off) may differ from the FP64 signs only where |p64|
    is inside the library's stated FP32 bound for the error model (for 2056-wide rows, the
    bound of the split-k kernel)."""
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16
    from tests.parity import adversarial_rows, fp32_bound, raw_flip_report
    if long_rows:
        K, L = 16, 20
        X0, _ = gaussian_clusters(1500, 2056, 4, 0.3, seed=8)
    else:
        K, L = 15, 50
        X0, _ = c2_points(n=4000, seed=8)
    W = projection_matrix(X0.shape[1], K, L, 4)
    X = adversarial_rows(X0, W, 3000, 3000, seed=8)
    ace = ACE(W, K, L, refine=False, bound=model)
    cg = codes_as_uint16(ace.hash(torch.from_numpy(X).cuda()))
    P, _ = oracle.project(X, W)
    rep = raw_flip_report(cg, P, fp32_bound(X, W, model), K, L)
    _say(rep)
    assert rep["violations"] == 0


def test_delete_matches_oracle():
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16
    X, _ = gaussian_clusters(6000, 20, 5, 0.01, seed=21)
    K, L = 12, 16
    W = projection_matrix(20, K, L, 21)
    drop = np.random.default_rng(1).permutation(6000)[:2500]
    ace = ACE(W, K, L)
    Xd = torch.from_numpy(X).cuda()
    ace.insert(Xd)
    ace.delete(Xd[torch.from_numpy(drop).cuda()].contiguous())
    co, amb = oracle.hash_codes(X, W, K, L)
    sk = oracle.Sketch(K, L)
    sk.insert_codes(co)
    assert sk.delete_codes(co[drop]) == 0
    assert np.array_equal(ace.counts().astype(np.int64), sk.counts)
    S2, S3 = ace.table_stats()
    assert np.array_equal(S2, sk.S2) and np.array_equal(S3, sk.S3)
    th = ace.threshold("const", 1.0)
    rc, tho = sk.threshold(oracle.MODE_CONST, 1.0)
    assert th["n"] == 3500 and abs(th["mu"] - tho["mu"]) <= 1e-12 * tho["mu"]


def test_codes_entry_points_and_checkpoint():
    import torch
    from paper_1706_06664_amd import ACE
    X, _ = gaussian_clusters(4000, 16, 3, 0.01, seed=31)
    K, L = 11, 10
    W = projection_matrix(16, K, L, 31)
    a = ACE(W, K, L)
    Xd = torch.from_numpy(X).cuda()
    codes = a.hash(Xd)
    a.insert_codes(codes)
    s1, T1 = a.score_codes(codes)
    b = ACE(W, K, L)
    b.set_counts(a.counts(), 4000)
    s2, T2 = b.score(Xd)
    assert torch.equal(T1, T2)
    S2a, S3a = a.table_stats()
    S2b, S3b = b.table_stats()
    assert np.array_equal(S2a, S2b) and np.array_equal(S3a, S3b)


def test_threshold_mean_past_int64():
    """sum_j S2_j beyond 2^63 (Eq. dynadd's mean from the counts): n = INT32_MAX identical
    points in L = 4 tables put n in one bucket of each, S2_j = n^2, sum_j S2_j = 4 n^2 > 2^63.
    Every point scores n, so mu = n, and each table's count variance is 0."""
    from paper_1706_06664_amd import ACE
    K, L, d = 1, 4, 8
    n = 2 ** 31 - 1
    a = ACE(projection_matrix(d, K, L, 3), K, L)
    counts = np.zeros((L, 2), np.int32)
    counts[:, 1] = n
    a.set_counts(counts, n)
    S2, _ = a.table_stats()
    assert [int(v) for v in S2] == [n * n] * L and L * n * n > 2 ** 63
    th = a.threshold("const", 1.0)
    assert th["n"] == n
    assert abs(th["mu"] - n) <= 1e-12 * n, th["mu"]
    assert th["sigma_table"] == 0.0
    assert abs(th["tau"] - (n - 1)) <= 1e-12 * n
    a.close()


def test_error_paths():
    import torch
    from paper_1706_06664_amd import ACE, AceError
    W = projection_matrix(8, 6, 4, 1)
    torch.manual_seed(0)
    X = torch.randn(100, 8, device="cuda")
    a = ACE(W, 6, 4)
    with pytest.raises(AceError) as e:
        a.threshold("scored")
    assert e.value.status == 4                      # ACE_E_EMPTY
    import paper_1706_06664_amd.ace as m
    assert a.lib.ace_debug_set_capacity(a.h, 150) == 0
    a.insert(X)
    with pytest.raises(AceError) as e:
        a.insert(X)
    assert e.value.status == 3                      # ACE_E_OVERFLOW, nothing enqueued
    assert a.counts().sum() == 100 * 4
    assert a.lib.ace_debug_fail_next(a.h) == 0
    with pytest.raises(AceError) as e:
        a.score(X)
    assert e.value.status == 5                      # ACE_E_DEVICE ...
    with pytest.raises(AceError) as e:
        a.threshold("const")
    assert e.value.status == 5                      # ... and sticky
    with pytest.raises(AceError) as e:
        ACE(W, 6, 4, mem_budget=1000)
    assert e.value.status == 2                      # ACE_E_NOMEM
    b = ACE(W, 6, 4)
    with pytest.raises(AceError) as e:
        b.delete(X[:3].contiguous())
    assert e.value.status == 6                      # ACE_E_STATE: more deletes than points
    b.insert(X[:10].contiguous())
    b.delete(X[50:53].contiguous())                 # never inserted: a bucket goes below zero
    with pytest.raises(AceError) as e:
        b.threshold("const")
    assert e.value.status == 6


@pytest.mark.timeout(600)
def test_parity_connection_log_full():
    """Full connection-log workload: 494,021 x 120, K=15, L=50, FP32."""
    X, _ = c2_points()
    W = projection_matrix(120, 15, 50, 1706066642)
    r = full_parity(X, W, 15, 50)
    _say(r)


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp8"])
def test_refine_queue_full_path(precision):
    """With the queue cut to 0 or 10 entries nearly every uncertain projection is decided
    inside the projection kernel; codes, refine counts and refined masks must match."""
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16
    rng = np.random.default_rng(6)
    d, K, L = 40, 16, 6
    W = projection_matrix(d, K, L, 98)
    zero = np.zeros((64, d), np.float32)
    near = []
    for i in range(700):
        y = rng.standard_normal(d)
        c = rng.integers(0, K * L)
        w = W[:, c].astype(np.float64)
        near.append((y - (y @ w) / (w @ w) * w).astype(np.float32))
    X = np.concatenate([zero, np.array(near), rng.standard_normal((300, d)).astype(np.float32)], axis=0)
    Xd = torch.from_numpy(X).cuda()
    co, amb = oracle.hash_codes(X, W, K, L)
    res = []
    for q in (0, 10):
        ace = ACE(W, K, L, precision=precision)
        assert ace.lib.ace_debug_set_refine_queue(ace.h, q) == 0
        cg, ref = ace.hash(Xd, want_refined=True)
        cg = codes_as_uint16(cg)
        bad, _, _ = compare_codes(cg, co, amb)
        assert bad == 0
        res.append((cg, ace.counters()["bits_refined"], codes_as_uint16(ref)))
        # zero rows: every bit refined, and marked so whether queued or decided in place
        assert np.all(res[-1][2][:64] == (1 << K) - 1)
    assert np.array_equal(res[0][0], res[1][0])
    assert res[0][1] == res[1][1] and res[0][1] >= 64 * K * L
    assert np.array_equal(res[0][2], res[1][2])
    # The query phase with the same short queues (the FP32 kernel gathers the counts of the
    # codes it decided in place, and leaves rows with queued bits for the full gather).
    T_ref = None
    for q in (0, 10):
        ace = ACE(W, K, L, precision=precision)
        assert ace.lib.ace_debug_set_refine_queue(ace.h, q) == 0
        ace.insert(Xd)
        _, T = ace.score(Xd)
        T = T.cpu().numpy().view(np.uint32).astype(np.int64)
        cg = res[0][0].astype(np.int64)
        own = ace.counts().astype(np.int64)[np.arange(L)[None, :], cg].sum(axis=1)
        assert np.array_equal(T, own)
        if T_ref is not None:
            assert np.array_equal(T, T_ref)
        T_ref = T
        ace.close()


@pytest.mark.parametrize("bits", [32, 16])
@pytest.mark.parametrize("n", [131_071, 131_072, 200_003])
def test_score_large_batches_from_codes(bits, n):
    """Scoring batches of 131,072 rows or more takes the table-by-table kernel (two rows per
    thread).  Codes with hot buckets (a quarter of the rows share one code per table) are
    inserted and scored through ace_insert_codes / ace_score_codes and compared with the
    oracle: every T, s, the counts and the scored-set statistics; odd n leaves the last
    thread's second row out."""
    import torch
    from paper_1706_06664_amd import ACE
    from tests.parity import check_thresh
    K, L = 13, 37
    rng = np.random.default_rng(n + bits)
    codes = rng.integers(0, 1 << K, size=(n, L), dtype=np.int64).astype(np.uint16)
    codes[: n // 4] = codes[0]
    sk = oracle.Sketch(K, L, cap=65535 if bits == 16 else None)
    sk.insert_codes(codes)
    T_o = sk.score_codes(codes)
    _, th_o = sk.threshold(oracle.MODE_SCORED, 1.0)
    ace = ACE(projection_matrix(8, K, L, 5), K, L, counter_bits=bits)
    cd = torch.from_numpy(codes.T.copy().view(np.int16)).to("cuda:0")
    ace.insert_codes(cd)
    s, T = ace.score_codes(cd)
    np.testing.assert_array_equal(T.cpu().numpy().astype(np.int64), T_o)
    np.testing.assert_allclose(s.cpu().numpy(), T_o / L, rtol=1e-6, atol=0)
    assert np.array_equal(ace.counts().astype(np.int64), sk.counts)
    check_thresh(ace.threshold("scored", 1.0), th_o)
    ace.close()


@pytest.mark.parametrize("K,L,bits,chunk", [(15, 50, 32, 0), (16, 7, 32, 1000), (12, 13, 16, 0), (10, 3, 32, 333)])
def test_score_matches_codes_path(K, L, bits, chunk):
    """ace_score (hash, FP64 pass, gather per chunk) against ace_score_codes on the same codes
    in a second context with the same counts: every T and s, and the scored-set statistics
    (per-block moments reduced in one more block above 64 blocks, atomics below).  Zero rows
    (every bit refined), near-orthogonal rows (some refined bits), random rows; ragged n,
    16-bit counters, several chunks."""
    import torch
    from paper_1706_06664_amd import ACE, codes_as_uint16
    from tests.parity import check_thresh
    rng = np.random.default_rng(K * 1000 + L)
    d = 36
    W = projection_matrix(d, K, L, K + L)
    zero = np.zeros((97, d), np.float32)
    near = []
    for _ in range(600):
        y = rng.standard_normal(d)
        c = rng.integers(0, K * L)
        w = W[:, c].astype(np.float64)
        near.append((y - (y @ w) / (w @ w) * w).astype(np.float32))
    X = np.concatenate([rng.standard_normal((23450, d)).astype(np.float32), zero, np.array(near),
                        rng.standard_normal((1789, d)).astype(np.float32)], axis=0)
    Xd = torch.from_numpy(X).cuda()
    kw = dict(counter_bits=bits, max_batch_rows=chunk)
    a = ACE(W, K, L, **kw)
    b = ACE(W, K, L, **kw)
    a.insert(Xd)
    b.insert(Xd)
    s_a, T_a = a.score(Xd)
    codes = b.hash(Xd)
    s_b, T_b = b.score_codes(codes)
    assert a.counters()["bits_refined"] >= 97 * K * L
    assert torch.equal(T_a, T_b)
    assert torch.equal(s_a, s_b)
    cg = codes_as_uint16(codes).astype(np.int64)
    own = a.counts().astype(np.int64)[np.arange(L)[None, :], cg].sum(axis=1)
    Tn = T_a.cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(Tn, own)
    ta, tb = a.threshold("scored", 1.0), b.threshold("scored", 1.0)
    check_thresh(ta, tb)
    # the moments themselves, from T on the host
    import math
    n = len(Tn)
    Ti = [int(v) for v in Tn]
    S1, S2 = sum(Ti), sum(v * v for v in Ti)
    mu = S1 / (n * L)
    sd = math.sqrt(n * S2 - S1 * S1) / (n * L)
    assert ta["m_scored"] == n
    assert abs(ta["mu_scored"] - mu) <= 1e-12 * mu and abs(ta["sigma"] - sd) <= 1e-9 * sd
    a.close()
    b.close()


def test_table_stats_past_2p21_counts():
    """S2_j = sum_b A_j[b]^2 and S3_j = sum_b A_j[b]^3 (the exact sums behind mu and sigma_table,
    Eq. dynadd / dynsub) when one bucket per table grows past 2^21 (its cube past 2^63:
    the update's 128-bit branch) and shrinks back below it by deletion (Sec. 3.4.1), with
    small buckets beside it: against Python integers from the counts."""
    import torch
    from paper_1706_06664_amd import ACE
    K, L, d = 4, 3, 8
    rng = np.random.default_rng(77)
    W = projection_matrix(d, K, L, 77)
    hot = rng.standard_normal((1, d)).astype(np.float32)
    rest = rng.standard_normal((300_000, d)).astype(np.float32)
    ace = ACE(W, K, L)
    hot_d = torch.from_numpy(hot).cuda().expand(2_200_000, d).contiguous()

    def check():
        counts = ace.counts().astype(np.int64)
        S2, S3 = ace.table_stats()
        for j in range(L):
            c = [int(v) for v in counts[j]]
            assert int(S2[j]) == sum(v * v for v in c)
            s3 = sum(v ** 3 for v in c)
            assert int(S3[j][0]) | (int(S3[j][1]) << 64) == s3
        return counts

    ace.insert(torch.cat([hot_d[:1_500_000], torch.from_numpy(rest).cuda()]))
    c1 = check()
    assert (c1.max(axis=1) >= 1_500_000).all() and (c1.max(axis=1) < (1 << 21)).all()
    ace.insert(hot_d[1_500_000:])
    c2 = check()
    assert (c2.max(axis=1) >= 2_200_000).all() and (c2.max(axis=1) > (1 << 21)).all()
    ace.delete(hot_d[:500_000])
    c3 = check()
    assert (c3.max(axis=1) < (1 << 21)).all()
    assert c3.sum() == L * 2_000_000
    ace.close()


def test_threshold_flag_matches_separate_calls():
    """ace_threshold_flag (threshold and flags enqueued together, Alg. 1 / Sec. 5.3
    reporting) against ace_threshold then ace_flag with the returned tau, in every mode; on
    an empty set it returns ACE_E_EMPTY and flags nothing."""
    import ctypes
    import torch
    from paper_1706_06664_amd import ACE, AceError
    import paper_1706_06664_amd.ace as m
    X, _ = gaussian_clusters(20_000, 24, 4, 0.05, seed=41)
    K, L = 12, 20
    W = projection_matrix(24, K, L, 41)
    a = ACE(W, K, L)
    Xd = torch.from_numpy(X).cuda()
    a.insert(Xd)
    _, T = a.score(Xd)
    for mode in ("scored", "const", "table"):
        th1 = a.threshold(mode, 1.0)
        f1 = a.flag(T, th1["tau"], mode)
        f2, th2 = a.threshold_flag(T, mode, 1.0)
        assert th1 == th2
        assert torch.equal(f1, f2)
        assert 0 < int(f2.sum()) < T.shape[0]
    b = ACE(W, K, L)
    flags = torch.ones(T.shape[0], dtype=torch.uint8, device="cuda")
    out = m.Thresh()
    st = b.lib.ace_threshold_flag(b.h, m.THR_SCORED, 1.0, T.data_ptr(), T.shape[0], flags.data_ptr(), None,
                                  ctypes.byref(out))
    assert st == 4                                   # ACE_E_EMPTY
    assert int(flags.sum()) == 0
    with pytest.raises(AceError) as e:
        b.threshold_flag(T, "const", 1.0)
    assert e.value.status == 4
    a.close()
    b.close()


def test_reset_clears_every_sum():
    """ace_reset (one launch for the counts and the small sums): counts, S2/S3, the scored
    set and n all return to zero, and a context reset and refilled equals a fresh one."""
    import torch
    from paper_1706_06664_amd import ACE, AceError
    X, _ = gaussian_clusters(30_000, 16, 3, 0.05, seed=43)
    K, L = 13, 9
    W = projection_matrix(16, K, L, 43)
    Xd = torch.from_numpy(X).cuda()
    a = ACE(W, K, L)
    a.insert(Xd)
    a.score(Xd)
    a.reset()
    assert int(np.abs(a.counts()).sum()) == 0
    S2, S3 = a.table_stats()
    assert not S2.any() and not S3.any()
    with pytest.raises(AceError) as e:
        a.threshold("const", 1.0)
    assert e.value.status == 4
    with pytest.raises(AceError) as e:
        a.threshold("scored", 1.0)
    assert e.value.status == 4
    a.insert(Xd[:20_000].contiguous())
    s_a, T_a = a.score(Xd)
    b = ACE(W, K, L)
    b.insert(Xd[:20_000].contiguous())
    s_b, T_b = b.score(Xd)
    assert np.array_equal(a.counts(), b.counts())
    assert torch.equal(T_a, T_b)
    assert a.threshold("scored", 1.0) == b.threshold("scored", 1.0)
    a.close()
    b.close()
