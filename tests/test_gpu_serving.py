"""Serving loop vs a sequential oracle replay (needs the GPU).

Requests are admitted onto several streams at once, yet every score must equal the one the
oracle computes when it replays the log one request at a time in admission order (a score
sees exactly the inserts admitted before it).  The same trace run with 1 slot and with many
slots must therefore give identical results.
"""
import numpy as np
import pytest

import oracle
from ace_inputs import projection_matrix, serving_trace

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(m):
    print(m, flush=True)


def _records(kind, n, row0, out0, t):
    from paper_1706_06664_amd import REQUEST_DTYPE
    r = np.zeros(len(kind), REQUEST_DTYPE)
    r["kind"], r["n"], r["row0"], r["out0"], r["t_arrival_s"] = kind, n, row0, out0, t
    return r


def _oracle_replay(kind, n, row0, out0, pool, W, K, L):
    """Sequential replay: hash every row once, then insert / score / delete request by
    request."""
    codes, amb = oracle.hash_codes(pool, W, K, L)
    sk = oracle.Sketch(K, L)
    T = np.zeros(int(n[kind == 1].sum()), np.int64)
    for r in range(len(kind)):
        c = codes[row0[r]:row0[r] + n[r]]
        if kind[r] == 0:
            sk.insert_codes(c)
        elif kind[r] == 2:
            assert sk.delete_codes(c) == 0
        else:
            T[out0[r]:out0[r] + n[r]] = sk.score_codes(c)
    return T, sk, int(np.count_nonzero(amb))


def _window_trace(nreq, d, window, seed):
    """A serving trace with a sliding window: every insert's rows are deleted again once
    `window` further requests of the trace have been admitted (Eq. dynsub)."""
    kind, n, row0, out0, t, pool = serving_trace(nreq, d, seed=seed, median_batch=32, max_batch=1024)
    k2, n2, r2, o2, due = [], [], [], [], []
    for r in range(nreq):
        k2.append(kind[r]); n2.append(n[r]); r2.append(row0[r]); o2.append(out0[r])
        if kind[r] == 0:
            due.append((r + window, n[r], row0[r]))
        while due and due[0][0] <= r:
            _, nn, rr = due.pop(0)
            k2.append(2); n2.append(nn); r2.append(rr); o2.append(0)
    return (np.array(k2, np.int32), np.array(n2, np.int64), np.array(r2, np.int64), np.array(o2, np.int64),
            pool)


@pytest.mark.parametrize("precision,d,slots,nreq,pinned,gmb,br,graphs", [
    ("fp32", 64, 1, 300, False, 0, 0, False), ("fp32", 64, 8, 300, False, 0, 0, False),
    ("fp32", 61, 3, 300, True, 1 << 30, 0, False), ("fp32", 64, 4, 300, True, 0, 100, False),
    ("bf16", 256, 4, 200, True, 0, 0, False), ("bf16", 256, 2, 200, False, 0, 0, False),
    ("fp8", 256, 6, 200, True, -1, 0, False),
    ("fp32", 64, 4, 300, True, 0, 100, True), ("fp32", 61, 1, 300, False, 0, 0, True),
    ("bf16", 256, 4, 200, True, 0, 300, True), ("fp8", 256, 3, 200, False, 0, 0, True)])
def test_serving_equals_sequential_replay(precision, d, slots, nreq, pinned, gmb, br, graphs):
    """Closed loop (every request queued at once), so batches mix inserts and scores.  With
    pinned rows, requests of at most gmb bytes are read by the gather kernel (d=61 takes its
    unaligned path), larger ones by copies (0: the 64 KiB default, -1: never gather).
    br: target rows per batch (0 = max_rows).  graphs: the hash of each batch is a replay of a
    captured graph (one per slot and row bucket), so every replay is checked here."""
    import torch
    from paper_1706_06664_amd import ACE
    K, L = 15, 50
    kind, n, row0, out0, t, pool = serving_trace(nreq, d, seed=5, median_batch=32, max_batch=1024)
    W = projection_matrix(d, K, L, 1706066645)
    T_o, sk, n_amb = _oracle_replay(kind, n, row0, out0, pool, W, K, L)
    assert n_amb == 0   # continuous rows: no projection inside the FP64 margin
    _say(dict(precision=precision, slots=slots, requests=nreq, rows=int(n.sum()), scored=int(T_o.size)))
    ace = ACE(W, K, L, precision=precision, refine=True)
    srv = ace.server(slots=slots, max_rows=1024, gather_max_bytes=gmb, batch_rows=br, graphs=graphs)
    s_out = np.full(T_o.size, -1.0, np.float32)
    T_out = np.zeros(T_o.size, np.uint32)
    src = torch.from_numpy(pool).pin_memory() if pinned else pool
    lat = srv.replay(_records(kind, n, row0, out0, np.zeros_like(t)), src, s_out, T_out, pinned=pinned)
    st = srv.stats()
    _say(st)
    assert st["requests"] == nreq and st["rows"] == int(n.sum())
    lim = {0: 64 * 1024, -1: -1}.get(gmb, gmb)
    assert st["gathered_requests"] == (int((4 * d * n <= lim).sum()) if pinned else 0)
    if pinned and gmb == 0 and d == 256:   # requests above 64 KiB take copies
        assert 0 < st["gathered_requests"] < nreq
    if br:
        assert st["batches"] >= int(n.sum()) // 1024 and st["mean_batch_requests"] < nreq / 20
    if graphs:
        assert st["graph_launches"] == st["batches"] and 1 <= st["graph_captures"] <= 4 * slots
    else:
        assert st["graph_launches"] == 0
    assert (lat >= 0).all()
    np.testing.assert_array_equal(T_out.astype(np.int64), T_o)
    np.testing.assert_allclose(s_out, T_o / L, rtol=1e-6, atol=0)
    srv.close()
    assert np.array_equal(ace.counts().astype(np.int64), sk.counts)
    th = ace.threshold("scored", 1.0)
    _, th_o = sk.threshold(oracle.MODE_SCORED, 1.0)
    assert th["n"] == th_o["n"] and th["m_scored"] == th_o["m_scored"]
    assert abs(th["mu"] - th_o["mu"]) <= 1e-12 * th_o["mu"]
    assert abs(th["sigma"] - th_o["sigma"]) <= 1e-12 * max(th_o["sigma"], 1e-300)
    ace.close()


def test_submit_wait_pageable_and_pinned():
    import torch
    from paper_1706_06664_amd import ACE
    K, L, d = 15, 50, 64
    kind, n, row0, out0, t, pool = serving_trace(60, d, seed=6, median_batch=40, max_batch=512)
    W = projection_matrix(d, K, L, 11)
    T_o, sk, _ = _oracle_replay(kind, n, row0, out0, pool, W, K, L)
    ace = ACE(W, K, L)
    srv = ace.server(slots=3, max_rows=512)
    outs = []
    for r in range(len(kind)):
        X = pool[row0[r]:row0[r] + n[r]]
        if kind[r] == 0:
            srv.submit("insert", np.ascontiguousarray(X))
            continue
        if r % 2:   # pinned rows: read by the gather kernel
            Xp = torch.from_numpy(np.ascontiguousarray(X)).pin_memory()
            T = torch.zeros(int(n[r]), dtype=torch.int32).pin_memory()
            s = torch.zeros(int(n[r]), dtype=torch.float32).pin_memory()
            tk = srv.submit("score", Xp, s, T.view(torch.int32), pinned=True)
            outs.append((r, tk, s, T))
        else:
            s = np.zeros(n[r], np.float32)
            T = np.zeros(n[r], np.uint32)
            tk = srv.submit("score", np.ascontiguousarray(X), s, T)
            outs.append((r, tk, s, T))
    for r, tk, s, T in outs:
        lat = srv.wait(tk)
        assert lat >= 0
        Tn = T.numpy().view(np.uint32) if hasattr(T, "numpy") else T
        sn = s.numpy() if hasattr(s, "numpy") else s
        np.testing.assert_array_equal(Tn.astype(np.int64), T_o[out0[r]:out0[r] + n[r]])
        np.testing.assert_allclose(sn, Tn / L, rtol=1e-6, atol=0)
    srv.drain()
    st = srv.stats()
    assert st["requests"] == len(kind)
    assert st["gathered_requests"] == sum(1 for r, *_ in outs if r % 2)
    srv.close()
    ace.close()


def test_open_loop_latency_stats():
    from paper_1706_06664_amd import ACE
    K, L, d = 15, 50, 256
    kind, n, row0, out0, t, pool = serving_trace(400, d, seed=7, median_batch=64, max_batch=2048,
                                                 rate_per_s=4000.0, pool_rows=20000)
    W = projection_matrix(d, K, L, 12)
    ace = ACE(W, K, L, precision="bf16")
    srv = ace.server(slots=4, max_rows=2048)
    m = int(n[kind == 1].sum())
    lat = srv.replay(_records(kind, n, row0, out0, t), pool, np.zeros(m, np.float32), np.zeros(m, np.uint32))
    st = srv.stats()
    _say(st)
    assert st["requests"] == 400 and st["inserts"] + st["scores"] == 400
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert abs(st["p99_ms"] - np.percentile(lat, 99, method="inverted_cdf")) < 1e-9
    # the replay spans at least the trace's own arrival window
    assert st["wall_ms"] >= 1e3 * t[-1] * 0.99
    srv.reset_stats()
    assert srv.stats()["requests"] == 0
    srv.close()
    ace.close()


def test_server_errors():
    import ctypes
    from paper_1706_06664_amd import ACE, AceError
    K, L, d = 10, 4, 16
    W = projection_matrix(d, K, L, 13)
    ace = ACE(W, K, L)
    srv = ace.server(slots=2, max_rows=100)
    X = np.zeros((101, d), np.float32)
    with pytest.raises(AceError) as e:
        srv.submit("insert", X)
    assert e.value.status == 1
    with pytest.raises(AceError) as e:
        srv.submit(3, X[:5])
    assert e.value.status == 1
    # a delete of more rows than were inserted is refused at admission
    with pytest.raises(AceError) as e:
        srv.submit("delete", X[:5])
    assert e.value.status == 6
    with pytest.raises(AceError) as e:
        srv.wait(12345)
    assert e.value.status == 1
    # the context refuses destruction while the server is attached
    assert ace.lib.ace_destroy(ace.h) == 6
    # a second server on the same context is refused by the library too
    from paper_1706_06664_amd.ace import ServerConfig
    h = ctypes.c_void_p()
    cfg = ServerConfig(1, 0, 10, 0, 0, 0)
    assert ace.lib.ace_server_create(ace.h, ctypes.byref(cfg), ctypes.byref(h)) == 6
    srv.close()
    srv2 = ace.server(slots=1, max_rows=10)
    srv2.submit("insert", np.ones((10, d), np.float32))
    srv2.drain()
    srv2.close()
    assert ace.threshold("const", 1.0)["n"] == 10
    ace.close()


@pytest.mark.parametrize("precision,d,slots,graphs,cbits", [
    ("fp32", 64, 4, False, 32), ("fp32", 61, 1, False, 32), ("bf16", 256, 4, True, 32), ("fp8", 256, 3, False, 32),
    ("fp32", 64, 4, True, 16)])
def test_sliding_window_equals_sequential_replay(precision, d, slots, graphs, cbits):
    """Inserts, scores and deletes of rows that leave a sliding window, all queued at once:
    every score, the counts, n, mu and sigma equal the oracle replaying the log one request
    at a time (deletes included), whatever the number of slots.  With 16-bit counters no
    count comes near the cap here, so the uncapped oracle applies."""
    from paper_1706_06664_amd import ACE
    K, L = 15, 50
    kind, n, row0, out0, pool = _window_trace(240, d, window=40, seed=8)
    W = projection_matrix(d, K, L, 1706066646)
    T_o, sk, n_amb = _oracle_replay(kind, n, row0, out0, pool, W, K, L)
    assert n_amb == 0
    nd = int((kind == 2).sum())
    assert nd > 20 and int(n[kind == 2].sum()) < int(n[kind == 0].sum())
    _say(dict(precision=precision, slots=slots, requests=len(kind), deletes=nd, scored=int(T_o.size)))
    assert int(n[kind == 0].sum()) < 65535   # no bucket can reach the 16-bit cap
    ace = ACE(W, K, L, precision=precision, refine=True, counter_bits=cbits)
    srv = ace.server(slots=slots, max_rows=1024, graphs=graphs)
    s_out = np.full(T_o.size, -1.0, np.float32)
    T_out = np.zeros(T_o.size, np.uint32)
    srv.replay(_records(kind, n, row0, out0, np.zeros(len(kind))), pool, s_out, T_out)
    st = srv.stats()
    _say(st)
    assert st["requests"] == len(kind) and st["deletes"] == nd
    assert st["delete_rows"] == int(n[kind == 2].sum()) and st["insert_rows"] == int(n[kind == 0].sum())
    assert st["inserts"] + st["scores"] + st["deletes"] == len(kind)
    np.testing.assert_array_equal(T_out.astype(np.int64), T_o)
    np.testing.assert_allclose(s_out, T_o / L, rtol=1e-6, atol=0)
    srv.close()
    assert np.array_equal(ace.counts().astype(np.int64), sk.counts)
    th = ace.threshold("scored", 1.0)
    _, th_o = sk.threshold(oracle.MODE_SCORED, 1.0)
    assert th["n"] == th_o["n"] == int(n[kind == 0].sum() - n[kind == 2].sum())
    assert th["m_scored"] == th_o["m_scored"]
    assert abs(th["mu"] - th_o["mu"]) <= 1e-12 * th_o["mu"]
    assert abs(th["sigma"] - th_o["sigma"]) <= 1e-12 * max(th_o["sigma"], 1e-300)
    ace.close()


def test_cancel_with_deletes_keeps_counts_consistent():
    """An insert cannot be withdrawn while a delete admitted after it still needs its rows;
    once the delete is withdrawn it can, and nothing of either reaches the counts."""
    from paper_1706_06664_amd import ACE, AceError
    K, L, d = 10, 8, 32
    W = projection_matrix(d, K, L, 14)
    rng = np.random.default_rng(3)
    A = rng.standard_normal((10, d)).astype(np.float32)
    B = rng.standard_normal((7, d)).astype(np.float32)
    ace = ACE(W, K, L)
    srv = ace.server(slots=2, max_rows=64)
    tb = srv.submit("insert", B)
    srv.drain()
    srv.hold(True)
    ta = srv.submit("insert", A)
    td = srv.submit("delete", A)
    with pytest.raises(AceError) as e:
        srv.submit("delete", np.concatenate([B, B]))     # 14 > 7 + 10 - 10 points admitted
    assert e.value.status == 6
    assert srv.cancel(ta) is False                     # the delete still needs A's rows
    assert srv.cancel(td) is True
    assert srv.cancel(ta) is True
    srv.hold(False)
    srv.drain()
    st = srv.stats()
    assert st["cancelled"] == 2 and st["deletes"] == 0
    srv.close()
    codes, _ = oracle.hash_codes(B, W, K, L)
    sk = oracle.Sketch(K, L)
    sk.insert_codes(codes)
    assert np.array_equal(ace.counts().astype(np.int64), sk.counts)
    assert ace.threshold("const", 1.0)["n"] == 7
    assert tb >= 0
    ace.close()


_BIG = {37: 24000, 120: 65536, 121: 9000, 250: 40000, 251: 17000, 333: 33333}
_bench_cache = {}


def _bench_shape_trace():
    """400 requests of the serving workload (d = 256, lognormal sizes, median 256) with six
    requests forced to 9,000-65,536 rows, and their sequential oracle replay (cached)."""
    if not _bench_cache:
        K, L, d = 15, 50, 256
        kind, n, row0, out0, t, pool = serving_trace(400, d, seed=5, n_override=_BIG)
        W = projection_matrix(d, K, L, 1706066645)
        T_o, sk, n_amb = _oracle_replay(kind, n, row0, out0, pool, W, K, L)
        _bench_cache.update(kind=kind, n=n, row0=row0, out0=out0, t=t, pool=pool, W=W, T_o=T_o, sk=sk,
                            n_amb=n_amb)
    return _bench_cache


@pytest.mark.parametrize("graphs", [False, True])
def test_serving_bench_configuration(graphs):
    """The configuration the serving benchmark runs: BF16 + refine, d = 256, K = 15, L = 50,
    8 slots, max_rows = 65,536, batch_rows = 4,096, pinned rows.  Requests above batch_rows
    form batches of their own, so the count-update path for large batches (LDS histogram,
    codes at a row stride of the graph bucket) and the graph buckets of 16,384, 32,768 and
    65,536 rows are captured, replayed and compared with the sequential oracle replay."""
    import torch
    from paper_1706_06664_amd import ACE
    K, L = 15, 50
    c = _bench_shape_trace()
    kind, n, row0, out0, T_o, sk = c["kind"], c["n"], c["row0"], c["out0"], c["T_o"], c["sk"]
    assert c["n_amb"] == 0
    _say(dict(graphs=graphs, requests=len(kind), rows=int(n.sum()), largest=int(n.max()), scored=int(T_o.size)))
    ace = ACE(c["W"], K, L, precision="bf16", refine=True)
    srv = ace.server(slots=8, max_rows=65_536, gather_max_bytes=65_536, batch_rows=4096, graphs=graphs)
    s_out = np.full(T_o.size, -1.0, np.float32)
    T_out = np.zeros(T_o.size, np.uint32)
    src = torch.from_numpy(c["pool"]).pin_memory()
    # twice through the same server: the second replay reuses every captured graph
    for rep in range(2):
        if rep:
            ace.reset()
            torch.cuda.synchronize()   # the reset runs on this stream, the batches on the slots'
            srv.reset_stats()
            s_out[:] = -1.0
            T_out[:] = 0
        srv.replay(_records(kind, n, row0, out0, np.zeros_like(c["t"])), src, s_out, T_out, pinned=True)
        st = srv.stats()
        _say(st)
        assert st["requests"] == len(kind) and st["rows"] == int(n.sum())
        if graphs:
            assert st["graph_launches"] == st["batches"]
            # buckets above 8,192 rows: 16,384 (9,000 and 17,000 rows), 32,768, 65,536
            assert st["graph_captures"] >= (4 if rep == 0 else 0)
        np.testing.assert_array_equal(T_out.astype(np.int64), T_o)
        np.testing.assert_allclose(s_out, T_o / L, rtol=1e-6, atol=0)
        assert np.array_equal(ace.counts().astype(np.int64), sk.counts)
        th = ace.threshold("scored", 1.0)
        _, th_o = sk.threshold(oracle.MODE_SCORED, 1.0)
        assert th["n"] == th_o["n"] and th["m_scored"] == th_o["m_scored"]
        assert abs(th["mu"] - th_o["mu"]) <= 1e-12 * th_o["mu"]
        assert abs(th["sigma"] - th_o["sigma"]) <= 1e-12 * max(th_o["sigma"], 1e-300)
    srv.close()
    ace.close()


def test_server_slots_follow_memory_budget():
    """Admission by memory: under a mem_budget that leaves room for 2.5 slots the server keeps
    2 of the 8 it asks for, requests queue for them, and the results still equal the
    sequential oracle replay; a budget without room for one slot is refused (ACE_E_NOMEM)."""
    from paper_1706_06664_amd import ACE, AceError
    K, L, d = 15, 50, 64
    kind, n, row0, out0, t, pool = serving_trace(300, d, seed=8, median_batch=32, max_batch=1024)
    W = projection_matrix(d, K, L, 21)
    T_o, sk, n_amb = _oracle_replay(kind, n, row0, out0, pool, W, K, L)
    assert n_amb == 0
    probe = ACE(W, K, L, max_batch_rows=4096)
    b_ctx = probe.memory()
    srv = probe.server(slots=1, max_rows=1024)
    b_slot = probe.memory() - b_ctx
    srv.close()
    assert probe.memory() == b_ctx
    probe.close()
    _say(dict(context_bytes=b_ctx, slot_bytes=b_slot))
    assert b_slot > 0
    ace = ACE(W, K, L, max_batch_rows=4096, mem_budget=b_ctx + (5 * b_slot) // 2)
    srv = ace.server(slots=8, max_rows=1024)
    assert srv.stats()["slots"] == 2
    assert ace.memory() <= b_ctx + (5 * b_slot) // 2
    s_out = np.full(T_o.size, -1.0, np.float32)
    T_out = np.zeros(T_o.size, np.uint32)
    srv.replay(_records(kind, n, row0, out0, np.zeros_like(t)), pool, s_out, T_out)
    np.testing.assert_array_equal(T_out.astype(np.int64), T_o)
    srv.close()
    assert np.array_equal(ace.counts().astype(np.int64), sk.counts)
    ace.close()
    tight = ACE(W, K, L, max_batch_rows=4096, mem_budget=b_ctx + b_slot // 2)
    with pytest.raises(AceError) as e:
        tight.server(slots=2, max_rows=1024)
    assert e.value.status == 2
    assert tight.memory() <= b_ctx + b_slot // 2
    tight.close()


def test_server_cancel_and_timed_wait():
    """Requests withdrawn while still queued never run: the results equal the sequential
    oracle replay of the log without them.  A timed wait on a queued request ends with
    ACE_E_TIMEOUT, and waiting on a withdrawn one with ACE_E_STATE.  The test hold keeps the
    requests queued so that which ones are withdrawn is decided here, not by timing."""
    from paper_1706_06664_amd import ACE, AceError
    K, L, d = 15, 50, 64
    kind, n, row0, out0, t, pool = serving_trace(200, d, seed=9, median_batch=32, max_batch=512)
    W = projection_matrix(d, K, L, 22)
    ace = ACE(W, K, L)
    srv = ace.server(slots=3, max_rows=512, batch_rows=256)
    srv.hold(True)
    tickets, outs = [], {}
    for r in range(len(kind)):
        X = np.ascontiguousarray(pool[row0[r]:row0[r] + n[r]])
        if kind[r] == 0:
            tickets.append(srv.submit("insert", X))
        else:
            s = np.full(n[r], -1.0, np.float32)
            T = np.zeros(n[r], np.uint32)
            tickets.append(srv.submit("score", X, s, T))
            outs[r] = (s, T)
    with pytest.raises(AceError) as e:
        srv.wait(tickets[5], timeout_ms=20.0)
    assert e.value.status == 7
    gone = [r for r in range(len(kind)) if r % 3 == 1]
    for r in gone:
        assert srv.cancel(tickets[r])
    assert not srv.cancel(tickets[gone[0]])   # already withdrawn
    with pytest.raises(AceError) as e:
        srv.wait(tickets[gone[0]])
    assert e.value.status == 6
    srv.hold(False)
    srv.drain()
    st = srv.stats()
    _say(st)
    assert st["cancelled"] == len(gone) and st["requests"] == len(kind) - len(gone)
    assert not srv.cancel(tickets[0])          # completed: nothing to withdraw
    # the oracle replays the log without the withdrawn requests
    keep = np.array([r not in set(gone) for r in range(len(kind))])
    codes, _ = oracle.hash_codes(pool, W, K, L)
    sk = oracle.Sketch(K, L)
    for r in range(len(kind)):
        if not keep[r]:
            continue
        c = codes[row0[r]:row0[r] + n[r]]
        if kind[r] == 0:
            sk.insert_codes(c)
        else:
            T_o = sk.score_codes(c)
            s, T = outs[r]
            np.testing.assert_array_equal(T.astype(np.int64), T_o)
            np.testing.assert_allclose(s, T_o / L, rtol=1e-6, atol=0)
    srv.close()
    assert np.array_equal(ace.counts().astype(np.int64), sk.counts)
    assert ace.threshold("const", 1.0)["n"] == int(n[keep & (kind == 0)].sum())
    ace.close()
