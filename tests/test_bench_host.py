"""Host logic of the benchmark (no GPU): the sliding-window log and the sha-gated traffic
figure of the committed counter summary."""
import os

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_window_records_deletes_each_insert_window_requests_later():
    from paper_1706_06664_amd import REQUEST_DTYPE
    rng = np.random.default_rng(0)
    n_req, window = 500, 37
    rec = np.zeros(n_req, REQUEST_DTYPE)
    rec["kind"] = (rng.random(n_req) < 0.3).astype(np.int32)
    rec["n"] = rng.integers(1, 50, n_req)
    rec["row0"] = np.concatenate([[0], np.cumsum(rec["n"])[:-1]])
    w = bench.window_records(rec, window)
    # the original requests keep their order; one delete per insert that has `window` successors
    orig = w[w["kind"] != 2]
    assert np.array_equal(orig, rec)
    ins = np.nonzero(rec["kind"] == 0)[0]
    due = ins[ins + window < n_req]
    dels = w[w["kind"] == 2]
    assert len(dels) == len(due)
    assert np.array_equal(dels["row0"], rec["row0"][due]) and np.array_equal(dels["n"], rec["n"][due])
    # each delete comes right after request i + window, and never before its insert
    where = np.nonzero(w["kind"] != 2)[0]
    for i in due:
        p = np.nonzero((w["kind"] == 2) & (w["row0"] == rec["row0"][i]))[0][0]
        assert where[i + window] < p
        assert (w["kind"][where[i + window] + 1:p] == 2).all()
    # live rows never go negative along the log
    live = np.cumsum(np.where(w["kind"] == 0, w["n"], 0) - np.where(w["kind"] == 2, w["n"], 0))
    assert (live >= 0).all()


def test_recorded_traffic_is_gated_by_the_source_hash(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    import hashlib
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    summ = tmp_path / "s.md"
    summ.write_text(f"text\ntraffic_bytes_per_launch: 12345\nsource_sha256: {sha}\n")
    old = bench.ROOT
    try:
        bench.ROOT = str(tmp_path)
        assert bench.recorded_traffic("k.hip", "s.md") == 12345.0
        src.write_text("changed\n")
        assert bench.recorded_traffic("k.hip", "s.md") is None
        assert bench.recorded_traffic("missing.hip", "s.md") is None
    finally:
        bench.ROOT = old
    # the committed projection summary matches the committed kernel source
    assert bench.recorded_traffic("paper_1706_06664_amd/csrc/hash_fp32.hip",
                                  "profiles/hash_fp32_direct_kernel__connection_log_494021x120.md") is not None
