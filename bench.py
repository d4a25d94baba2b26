#!/usr/bin/env python3
"""Benchmark of the ACE hot path on one MI355X.

One step = reset the count arrays, insert every point (hash + count update),
score every point (hash + gather-sum), compute the mean/std threshold and flag
the points below it: the whole of Alg. 1 plus the Sec. 5.3 threshold over one
synthetic batch that is already resident in HBM.

Timing: W warm-up steps, then K steps each bracketed by HIP events on the launch
stream with the library's own event profiling off; `ms_per_step` is the median.
A separate profiled pass of the same steps gives the per-kernel launch times
(roofline, HBM fractions and the phase split).

Headline workload (the `value`): connection-log shaped points, 494,021 x 120
(38 lognormal columns, 82 one-hot columns, 20% anomalies from rare clusters),
K = 15 bits, L = 50 tables, FP32 projections refined in FP64 inside the FP32
error bound.  The other workloads (split-BF16 and e4m3 against FP32 on a dense
4,000,000 x 1024 low-rank workload and a 1,000,000 x 4096 heavy-tailed one, the
serving loop, the estimator study) go into a compact `workloads` block of the
JSON line; their full records go to stderr and, with --detail PATH, to a file.

Prints one JSON line on stdout.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3e12, "bf16": 2.5e15, "fp8": 5.0e15}
HBM_PEAK = 8.0e12
HASH_KERNEL = {"fp32": "hash_fp32_direct_kernel", "bf16": "hash_bf16_kernel", "fp8": "hash_fp8_kernel"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def r4(x):
    """Four significant digits (keeps the JSON line short)."""
    if isinstance(x, float):
        return float(f"{x:.4g}")
    if isinstance(x, dict):
        return {k: r4(v) for k, v in x.items()}
    if isinstance(x, list):
        return [r4(v) for v in x]
    return x


def recorded_traffic(source: str, summary: str):
    """HBM bytes per launch from a committed counter summary, or None once the kernel
    source differs from the one the counters were taken on."""
    import hashlib
    try:
        with open(os.path.join(ROOT, summary)) as f:
            text = f.read()
        with open(os.path.join(ROOT, source), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines() if line.startswith(("traffic_bytes", "source_sha")))
    if vals.get("source_sha256", "").strip() != sha:
        return None
    return float(vals["traffic_bytes_per_launch"])


# ---- CPU baseline (the oracle, untuned) ------------------------------------------------------

def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def oracle_step_rate(X, W, K, L, target_s):
    """The oracle on a bounded prefix of the workload: hash + insert every sample row, then
    hash + score + threshold + flags.  Returns (points/s, rows, seconds)."""
    import oracle

    def run(m):
        t0 = time.perf_counter()
        c, _ = oracle.hash_codes(X[:m], W, K, L)
        sk = oracle.Sketch(K, L)
        sk.insert_codes(c)
        c2, _ = oracle.hash_codes(X[:m], W, K, L)
        T = sk.score_codes(c2)
        rc, th = sk.threshold(oracle.MODE_SCORED, 1.0)
        sk.flags(T, th["tau"], oracle.MODE_SCORED)
        return time.perf_counter() - t0

    m = 1000
    t = run(m)
    m2 = int(min(X.shape[0], max(m, m * target_s / max(t, 1e-3))))
    t2 = run(m2)
    return m2 / t2, m2, t2


def cpu_baseline(X, W, K, L, target_s=10.0):
    """All host threads, in this process; then one thread, in a child process (the oracle's
    OpenMP team size is fixed when its library loads)."""
    threads = oracle_threads()
    v, m, t = oracle_step_rate(X, W, K, L, target_s)
    out = {"value": v, "unit": "points/s", "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"first {m} of {X.shape[0]} headline rows: hash+insert, then hash+score+threshold+flags, "
                     f"{t:.1f} s on {threads} threads"}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-leg", str(target_s)], env=env,
                           capture_output=True, text=True, timeout=600)
        one = json.loads(r.stdout.strip().splitlines()[-1])
        out["one_core"] = {"value": one["value"], "cores": 1, "rows": one["rows"]}
    except Exception as e:   # reported, never fatal: the GPU numbers stand on their own
        out["one_core"] = {"error": str(e)[:200]}
    return out


def cpu_leg(target_s):
    """Child process of cpu_baseline: the same oracle run on the threads OMP_NUM_THREADS gives."""
    from ace_inputs import c2_points, projection_matrix
    X, _ = c2_points()
    W = projection_matrix(120, 15, 50, 1706066642)
    v, m, t = oracle_step_rate(X, W, 15, 50, target_s)
    print(json.dumps({"value": v, "rows": m, "seconds": t}), flush=True)


def oracle_sample_check(Xd, W, K, L, codes_by_mode, rows):
    """FP64 oracle hashing of the first `rows` rows (rows/s on the host threads), and the code
    bits of each GPU mode on those rows that differ from the FP64 signs outside the oracle's
    margin (the unrefined flips, which the refinement must bring to 0)."""
    import numpy as np
    import oracle
    Xs = Xd[:rows].cpu().numpy()
    t0 = time.perf_counter()
    co, amb = oracle.hash_codes(Xs, W, K, L)
    dt = time.perf_counter() - t0
    out = {"rows": rows, "oracle_rows_per_s": rows / dt, "oracle_threads": oracle_threads(),
           "ambiguous_bits": int(np.unpackbits(amb.view(np.uint8)).sum())}
    for mode, cg in codes_by_mode.items():
        diff = np.bitwise_and(np.bitwise_xor(cg, co), np.bitwise_not(amb))
        out[f"{mode}_unrefined_flips"] = int(np.unpackbits(diff.view(np.uint8)).sum())
    return out


# ---- GPU workloads ---------------------------------------------------------------------------

def median(v):
    s = sorted(v)
    m = len(s)
    return s[m // 2] if m % 2 else 0.5 * (s[m // 2 - 1] + s[m // 2])


def run_workload(Xd, W, K, L, precision, steps, warmup, refine=1, keep=None, counter_bits=32, signs=None):
    """Time `steps` full steps (median, HIP events on the launch stream, profiling off), then
    profile as many steps again for the per-kernel launch times.  If `keep` is a dict, the
    last step's T (int32, device) is stored in keep["T"]."""
    import torch
    from paper_1706_06664_amd import ACE
    n, d = Xd.shape
    s = torch.empty(n, dtype=torch.float32, device=Xd.device)
    T = torch.empty(n, dtype=torch.int32, device=Xd.device)
    ace = ACE(W if signs is None else None, K, L, precision=precision, device=0, refine=refine,
              counter_bits=counter_bits, signs=signs, d=d)
    st = torch.cuda.current_stream()

    def step():
        ace.reset()
        ace.insert(Xd)
        ace.score(Xd, s=s, T=T)
        flags, th = ace.threshold_flag(T, "scored", 1.0)   # threshold, then flags on the device
        return flags, th

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in ev:
        e0.record(st)
        flags, th = step()
        e1.record(st)
    torch.cuda.synchronize()
    times = [e0.elapsed_time(e1) for e0, e1 in ev]
    # profiled pass: HIP events around every launch, on its stream
    ace.profile()
    c0 = ace.counters()
    ace.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    prof_ms = (time.perf_counter() - t0) * 1e3 / steps
    ace.profile_enable(False)
    prof = ace.profile()
    c1 = ace.counters()
    ace.close()
    if keep is not None:
        keep["T"] = T
    ms = median(times)
    hash_ms = prof["hash_ms"] / max(1, prof["hash_launches"])
    rows = prof["hash_rows"] / max(1, prof["hash_launches"])
    flop = 2.0 * rows * d * K * L
    executed = flop * (16.0 / K) * (3.0 if precision == "bf16" else 1.0)
    kernel = HASH_KERNEL[precision] if signs is None else "hash_struct_kernel"
    ach = flop / (hash_ms / 1e3)
    bits = c1["bits_hashed"] - c0["bits_hashed"]

    def per_launch(key):
        return prof[f"{key}_ms"] / max(1, prof[f"{key}_launches"])

    # HBM fractions of the count kernels (a5, a6) and the convert (a1): algorithmic bytes
    # per launch over the average launch time.  Rows per launch from the launch counts.
    hbm = {}
    tables = float(L) * (1 << K) * (2 if counter_bits == 16 else 4)
    if prof["update_launches"]:
        r_u = n * steps / prof["update_launches"]
        b = 2.0 * L * r_u + 2.0 * tables
        hbm["update"] = {"ms": per_launch("update"), "bytes": b, "frac": b / (per_launch("update") / 1e3) / HBM_PEAK}
    if prof["score_launches"]:
        r_s = n * steps / prof["score_launches"]
        b = (2.0 * L + 8.0) * r_s + tables
        hbm["score"] = {"ms": per_launch("score"), "bytes": b, "frac": b / (per_launch("score") / 1e3) / HBM_PEAK}
    if prof["convert_launches"]:
        r_c = 2.0 * n * steps / prof["convert_launches"]
        out_b = {"bf16": 4.0 * d, "fp8": 1.0 * d}.get(precision, 0.0)
        b = (4.0 * d + out_b + 12.0) * r_c
        hbm["convert"] = {"ms": per_launch("convert"), "bytes": b,
                          "frac": b / (per_launch("convert") / 1e3) / HBM_PEAK}
    return {
        "points_per_s": n / (ms / 1e3), "ms_per_step": ms, "ms_per_step_mean": sum(times) / len(times),
        "ms_per_step_min": min(times), "ms_per_step_max": max(times), "ms_per_step_profiled": prof_ms,
        "phase_ms_per_step": {k: prof[k] / steps for k in ("convert_ms", "hash_ms", "refine_ms", "update_ms",
                                                            "score_ms", "other_ms")},
        "roofline": {"bound": "mfma", "achieved": ach / 1e12, "peak": PEAK[precision] / 1e12, "unit": "TFLOP/s",
                     "frac": ach / PEAK[precision], "traffic": None, "kernel": kernel,
                     "avg_launch_ms": hash_ms, "rows_per_launch": rows,
                     "executed_frac": executed / (hash_ms / 1e3) / PEAK[precision]},
        "hbm": hbm,
        "refined_bit_frac": (c1["bits_refined"] - c0["bits_refined"]) / max(1, bits),
        "raw_flip_rate": (c1["bits_flipped"] - c0["bits_flipped"]) / max(1, bits),
        "in_bound_unrefined_frac": (c1["bits_in_bound_unrefined"] - c0["bits_in_bound_unrefined"]) / max(1, bits),
        "saturated_increments_last_step": c1["saturated_increments"],
        "flagged": int(flags.sum().item()), "tau": th["tau"],
    }


def brief(r):
    """The fields of a run_workload record that the JSON line keeps."""
    out = {"ms": r["ms_per_step"], "pts_s": r["points_per_s"], "proj_frac": r["roofline"]["frac"],
           "refined": r["refined_bit_frac"]}
    if r["roofline"]["kernel"] == "hash_bf16_kernel":
        out["proj_exec_frac"] = r["roofline"]["executed_frac"]
    if r["raw_flip_rate"]:
        out["raw_flips"] = r["raw_flip_rate"]
    return out


def cache_codes_run(Xd, W, K, L, steps, warmup):
    """The same step with each row hashed once: hash, then insert and score from the codes
    (ace_hash, ace_insert_codes, ace_score_codes), threshold and flags.  Reported beside the
    headline, whose insert and score each hash the rows."""
    import torch
    from paper_1706_06664_amd import ACE
    ace = ACE(W, K, L, precision="fp32", device=0)
    st = torch.cuda.current_stream()

    def step():
        ace.reset()
        codes = ace.hash(Xd)
        ace.insert_codes(codes)
        _, T = ace.score_codes(codes)
        return ace.threshold_flag(T, "scored", 1.0)[0]

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in ev:
        e0.record(st)
        step()
        e1.record(st)
    torch.cuda.synchronize()
    ms = median([e0.elapsed_time(e1) for e0, e1 in ev])
    ace.close()
    return {"points_per_s": Xd.shape[0] / (ms / 1e3), "ms_per_step": ms,
            "step": "hash once, insert codes, score codes, threshold, flags"}


def paper_shape_runs(steps, warmup):
    """Synthetic Gaussian-mixture rows of the shapes of the paper's three datasets (Shuttle
    34,987 x 9, ALOI 50,000 x 27, KDD-Cup99 HTTP 596,853 x 36) at K = 15, L = 50, FP32 with
    FP64 refine: context beside the paper's single-core times (Tables 3-5), not a like-for-like
    comparison (different data, different machine)."""
    import torch
    from ace_inputs import gaussian_clusters, projection_matrix
    out = {}
    for name, n, d, seed, paper_s in (("shuttle_shape", 34_987, 9, 31, 0.81), ("aloi_shape", 50_000, 27, 32, 1.26),
                                      ("kdd_http_shape", 596_853, 36, 33, 23.33)):
        X, _ = gaussian_clusters(n, d, 8, 0.02, seed=seed)
        W = projection_matrix(d, 15, 50, 1706066650 + seed)
        r = run_workload(torch.from_numpy(X).to("cuda:0"), W, 15, 50, "fp32", steps, warmup)
        out[name] = {"n": n, "d": d, "points_per_s": r["points_per_s"], "ms_per_step": r["ms_per_step"],
                     "paper_points_per_s_cpu": n / paper_s}
        log(f"  {name}: {r['ms_per_step']:.3f} ms/step")
    return out


def raw_score_error(Xs, W, K, L, precision):
    """Score error of raw low-precision signs (refinement off) against the refined scores,
    which equal the FP64 oracle's (checked by the GPU tests): insert and score the sample."""
    import numpy as np
    from paper_1706_06664_amd import ACE
    out = []
    for refine in (True, False):
        a = ACE(W, K, L, precision=precision, refine=refine)
        a.insert(Xs)
        s, T = a.score(Xs)
        out.append(T.cpu().numpy().astype(np.float64))
        a.close()
    ref, raw = out
    rel = np.abs(raw - ref) / np.maximum(ref, 1.0)
    return {"rows": int(Xs.shape[0]), "max_rel": float(rel.max()), "mean_rel": float(rel.mean()),
            "rows_changed": int((raw != ref).sum())}


def popcount_xor(a, b):
    """Number of differing bits between two int16 device tensors of codes."""
    import torch
    table = torch.tensor([bin(i).count("1") for i in range(256)], dtype=torch.int64, device=a.device)
    x = torch.bitwise_xor(a, b).contiguous().view(torch.uint8)
    return int(table[x.long()].sum().item())


def sample_codes(ace_args, Xs):
    """Codes of the sample rows as host uint16 [rows][L]."""
    from paper_1706_06664_amd import ACE, codes_as_uint16
    a = ACE(*ace_args[:3], **ace_args[3])
    c = codes_as_uint16(a.hash(Xs))
    a.close()
    return c


def low_rank_runs(n3, steps, warmup, sample_rows):
    """Dense low-rank 4,000,000 x 1024 rows, K = 15, L = 64: FP32 and split-BF16 refined steps,
    the raw-sign score error, and the oracle's check of a 65,536-row sample."""
    import torch
    from ace_inputs import low_rank_points_torch, projection_matrix
    d3, K3, L3 = 1024, 15, 64
    X3, _ = low_rank_points_torch(n3, d3, seed=3, device="cuda:0")
    W3 = projection_matrix(d3, K3, L3, 1706066643)
    lr = {"workload": f"low-rank {n3}x{d3}, K={K3}, L={L3}"}
    for prec in ("fp32", "bf16"):
        log(f"low-rank {n3}x{d3} {prec}: warmup {warmup}, steps {steps}")
        lr[prec] = run_workload(X3, W3, K3, L3, prec, steps, warmup)
        log(f"  {lr[prec]['ms_per_step']:.3f} ms/step (profiled {lr[prec]['ms_per_step_profiled']:.3f})")
    lr["bf16_speedup"] = lr["fp32"]["ms_per_step"] / lr["bf16"]["ms_per_step"]
    Xs = X3[:sample_rows].contiguous()
    lr["bf16_raw_score_error"] = raw_score_error(Xs, W3, K3, L3, "bf16")
    codes = {m: sample_codes((W3, K3, L3, {"precision": m}), Xs) for m in ("fp32", "bf16")}
    log(f"low-rank oracle sample: {sample_rows} rows")
    lr["oracle_sample"] = oracle_sample_check(X3, W3, K3, L3, codes, sample_rows)
    log(f"  {lr['oracle_sample']}")
    del X3, Xs
    torch.cuda.empty_cache()
    return lr


def heavy_tail_runs(steps, warmup, sample_rows):
    """Heavy-tailed 1,000,000 x 4096 rows, K = 16, L = 100: FP32 and split-BF16 refined steps,
    and FP8 e4m3 with raw signs (refine = 2 also counts the bits inside the FP8 bound).  The
    FP8 raw flip rate and score error are taken against the FP32 refined codes and scores,
    which equal the FP64 signs (GPU tests, and the oracle sample here)."""
    import torch
    from ace_inputs import heavy_tail_points_torch, projection_matrix, structured_signs
    from paper_1706_06664_amd import ACE
    n4, d4, K4, L4 = 1_000_000, 4096, 16, 100
    X4, _ = heavy_tail_points_torch(n4, d4, seed=4, device="cuda:0")
    W4 = projection_matrix(d4, K4, L4, 1706066644)
    out = {"workload": f"heavy-tail t(3) {n4}x{d4}, K={K4}, L={L4}"}
    keep = {}
    for prec, refine in (("fp32", 1), ("bf16", 1), ("fp8", 2)):
        log(f"heavy-tail {n4}x{d4} {prec} refine={refine}: warmup {warmup}, steps {steps}")
        k = {}
        out[prec] = run_workload(X4, W4, K4, L4, prec, steps, warmup, refine=refine, keep=k)
        keep[prec] = k["T"].clone()
        log(f"  {out[prec]['ms_per_step']:.3f} ms/step")
    c32 = ACE(W4, K4, L4, precision="fp32").hash(X4)
    c8 = ACE(W4, K4, L4, precision="fp8", refine=0).hash(X4)
    flips = popcount_xor(c32, c8)
    t32 = keep["fp32"].double()
    t8 = keep["fp8"].double()
    rel = (t8 - t32).abs() / t32.clamp_min(1.0)
    out["fp8_raw_flip_rate"] = flips / (n4 * K4 * L4)
    out["fp8_raw_score_error"] = {"max_rel": float(rel.max().item()), "mean_rel": float(rel.mean().item()),
                                  "rows_changed": int((t8 != t32).sum().item()), "rows": n4}
    out["fp8_in_bound_frac"] = out["fp8"]["in_bound_unrefined_frac"]
    out["bf16_speedup"] = out["fp32"]["ms_per_step"] / out["bf16"]["ms_per_step"]
    out["fp8_raw_speedup"] = out["fp32"]["ms_per_step"] / out["fp8"]["ms_per_step"]
    del c32, c8
    Xs = X4[:sample_rows].contiguous()
    codes = {m: sample_codes((W4, K4, L4, {"precision": m}), Xs) for m in ("fp32", "bf16")}
    # e4m3 before and after refinement on the sample: raw signs, and the FP64 pass over every
    # bit inside the e4m3 bound (almost all of them on this data), timed
    codes["fp8_raw"] = sample_codes((W4, K4, L4, {"precision": "fp8", "refine": 0}), Xs)
    a8 = ACE(W4, K4, L4, precision="fp8", refine=1)
    a8.hash(Xs)
    torch.cuda.synchronize()
    c0 = a8.counters()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    c8 = a8.hash(Xs)
    e1.record()
    torch.cuda.synchronize()
    c1 = a8.counters()
    from paper_1706_06664_amd import codes_as_uint16
    codes["fp8_refined"] = codes_as_uint16(c8)
    out["fp8_refined_sample"] = {"rows": sample_rows, "hash_ms": e0.elapsed_time(e1),
                                 "refined_frac": (c1["bits_refined"] - c0["bits_refined"]) /
                                                 max(1, c1["bits_hashed"] - c0["bits_hashed"])}
    a8.close()
    log(f"heavy-tail oracle sample: {sample_rows} rows")
    out["oracle_sample"] = oracle_sample_check(X4, W4, K4, L4, codes, sample_rows)
    log(f"  {out['oracle_sample']}")
    # Structured projections (H D3 H D2 H D1, one 4096-point block per row): another hash
    # family (the paper's fast-transform hashing), refined to the FP64 signs of its own
    # dense equivalent.
    s4, _ = structured_signs(d4, K4, L4, 1706066647)
    log(f"heavy-tail {n4}x{d4} structured fp32: steps {steps}")
    st = run_workload(X4, None, K4, L4, "fp32", steps, warmup, signs=s4)
    rows = st["roofline"]["rows_per_launch"]
    st["roofline"] = {"bound": "hbm", "kernel": "hash_struct_kernel", "avg_launch_ms": st["roofline"]["avg_launch_ms"],
                      "achieved": 4.0 * d4 * rows / (st["roofline"]["avg_launch_ms"] / 1e3) / 1e9, "peak": 8000.0,
                      "unit": "GB/s", "adds_per_row": 3 * d4 * 12}
    st["roofline"]["frac"] = st["roofline"]["achieved"] / 8000.0
    out["structured_fp32"] = st
    out["structured_speedup_vs_fp32"] = out["fp32"]["ms_per_step"] / st["ms_per_step"]
    log(f"  {st['ms_per_step']:.3f} ms/step")
    del X4, Xs
    torch.cuda.empty_cache()
    return out


def serving_log(n_req=100_000, d=256, seed=5):
    """The serving workload's request log: n_req requests (70% inserts, 30% scores; lognormal
    sizes, median 256 rows, sigma 1, clipped to 1..65,536; Poisson arrivals), every request
    with rows of its own in request order, the mixture means drifting with the request id.
    The rows (about 43 GB for 100,000 requests) are drawn on the GPU and kept in pinned host
    memory (pageable if pinning fails): serving reads them over the host link."""
    import numpy as np
    import torch
    from ace_inputs import serving_requests, serving_rows_torch
    from paper_1706_06664_amd import REQUEST_DTYPE
    reqs = serving_requests(n_req, seed=seed)
    kind = np.array([0 if q.kind == "insert" else 1 for q in reqs], np.int32)
    n = np.array([q.n for q in reqs], np.int64)
    t = np.array([q.arrival_s for q in reqs], np.float64)
    rows = int(n.sum())
    t0 = time.perf_counter()
    try:
        pool = torch.empty((rows, d), dtype=torch.float32, pin_memory=True)
        pinned = True
    except RuntimeError:
        pool = torch.empty((rows, d), dtype=torch.float32)
        pinned = False
    serving_rows_torch(n, d, pool, seed=seed, device="cuda:0")
    torch.cuda.synchronize()
    log(f"serving log: {n_req} requests, {rows} rows ({rows * d * 4 / 1e9:.1f} GB, "
        f"{'pinned' if pinned else 'pageable'}) drawn in {time.perf_counter() - t0:.1f} s")
    rec = np.zeros(n_req, REQUEST_DTYPE)
    sc = kind == 1
    out0 = np.zeros(n_req, np.int64)
    out0[sc] = np.concatenate([[0], np.cumsum(n[sc])[:-1]])
    rec["kind"], rec["n"], rec["row0"], rec["out0"] = kind, n, np.concatenate([[0], np.cumsum(n)[:-1]]), out0
    return {"rec": rec, "t": t, "pool": pool, "pinned": pinned, "rows": rows, "scored": int(n[sc].sum()),
            "n_req": n_req, "d": d}


def window_records(rec, window):
    """The log with a sliding window: each insert's rows are deleted again (Eq. dynsub) right
    after the request `window` places later, so at most the last `window` requests' inserts
    stay counted."""
    import numpy as np
    n_req = len(rec)
    ins = np.nonzero((rec["kind"] == 0) & (np.arange(n_req) + window < n_req))[0]
    dels = rec[ins].copy()
    dels["kind"], dels["out0"] = 2, 0
    key = np.concatenate([2 * np.arange(n_req), 2 * (ins + window) + 1])
    return np.concatenate([rec, dels])[np.argsort(key, kind="stable")]


def serving_runs(lg, slots=8, batch_rows=4096, gather_max_bytes=65536, graphs=False, window=None):
    """Serving workload: d = 256, K = 15, L = 50, the whole request log through the serving
    loop.  Closed loop (every request queued at once) gives the saturation rate in FP32 and
    BF16; open loop (Poisson arrivals at 0.5, 0.8 and 0.95 of the BF16 saturation request
    rate) gives latency percentiles, from arrival to completion (host copies included).
    window: also a closed-loop BF16 run of the log with a sliding window of that many
    requests (every insert deleted again `window` requests later)."""
    import numpy as np
    import torch
    from ace_inputs import projection_matrix
    from paper_1706_06664_amd import ACE
    K, L, d = 15, 50, lg["d"]
    W = projection_matrix(d, K, L, 1706066645)
    rec, t, pool, n_req = lg["rec"], lg["t"], lg["pool"], lg["n_req"]
    s_out = torch.zeros(lg["scored"], dtype=torch.float32, pin_memory=lg["pinned"])
    T_out = torch.zeros(lg["scored"], dtype=torch.int32, pin_memory=lg["pinned"])

    def run(prec, arr=None, recs=None):
        ace = ACE(W, K, L, precision=prec)
        srv = ace.server(slots=slots, max_rows=65_536, gather_max_bytes=gather_max_bytes, batch_rows=batch_rows,
                         graphs=graphs)
        srv.replay(rec[:500], pool, s_out, T_out, pinned=lg["pinned"])   # warm-up
        ace.reset()
        torch.cuda.synchronize()
        srv.reset_stats()
        r = (rec if recs is None else recs).copy()
        if arr is not None:
            r["t_arrival_s"] = arr
        srv.replay(r, pool, s_out, T_out, pinned=lg["pinned"])
        st = srv.stats()
        srv.close()
        ace.close()
        wall = st["wall_ms"] / 1e3
        return {"points_per_s": st["rows"] / wall, "requests_per_s": st["requests"] / wall,
                "deletes": st["deletes"], "delete_rows": st["delete_rows"],
                "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "p99_queue_ms": st["p99_queue_ms"],
                "max_ms": st["max_ms"], "batches": st["batches"],
                "mean_batch_requests": st["mean_batch_requests"], "graph_launches": st["graph_launches"]}

    out = {"workload": f"serving d={d}, K={K}, L={L}: {n_req} requests, {lg['rows']} rows, 70% inserts, "
                       f"lognormal sizes (median 256, sigma 1), drift by request id",
           "server": {"slots": slots, "batch_rows": batch_rows, "gather_max_bytes": gather_max_bytes,
                      "max_rows": 65_536, "graphs": graphs, "pinned_rows": lg["pinned"]}}
    for prec in ("fp32", "bf16"):
        log(f"serving closed loop {prec}{' (graphs)' if graphs else ''}")
        out[f"closed_loop_{prec}"] = run(prec)
        log(f"  {out[f'closed_loop_{prec}']['points_per_s']:.3e} points/s")
    if window:
        log(f"serving closed loop bf16, sliding window of {window} requests")
        out["closed_loop_bf16_window"] = run("bf16", recs=window_records(rec, window))
        out["closed_loop_bf16_window"]["window_requests"] = window
        log(f"  {out['closed_loop_bf16_window']['points_per_s']:.3e} points/s "
            f"({out['closed_loop_bf16_window']['deletes']} deletes)")
    sat = out["closed_loop_bf16"]["requests_per_s"]
    out["open_loop_bf16"] = []
    base_rate = n_req / t[-1]
    for load in (0.5, 0.8, 0.95):
        log(f"serving open loop bf16 at {load} of saturation{' (graphs)' if graphs else ''}")
        o = run("bf16", arr=t * (base_rate / (load * sat)))
        o["load"] = load
        o["offered_requests_per_s"] = load * sat
        out["open_loop_bf16"].append(o)
        log(f"  p50 {o['p50_ms']:.3f} ms, p99 {o['p99_ms']:.3f} ms, {o['points_per_s']:.3e} points/s")
    out["bf16_vs_fp32_closed_loop"] = out["closed_loop_bf16"]["points_per_s"] / out["closed_loop_fp32"]["points_per_s"]
    out["pcie_bound_points_per_s"] = 55e9 / (4 * d)
    return out


def exact_score_runs(X, W, K, n_queries=4096, reps=5):
    """Exact S(q, D) (Eq. thescore) of n_queries rows of the connection-log workload against
    all of its rows, timed with HIP events on the launch stream (FP64 matrix roofline:
    2 m n d FLOP per launch), then the estimator study of Sec. 3 on the same queries: the
    ACE estimate T/L at several L against the exact S (relative RMSE), beside the standard
    deviation of uniform sampling with L points, sqrt((n sum p^2K - S^2) / L) (Theorem 2's
    comparison)."""
    import numpy as np
    import torch
    from ace_inputs import projection_matrix
    from paper_1706_06664_amd import ACE, exact_score
    n, d = X.shape
    Xd = torch.from_numpy(X).to("cuda:0")
    idx = torch.from_numpy(np.linspace(0, n - 1, n_queries).astype(np.int64)).to("cuda:0")
    Qd = Xd[idx].contiguous()
    S, S2 = exact_score(Qd, Xd, K, want_S2=True)
    st = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        exact_score(Qd, Xd, K, stream=st)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flop = 2.0 * n_queries * n * d
    out = {"workload": f"exact S of {n_queries} connection-log rows against {n}x{d}, K={K}",
           "ms_per_launch": ms, "pairs_per_s": n_queries * n / (ms / 1e3),
           "roofline": {"bound": "mfma", "achieved": flop / (ms / 1e3) / 1e12, "peak": 78.6, "unit": "TFLOP/s",
                        "frac": flop / (ms / 1e3) / 78.6e12, "kernel": "exact_score_kernel (FP64 MFMA + arccos)"}}
    S, S2 = S.double(), S2.double()
    study = []
    for L in (10, 20, 50, 100, 200):
        Wl = projection_matrix(d, K, L, 1706066700 + L)
        a = ACE(Wl, K, L)
        a.insert(Xd)
        s, _ = a.score(Qd)
        a.close()
        err = s.double() - S
        rse_sd = torch.sqrt(torch.clamp(n * S2 - S * S, min=0) / L)
        study.append({"L": L, "ace_rel_rmse": float(torch.sqrt((err ** 2).mean()) / S.mean()),
                      "ace_mean_rel_bias": float(err.mean() / S.mean()),
                      "rse_rel_sd": float(torch.sqrt((rse_sd ** 2).mean()) / S.mean())})
    out["estimator_study"] = study
    out["S_mean"] = float(S.mean())
    return out


def workloads_block(extra):
    """The compact summary the JSON line carries: BF16-vs-FP32 speed-ups with refined
    fractions, raw flip rates and the unrefined flips the oracle sample found, the e4m3 flip
    rate and score error, and the serving loop's rates and latencies."""
    ns = {}
    lr = extra.get("low_rank_1024")
    if lr:
        ns["low_rank_4000000x1024"] = {
            "bf16_vs_fp32": lr["bf16_speedup"], "fp32": brief(lr["fp32"]), "bf16": brief(lr["bf16"]),
            "bf16_hbm_convert_frac": lr["bf16"]["hbm"].get("convert", {}).get("frac"),
            "bf16_raw_score_err": {"mean": lr["bf16_raw_score_error"]["mean_rel"],
                                   "max": lr["bf16_raw_score_error"]["max_rel"]},
            "oracle_sample": {k: v for k, v in lr["oracle_sample"].items() if k != "oracle_threads"}}
    ht = extra.get("heavy_tail_4096")
    if ht:
        ns["heavy_tail_1000000x4096"] = {
            "bf16_vs_fp32": ht["bf16_speedup"], "fp32": brief(ht["fp32"]), "bf16": brief(ht["bf16"]),
            "e4m3_refined_sample": {"rows": ht["fp8_refined_sample"]["rows"],
                                    "hash_ms": ht["fp8_refined_sample"]["hash_ms"],
                                    "refined": ht["fp8_refined_sample"]["refined_frac"],
                                    "raw_flips": ht["oracle_sample"]["fp8_raw_unrefined_flips"],
                                    "flips_after": ht["oracle_sample"]["fp8_refined_unrefined_flips"]},
            "e4m3_raw": {"ms": ht["fp8"]["ms_per_step"], "vs_fp32": ht["fp8_raw_speedup"],
                         "proj_frac": ht["fp8"]["roofline"]["frac"], "flip_rate": ht["fp8_raw_flip_rate"],
                         "score_err_mean": ht["fp8_raw_score_error"]["mean_rel"],
                         "score_err_max": ht["fp8_raw_score_error"]["max_rel"], "in_bound": ht["fp8_in_bound_frac"]},
            "structured": {"ms": ht["structured_fp32"]["ms_per_step"], "vs_fp32": ht["structured_speedup_vs_fp32"]},
            "oracle_sample": {k: v for k, v in ht["oracle_sample"].items() if k != "oracle_threads"}}
    if "connection_log_bf16" in extra:
        ns["connection_log_bf16"] = dict(brief(extra["connection_log_bf16"]),
                                         vs_fp32=extra["connection_log_bf16_speedup"])
    if "connection_log_cache_codes" in extra:
        ns["connection_log_hash_once"] = {"ms": extra["connection_log_cache_codes"]["ms_per_step"],
                                          "pts_s": extra["connection_log_cache_codes"]["points_per_s"]}
    if "connection_log_counters16" in extra:
        ns["connection_log_counters16"] = {"ms": extra["connection_log_counters16"]["ms_per_step"],
                                           "update_ms": extra["connection_log_counters16"]["phase_ms_per_step"]["update_ms"]}
    if "hot_bucket" in extra:
        ns["hot_bucket_494021x120"] = {"ms": extra["hot_bucket"]["ms_per_step"],
                                       "update_ms": extra["hot_bucket"]["phase_ms_per_step"]["update_ms"],
                                       "score_ms": extra["hot_bucket"]["phase_ms_per_step"]["score_ms"]}
    for key in ("serving_256", "serving_256_graphs"):
        sv = extra.get(key)
        if sv:
            ns[key] = {"closed_pts_s": {"fp32": sv["closed_loop_fp32"]["points_per_s"],
                                        "bf16": sv["closed_loop_bf16"]["points_per_s"]},
                       "open_bf16": [{"load": o["load"], "p50_ms": o["p50_ms"], "p99_ms": o["p99_ms"],
                                      "pts_s": o["points_per_s"]} for o in sv["open_loop_bf16"]],
                       "requests": sv["workload"].split(": ")[1].split(",")[0],
                       **({"bf16_window_pts_s": sv["closed_loop_bf16_window"]["points_per_s"],
                           "window_requests": sv["closed_loop_bf16_window"]["window_requests"]}
                          if "closed_loop_bf16_window" in sv else {}),
                       "rows": sv["workload"].split(": ")[1].split(", ")[1]}
    ex = extra.get("exact_score_connection_log")
    if ex:
        ns["exact_S"] = {"ms": ex["ms_per_launch"], "fp64_mfma_frac": ex["roofline"]["frac"]}
    return r4(ns)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true", help="skip every workload but the headline")
    ap.add_argument("--low-rank-n", type=int, default=4_000_000)
    ap.add_argument("--sample-rows", type=int, default=65_536,
                    help="rows of the low-rank and heavy-tail workloads the oracle hashes")
    ap.add_argument("--detail", default=None, help="write every record to this JSON file")
    ap.add_argument("--serving-requests", type=int, default=100_000)
    ap.add_argument("--cpu-leg", type=float, default=None, help=argparse.SUPPRESS)
    ap.add_argument("--traffic-run", action="store_true",
                    help="for counter runs: one 256 MiB device copy (calibration), then two headline inserts "
                         "and scores; prints no JSON")
    args = ap.parse_args()
    if args.cpu_leg is not None:
        cpu_leg(args.cpu_leg)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the multi-GPU layout "
              f"is a design, not a run)", file=sys.stderr)
        sys.exit(2)
    steps, warmup = max(1, args.steps), max(0, args.warmup)

    import torch
    from ace_inputs import c2_points, projection_matrix

    K, L, d = 15, 50, 120
    X, _ = c2_points()
    n = X.shape[0]
    W = projection_matrix(d, K, L, 1706066642)
    Xd = torch.from_numpy(X).to("cuda:0")
    if args.traffic_run:
        from paper_1706_06664_amd import ACE
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")   # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        ace = ACE(W, K, L, precision="fp32")
        for _ in range(2):
            ace.reset()
            ace.insert(Xd)
            ace.score(Xd)
        torch.cuda.synchronize()
        log("traffic run done: copy 256 MiB, 2 x (insert + score) of the headline workload")
        return
    log(f"connection-log {n}x{d} fp32: warmup {warmup}, steps {steps}")
    head = run_workload(Xd, W, K, L, "fp32", steps, warmup)
    log(f"  {head['ms_per_step']:.3f} ms/step median (mean {head['ms_per_step_mean']:.3f}, "
        f"profiled {head['ms_per_step_profiled']:.3f})")

    extra = {}
    if not args.headline_only:
        log("connection-log bf16")
        b = run_workload(Xd, W, K, L, "bf16", steps, warmup)
        extra["connection_log_bf16"] = b
        extra["connection_log_bf16_speedup"] = head["ms_per_step"] / b["ms_per_step"]
        log(f"  {b['ms_per_step']:.3f} ms/step")
        from ace_inputs import structured_signs
        s2, _ = structured_signs(d, K, L, 1706066646)
        log("connection-log structured fp32")
        extra["connection_log_structured"] = run_workload(Xd, None, K, L, "fp32", steps, warmup, signs=s2)
        log(f"  {extra['connection_log_structured']['ms_per_step']:.3f} ms/step")
        log("connection-log fp32, rows hashed once per step")
        extra["connection_log_cache_codes"] = cache_codes_run(Xd, W, K, L, steps, warmup)
        log(f"  {extra['connection_log_cache_codes']['ms_per_step']:.3f} ms/step")
        log("paper-shape context runs")
        extra["paper_shapes"] = paper_shape_runs(steps, warmup)
        log("connection-log fp32, 16-bit counters")
        c16 = run_workload(Xd, W, K, L, "fp32", steps, warmup, counter_bits=16)
        extra["connection_log_counters16"] = c16
        log(f"  {c16['ms_per_step']:.3f} ms/step, {c16['saturated_increments_last_step']} saturated increments")
        log("connection-log shape, every row the same (one hot bucket per table)")
        Xhot = Xd[:1].expand(n, d).contiguous()
        extra["hot_bucket"] = run_workload(Xhot, W, K, L, "fp32", steps, warmup)
        log(f"  {extra['hot_bucket']['ms_per_step']:.3f} ms/step, update "
            f"{extra['hot_bucket']['phase_ms_per_step']['update_ms']:.4f} ms")
        del Xd, Xhot
        torch.cuda.empty_cache()
        # the large workloads: at least 10 timed steps after 3 warm-ups (median)
        big_steps, big_warm = max(10, steps // 2), max(3, warmup)
        extra["low_rank_1024"] = low_rank_runs(args.low_rank_n, big_steps, big_warm, args.sample_rows)
        extra["heavy_tail_4096"] = heavy_tail_runs(big_steps, big_warm, args.sample_rows)
        lg = serving_log(args.serving_requests)
        extra["serving_256"] = serving_runs(lg, window=10_000)
        extra["serving_256_graphs"] = serving_runs(lg, graphs=True)
        del lg
        torch.cuda.empty_cache()
        log("exact S(q, D) and estimator study")
        extra["exact_score_connection_log"] = exact_score_runs(X, W, K)
        log(f"  {extra['exact_score_connection_log']['ms_per_launch']:.3f} ms per launch")

    base = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle): all host threads, then one")
        base = cpu_baseline(X, W, K, L)
        log(f"  {base['value']:.3e} points/s on {base['cores']} threads; one core: {base['one_core']}")

    roof = dict(head["roofline"])
    tb = recorded_traffic("paper_1706_06664_amd/csrc/hash_fp32.hip",
                          "profiles/hash_fp32_direct_kernel__connection_log_494021x120.md")
    roof["traffic"] = tb
    if tb is not None:
        roof["traffic_unit"] = "bytes/launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE, copy-calibrated)"
        roof["algorithmic_bytes"] = 4.0 * n * d + 2.0 * n * L + 4.0 * d * K * L
    roof.pop("rows_per_launch", None)
    out = {
        "metric": "points/s insert+score (K=15,L=50)",
        "value": head["points_per_s"],
        "unit": "points/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": head["ms_per_step"],
        "ms_per_step_mean": head["ms_per_step_mean"],
        "timing": "median of the timed steps, HIP events on the launch stream, library profiling off",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "connection-log 494021x120, K=15, L=50, FP32 + FP64 refine",
                   "n": n, "d": d, "K": K, "L": L, "precision": "fp32", "refine": True},
        "roofline": r4(roof),
        "cpu_baseline": r4(base) if base else None,
        "hbm": r4({k: {"kernel": {"update": "update_lds_kernel", "score": "score_tables_kernel + mom_reduce_kernel"}.get(k, k), "ms": v["ms"],
                       "frac": v["frac"]} for k, v in head["hbm"].items()}),
        "phase_ms_per_step": r4(head["phase_ms_per_step"]),
        "refined_bit_frac": r4(head["refined_bit_frac"]),
        "flagged": head["flagged"],
    }
    if extra:
        out["workloads"] = workloads_block(extra)
    line = json.dumps(out, separators=(",", ":"))
    if args.detail:
        with open(args.detail, "w") as f:
            json.dump({"headline": head, **extra, "cpu_baseline": base}, f, indent=1, default=float)
    log(f"detail: {json.dumps(r4(extra), separators=(',', ':'))}")
    if len(line) > 8000:
        log(f"warning: JSON line is {len(line)} bytes")
    print(line, flush=True)


if __name__ == "__main__":
    main()
