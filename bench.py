"""Benchmark of the FGIM merge on one MI355X.

One step = one fgim_merge call (stage 1 cross-querying, stage 2 refinement
rounds with indegree repair, stage 3 prune + reverse fill) over a seeded
synthetic workload, with inputs resident in HBM.  Every form of the metric
is timed over the same K steps after W warm-up steps: the FP32 form (the
exact, parity form; it gives `value`) and the BF16 and FP8 forms (beam on a
low-precision copy, FP32 re-rank).  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--config cfg4] [--also cfg3]
                  [--forms fp32,bf16,fp8] [--no-cpu-baseline] [--no-recall]
                  [--no-parity] [--queries Q] [--parity-nodes N] [--autotune]
  python bench.py --refine-study cfg2,cfg3ov [--study-batches 1,4,16,64]
                  [--study-rounds 6] [--study-nodes 5000] [--steps K]

The second form compares refinement schedules instead: k-NNG recall and
stage-2 time after each number of rounds, synchronous and streamlined
(Section 4.2.1), from one stage-1 result.

Defaults: the precision-form workload (2 x 500,000 vectors, d = 768,
cosine), plus the batching-form workload (8 uneven sub-indexes, 2 M vectors,
d = 96, inner product) as `also`.

Roofline of the dominant kernel (the stage-1 beam search): algorithmic bytes
per launch (distance computations x row bytes + expansions x adjacency row
bytes + per-vertex query, local candidates and output) over the kernel's
duration, timed with hipEvents on the stream the kernel runs on.  The
denominators are the published 8 TB/s and a read stream's bandwidth
measured in the same run (the beam kernel only reads; a copy kernel's
read + write bandwidth is reported beside it).

Parity at full size: every form's stage-1 rows of sampled vertices are
compared bit for bit with the oracle's (the FP8 form excepted: the oracle's
exhaustive FP8 encoder is too slow for a full copy), and the FP32 form's
stage-3 rows of sampled vertices with the oracle's Algorithm 5 on the same
stage-2 lists.  A mismatch is reported in the line and makes the exit code 3.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "vectors merged/sec + k-NNG recall & search recall@10, FP32 vs BF16/FP8 form"
BEAM_SOURCES = ["paper_2603_21710_amd/csrc/beam_impl.h", "paper_2603_21710_amd/csrc/fgim_device.h",
                "paper_2603_21710_amd/csrc/beam_f32.hip", "paper_2603_21710_amd/csrc/beam_bf16.hip",
                "paper_2603_21710_amd/csrc/beam_fp8.hip"]
ROW_BYTES = {"fp32": 4, "bf16": 2, "fp8": 1}
DTYPE = {"fp32": "f32", "bf16": "bf16 scoring, f32 re-rank", "fp8": "fp8-e4m3 scoring, f32 re-rank"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def beam_source_hash() -> str:
    """sha256 of the beam-kernel sources with comments and blank space
    removed: a comment edit keeps committed counters valid, a code edit
    does not."""
    h = hashlib.sha256()
    for p in BEAM_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(cfg_name: str, precision: str):
    """HBM bytes per beam-kernel launch from the committed rocprofv3 counter
    summary, or None when absent or taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"beam_kernel_{cfg_name}_{precision}_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("beam sources sha256") != beam_source_hash():
        return None
    try:
        return float(vals["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def copy_peak_gbs(dev, gib: float = 2.0, reps: int = 20) -> float:
    """Bandwidth of a plain device-to-device copy (read + write bytes over
    time, median of reps): the measured HBM ceiling the roofline is also
    quoted against."""
    n = int(gib * (1 << 30)) // 4
    src = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / float(np.median(ts)) / 1e9


def read_peak_gbs(fg, dev, gib: float = 4.0, reps: int = 20) -> float:
    """Bandwidth of a plain read stream (the library's read-stream kernel:
    bytes read over time, median of reps), the ceiling of a kernel that only
    reads, such as the beam search; a copy is slower since it also writes."""
    n = int(gib * (1 << 30)) // 4
    src = torch.empty(n, dtype=torch.int32, device=dev).fill_(1)
    for _ in range(3):
        fg.read_stream(src)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fg.read_stream(src)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    del src
    torch.cuda.empty_cache()
    return n * 4 / float(np.median(ts)) / 1e9


def refine_study(fg, cfg, batch_list, max_rounds, n_nodes, reps, dev):
    """Refinement schedules compared on one workload: k-NNG recall and
    stage-2 time after r = 1..max_rounds rounds, synchronous (B = 1) and
    streamlined (B vertex ranges per round), all from one stage-1 result."""
    from workloads.evaluate import exact_knn_screened, tie_recall
    X, graphs, reach, build_s = build_inputs(cfg, "cuda")
    N = X.shape[0]
    Xd = torch.from_numpy(X).to(dev)
    gl = [(torch.from_numpy(a.view(np.int32)).to(dev), int(e)) for _, a, e in graphs]
    m = fg.Merge(Xd, gl, cfg.metric)
    knodes = sample_nodes(N, n_nodes, 7)
    _, kd, _ = exact_knn_screened(X, X[knodes], cfg.k, cfg.metric, exclude=knodes, Xdev=Xd)
    ids0, dist0, st1 = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L), stats=True)

    def recall(ids):
        return tie_recall(X, X[knodes], fg.as_uint32(ids)[knodes], kd[:, -1], cfg.k, cfg.metric)

    out = {"workload": cfg.name, "N": N, "k": cfg.k, "rounds_configured": cfg.rounds,
           "stage1_ms": round(st1["ms_stage"][0], 3), "knng_recall_after_stage1": round(recall(ids0), 5),
           "recall_nodes": len(knodes), "schedules": {}}
    for B in batch_list:
        rows = []
        for r in range(1, max_rounds + 1):
            p = fg.params(k=cfg.k, L=cfg.L, rounds=r, stream_batches=B)
            ms = []
            for _ in range(reps + 1):
                ids, dist = ids0.clone(), dist0.clone()
                _, st = fg.refine(m, p, ids, dist, stats=True)
                ms.append(st["ms_stage"][1])
            rows.append({"rounds": r, "stage2_ms": round(float(np.median(ms[1:])), 3),
                         "knng_recall": round(recall(ids), 5), "proposals": st["proposals"]})
            log(f"{cfg.name} B={B} rounds={r}: {rows[-1]}")
        out["schedules"][str(B)] = rows
    # rounds and time each schedule needs to reach what the synchronous
    # rounds reach after the configured number of rounds
    target = out["schedules"]["1"][cfg.rounds - 1]["knng_recall"] if 1 in batch_list else None
    if target is not None:
        out["target_recall"] = target
        for B in batch_list:
            hit = [row for row in out["schedules"][str(B)] if row["knng_recall"] >= target]
            if hit:
                t = out["stage1_ms"] + hit[0]["stage2_ms"]
                out.setdefault("to_target", {})[str(B)] = {
                    "rounds": hit[0]["rounds"], "stage2_ms": hit[0]["stage2_ms"],
                    "stage1_plus_2_vectors_per_s": round(N / (t / 1e3), 1)}
    return out


def _timed(fn, reps=3):
    """(result of the last call, median seconds over reps after one untimed call)."""
    out = fn()
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return out, float(np.median(ts))


def rows_study(fg, cfg, n_queries, dev):
    """The follow-on rows on one full-size workload: the selection rules
    (alpha-RNG, tau-MNG; on inner-product data through the MIPS transform),
    validity (a quarter of the vertices dropped), and HNSW-adaptive merging
    (the upper layers and the layered search against the flat one), each
    with its time and search recall@10 against FP64 truth."""
    from workloads import make_queries
    from workloads.evaluate import exact_knn_screened, tie_recall
    X, graphs, _, _ = build_inputs(cfg, "cuda")
    N = X.shape[0]
    Xd = torch.from_numpy(X).to(dev)
    gl = [(torch.from_numpy(a.view(np.int32)).to(dev), int(e)) for _, a, e in graphs]
    Q = make_queries(cfg, n_queries)
    Qd = torch.from_numpy(Q).to(dev)
    _, qd, _ = exact_knn_screened(X, Q, 10, cfg.metric, Xdev=Xd)
    out = {"workload": cfg.name, "N": N, "queries": n_queries}

    def recall_of(pg, entry, Xs=Xd, Qs=Qd, metric=cfg.metric, kth=qd[:, -1], L=64):
        found, _ = fg.search(Xs, pg, entry, Qs, L, 10, metric)
        return round(tie_recall(X, Q, fg.as_uint32(found), kth, 10, cfg.metric), 5)

    base = fg.params(k=cfg.k, L=cfg.L, R=cfg.R, rounds=cfg.rounds)
    m = fg.Merge(Xd, gl, cfg.metric)
    (pg, deg, entry, st), t = _timed(lambda: fg.merge(m, base, stats=True), 2)
    out["rng"] = {"merge_ms": round(t * 1e3, 2), "stage3_ms": round(st["ms_stage"][2], 3),
                  "mean_degree": round(float(deg.float().mean()), 3), "recall@10_L64": recall_of(pg, entry)}
    log(f"{cfg.name} rng: {out['rng']}")

    # selection rules: metric ones, so inner-product data goes through MIPS
    if cfg.metric == "ip":
        (Xt, Mx), t = _timed(lambda: fg.mips_to_l2(Xd), 5)
        d = X.shape[1]
        # read every row once, write every transformed row once, and the
        # squared length parked and read back (8 B a row)
        moved = N * d * 4 + N * (d + 4) * 4 + N * 8
        out["mips_to_l2"] = {"ms": round(t * 1e3, 3), "bytes": moved, "GB/s": round(moved / t / 1e9, 1),
                             "frac_of_8TB/s": round(moved / t / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"{cfg.name} mips: {out['mips_to_l2']}")
        Xs = Xt.contiguous()
        Qs = torch.nn.functional.pad(Qd, (0, 4))
        rmetric = "l2"
    else:
        Xs, Qs, rmetric = Xd, Qd, cfg.metric
    mr = fg.Merge(Xs, gl, rmetric)
    first = fg.merge(mr, base)[0]
    tau = 0.1 * float(np.median(np.sqrt(np.maximum(
        ((Xs[:2000] - Xs[first[:2000, 0].long().clamp_min(0)]) ** 2).sum(1).cpu().numpy(), 0.0))))
    for rule, param in (("rng", 0.0), ("alpha", 1.2), ("tau", tau)):
        p = fg.params(k=cfg.k, L=cfg.L, R=cfg.R, rounds=cfg.rounds, select_rule=rule, select_param=param)
        (pg, deg, entry, st), t = _timed(lambda: fg.merge(mr, p, stats=True), 2)
        out.setdefault("rules", {})[rule] = {
            "param": round(param, 6), "metric": rmetric, "merge_ms": round(t * 1e3, 2),
            "stage3_ms": round(st["ms_stage"][2], 3), "mean_degree": round(float(deg.float().mean()), 3),
            "recall@10_L64": recall_of(pg, entry, Xs, Qs, rmetric)}
        log(f"{cfg.name} {rule}: {out['rules'][rule]}")

    # validity: a quarter of the vertices dropped (seeded)
    rng = np.random.default_rng(4242)
    valid = (rng.random(N) >= 0.25).astype(np.uint8)
    keep = np.nonzero(valid)[0]
    _, vqd, _ = exact_knn_screened(X[keep], Q, 10, cfg.metric)
    mv = fg.Merge(Xd, gl, cfg.metric, valid=torch.from_numpy(valid).to(dev))
    (pg, deg, entry, st), t = _timed(lambda: fg.merge(mv, base, stats=True), 2)
    found, _ = fg.search(Xd, pg, entry, Qd, 64, 10, cfg.metric)
    fnd = fg.as_uint32(found)
    out["validity"] = {"dropped": int(N - keep.size), "merge_ms": round(t * 1e3, 2),
                       "stages_ms": [round(x, 3) for x in st["ms_stage"]],
                       "recall@10_L64": round(tie_recall(X, Q, fnd, vqd[:, -1], 10, cfg.metric), 5),
                       "dropped_in_results": int(np.isin(fnd[fnd != 0xFFFFFFFF], np.nonzero(valid == 0)[0]).sum())}
    log(f"{cfg.name} validity: {out['validity']}")

    # HNSW-adaptive: levels drawn as HNSW draws them (mL = 1 / ln M), M = R
    M = cfg.R
    lv = np.minimum(np.floor(-np.log(np.random.default_rng(77).random(N)) / np.log(M)), 8).astype(np.uint8)
    lvd = torch.from_numpy(lv).to(dev)
    layers, t = _timed(lambda: fg.hnsw_layers(Xd, lvd, M, 64, cfg.metric), 2)
    out["hnsw"] = {"M": M, "ef": 64, "layers": len(layers[2]), "members": layers[2], "build_ms": round(t * 1e3, 2),
                   "search": {}}
    pg, deg, entry, _ = fg.merge(m, base)
    for L in (16, 32, 64):
        (fl, _), tl = _timed(lambda: fg.search_layers(Xd, pg, layers, M, Qd, L, 10, cfg.metric), 3)
        (ff, _), tf = _timed(lambda: fg.search(Xd, pg, entry, Qd, L, 10, cfg.metric), 3)
        out["hnsw"]["search"][str(L)] = {
            "layered": {"queries/s": round(n_queries / tl, 1),
                        "recall@10": round(tie_recall(X, Q, fg.as_uint32(fl), qd[:, -1], 10, cfg.metric), 5)},
            "flat": {"queries/s": round(n_queries / tf, 1),
                     "recall@10": round(tie_recall(X, Q, fg.as_uint32(ff), qd[:, -1], 10, cfg.metric), 5)}}
        log(f"{cfg.name} hnsw L={L}: {out['hnsw']['search'][str(L)]}")
    return out


def build_inputs(cfg, device):
    from workloads import build_input_pg, make_vectors, reach_fraction, split_sizes
    t0 = time.time()
    X = make_vectors(cfg)
    graphs, reach, deg = [], [], []
    parts = split_sizes(cfg)
    for i, (off, n) in enumerate(parts):
        t1 = time.time()
        pg = build_input_pg(X[off:off + n], cfg.r_in, cfg.metric, device=device)
        graphs.append((off, pg.adj, pg.entry))
        reach.append(reach_fraction(pg.adj, pg.entry))
        deg.append(pg.mean_degree)
        if n >= 1_000_000:
            log(f"input graph {i + 1}/{len(parts)}: n={n} in {time.time() - t1:.1f}s")
    build_s = time.time() - t0
    log(f"inputs {cfg.name}: N={X.shape[0]} d={X.shape[1]} h={len(graphs)} built in {build_s:.1f}s; "
        f"input reach {min(reach):.4f}..{max(reach):.4f}, mean degree {np.mean(deg):.2f}")
    return X, graphs, reach, build_s


def counting_lanes(used_p, dim):
    """Lanes per distance of the distance-counting launch: half of the timed
    launch's P where that keeps at most four chunks per lane (doubling from two
    chunks per lane leaves one, the slowest shape), else double P where it
    fits, else half of P; never P itself, so a kernel trace tells the two
    launches apart."""
    chunks = max(1, dim // 4)
    if used_p >= 2 and chunks // (used_p // 2) <= 4:
        return used_p // 2
    if used_p * 2 <= min(64, chunks):
        return used_p * 2
    return max(1, used_p // 2)


def beam_roofline(fg, m, cfg, X, graphs, precision, st, beam_ms, peak_meas, count_launch=True):
    """Roofline of the beam kernel for one form (see the module docstring)."""
    # The distance count is measured with the largest visited cache, which
    # re-scores almost no vertex, so it is (slightly above) the count of
    # Algorithm 1.  That counting launch uses another lanes-per-distance
    # (another kernel instance, the same count), so a kernel trace of this
    # script lists the timed launches under their own name.
    used_p = st["lanes_per_dist"]
    alt_p = counting_lanes(used_p, X.shape[1])
    st_big = st
    if count_launch:
        log(f"{cfg.name} {precision}: counting launch ({alt_p} lanes per distance, 16384 visited slots)")
        _, _, st_big = fg.cross_query(m, fg.params(k=cfg.k, L=st["L_used"], precision=precision,
                                                   visited_slots=16384, waves_per_cu=8,
                                                   lanes_per_dist=alt_p), stats=True)
    d, k = X.shape[1], cfg.k
    ndc, nexp, searches = st_big["ndc"], st_big["expansions"], st_big["searches"]
    local = sum(int((a != 0xFFFFFFFF).sum()) for _, a, _ in graphs)
    stride_mean = float(np.mean([a.shape[1] for _, a, _ in graphs]))
    row_bytes = d * ROW_BYTES[precision] + (4 if precision == "fp8" else 0)
    alg_bytes = (ndc * row_bytes + nexp * stride_mean * 4
                 + X.shape[0] * (d * 4 + stride_mean * 4 + k * 8) + local * d * 4)
    if precision != "fp32":
        alg_bytes += searches * min(st["L_used"], 2 * cfg.k) * d * 4
    kern_s = float(np.mean(beam_ms)) / 1e3
    achieved = alg_bytes / kern_s / 1e9
    traffic = measured_traffic(cfg.name, precision)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "measured_peak": round(peak_meas, 1), "measured_peak_kind": "read stream (fgim_read_stream over 4 GiB)",
            "frac_of_measured_peak": round(achieved / peak_meas, 4),
            "traffic_frac_of_measured_peak": None if traffic is None else round(traffic / kern_s / 1e9 / peak_meas, 4),
            "kernel": "beam_kernel (stage-1 cross-query)", "kernel_ms": round(kern_s * 1e3, 3),
            "algorithmic_bytes": int(alg_bytes), "ndc_per_search": round(ndc / max(1, searches), 2),
            "expansions_per_search": round(nexp / max(1, searches), 2),
            "ndc_source": "counting launch, 16384 visited slots" if count_launch else "timed launch",
            "launch": {"lanes_per_dist": st["lanes_per_dist"], "waves_per_cu": st["waves_per_cu"],
                       "visited_slots": st["visited_slots"]},
            "beam_sources_sha256": beam_source_hash()}
    # Algorithmic bytes count every row gather as an HBM read; rows re-read
    # by concurrent searches (the entry region of each graph above all) hit
    # L2, so `frac` can pass what HBM alone could serve: `cache_assisted`
    # says the algorithmic bytes exceed the counted fabric traffic by more
    # than 5 %.  `traffic` (FETCH_SIZE + WRITE_SIZE) still counts reads the
    # memory-side cache serves, so it bounds HBM bytes from above;
    # `traffic_exceeds_read_stream` says its rate passed the read stream
    # measured in this run, which only the memory-side cache can explain.
    roof["cache_assisted"] = bool(traffic is not None and alg_bytes > 1.05 * traffic)
    roof["algorithmic_over_traffic"] = None if traffic is None else round(alg_bytes / traffic, 4)
    roof["traffic_frac"] = None if traffic is None else round(traffic / kern_s / 1e9 / HBM_PEAK_GBS, 4)
    roof["traffic_exceeds_read_stream"] = bool(traffic is not None and traffic / kern_s / 1e9 > peak_meas)
    return roof


def sample_nodes(N: int, n: int, seed: int) -> np.ndarray:
    return np.sort(np.random.default_rng(seed).choice(N, min(n, N), replace=False))


def stage1_parity(fg, m, cfg, X, graphs, precision, L_used, nodes, deq=None):
    """Stage-1 rows of `nodes` from the GPU (the timed launch configuration)
    against the oracle's, bit for bit (ids and distance bits).  Returns the
    report and the oracle's time per vertex."""
    import oracle
    ids, dist, _ = fg.cross_query(m, fg.params(k=cfg.k, L=L_used, precision=precision))
    gi = ids.cpu().numpy().view(np.uint32)[nodes]
    gd = dist.cpu().numpy()[nodes]
    t0 = time.perf_counter()
    if precision == "fp32":
        oi, od, _ = oracle.cross_query(X, graphs, cfg.k, L_used, cfg.metric, nodes=nodes)
    else:
        oi, od, _ = oracle.cross_query(X, graphs, cfg.k, L_used, cfg.metric, nodes=nodes, Xs=deq,
                                       rerank=min(L_used, 2 * cfg.k))
    t = (time.perf_counter() - t0) / len(nodes)
    bad = np.nonzero((gi != oi).any(1) | (gd.view(np.uint32) != od.view(np.uint32)).any(1))[0]
    rep = {"vertices": int(len(nodes)), "mismatched_vertices": int(bad.size)}
    if bad.size:
        rep["first_mismatch"] = int(nodes[bad[0]])
    return rep, ids, dist, t


def stage23_parity(fg, m, cfg, X, p, ids, dist, nodes):
    """Stage 2 on the GPU from its stage-1 lists, checked by properties that
    hold at any size (sorted unique lists without self-loops, distances equal
    to the oracle's distance of each sampled pair, indegrees equal to a
    recount); stage 3 on those lists, sampled rows against the oracle's
    Algorithm 5 on the same lists."""
    import oracle
    T, _ = fg.refine(m, p, ids, dist)
    li = ids.cpu().numpy().view(np.uint32)
    ld = dist.cpu().numpy()
    Th = T.cpu().numpy().view(np.uint32)
    N = li.shape[0]
    rec = np.bincount(li[li != 0xFFFFFFFF].astype(np.int64), minlength=N)
    bad2 = 0
    for u in nodes[:2000]:
        row = [(float(ld[u, t]), int(li[u, t])) for t in range(cfg.k) if li[u, t] != 0xFFFFFFFF]
        ok = row == sorted(row) and len({v for _, v in row}) == len(row) and all(v != u for _, v in row)
        ok = ok and all(d == oracle.distance(X[u], X[v], cfg.metric) for d, v in row)
        bad2 += not ok
    pg, deg = fg.prune(m, p, ids, dist, T)
    pi, pd, pdeg = oracle.prune_rows(X, li, ld, Th, cfg.R, nodes[:2000], cfg.metric)
    gp = pg.cpu().numpy().view(np.uint32)[nodes[:2000]]
    gdeg = deg.cpu().numpy()[nodes[:2000]]
    bad3 = int(((gp != pi).any(1) | (gdeg != pdeg)).sum())
    return {"stage2_property_checked_vertices": int(min(2000, len(nodes))),
            "stage2_bad_vertices": int(bad2), "stage2_indegree_recount_ok": bool((rec == Th).all()),
            "stage3_vertices": int(min(2000, len(nodes))), "stage3_mismatched_vertices": bad3}


def measure(fg, cfg, forms, args, dev, peak_meas, with_parity, with_recall):
    """Build the inputs of one workload and time every form over K steps."""
    from workloads import make_queries
    from workloads.evaluate import exact_knn_screened, tie_recall
    X, graphs, reach, build_s = build_inputs(cfg, "cuda")
    Xd = torch.from_numpy(X).to(dev)
    gl = [(torch.from_numpy(a.view(np.int32)).to(dev), int(e)) for _, a, e in graphs]
    out = {"workload": cfg.name, "sizes": list(cfg.sizes), "dim": cfg.dim, "metric": cfg.metric,
           "r_in": cfg.r_in, "k": cfg.k, "L": cfg.L, "rounds": cfg.rounds, "R": cfg.R,
           "input_build_s": round(build_s, 1), "input_reach": [round(r, 4) for r in reach], "forms": {}}
    nodes = sample_nodes(X.shape[0], args.parity_nodes, 12345)
    gt = None
    if with_recall:
        t0 = time.time()
        Q = make_queries(cfg, args.queries)
        knodes = sample_nodes(X.shape[0], args.queries, 7)
        def prog(what):
            return lambda done, total: log(f"ground truth {cfg.name} {what}: {done}/{total}")
        log(f"ground truth {cfg.name}: {len(knodes)} vertices and {Q.shape[0]} queries")
        _, kd, fb1 = exact_knn_screened(X, X[knodes], cfg.k, cfg.metric, exclude=knodes, Xdev=Xd,
                                        progress=prog("vertices"))
        _, qd, fb2 = exact_knn_screened(X, Q, 10, cfg.metric, Xdev=Xd, progress=prog("queries"))
        gt = (Q, knodes, kd, qd)
        log(f"ground truth {cfg.name}: {time.time() - t0:.1f}s (fallbacks {fb1}, {fb2})")
    for form in forms:
        t0 = time.time()
        lowp = lows = None
        quant_ms = None
        if form != "fp32":
            torch.cuda.synchronize()
            tq = time.perf_counter()
            lowp, lows = fg.quantize(Xd, form)
            torch.cuda.synchronize()
            quant_ms = (time.perf_counter() - tq) * 1e3
        m = fg.Merge(Xd, gl, cfg.metric, lowp, lows)
        p = fg.params(k=cfg.k, L=cfg.L, R=cfg.R, rounds=cfg.rounds, precision=form, autotune=args.autotune)
        tune_ms = None
        for _ in range(args.warmup):
            _, _, _, stw = fg.merge(m, p, stats=True)
            tune_ms = stw["ms_tune"] if tune_ms is None else tune_ms
            if sum(stw["ms_stage"]) > 5000:
                log(f"{cfg.name} {form}: warm-up merge {sum(stw['ms_stage']):.0f} ms")
        torch.cuda.synchronize()
        beam_ms, stage_ms = [], []
        t1 = time.perf_counter()
        for step in range(args.steps):
            pg, deg, entry, st = fg.merge(m, p, stats=True)
            beam_ms.append(st["ms_beam_kernel"])
            stage_ms.append(st["ms_stage"])
            if sum(st["ms_stage"]) > 5000:  # long merges: a line per step
                log(f"{cfg.name} {form}: step {step + 1}/{args.steps} {sum(st['ms_stage']):.0f} ms")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t1
        ms = wall * 1e3 / args.steps
        f = {"value": round(X.shape[0] / (ms / 1e3), 1), "unit": "vectors/s", "ms_per_step": round(ms, 3),
             "dtype": DTYPE[form], "L_used": st["L_used"],
             "stages_ms": [round(x, 3) for x in np.mean(stage_ms, 0).tolist()],
             "refine": {"proposals": st["proposals"], "rechecked": st["rechecked"], "repaired": st["repaired"],
                        "repair_batches": st["repair_batches"], "repair_alone": st["repair_alone"],
                        "attempts": st["refine_attempts"]}}
        if quant_ms is not None:
            f["quantize_ms"] = round(quant_ms, 3)
        f["roofline"] = beam_roofline(fg, m, cfg, X, graphs, form, st, beam_ms, peak_meas,
                                      count_launch=not args.no_ndc_count)
        if args.autotune:
            f["roofline"]["launch"]["tune_ms_first_call"] = round(tune_ms or 0.0, 1)
        log(f"{cfg.name} {form}: {ms:.2f} ms/step, stages {f['stages_ms']} ms, beam kernel "
            f"{np.mean(beam_ms):.2f} ms ({f['roofline']['frac']} of 8 TB/s algorithmic)")
        ids = dist = None
        if with_parity and form != "fp8":
            deq = None
            if form == "bf16":
                import oracle
                deq = oracle.quantize_bf16(X)[1]
            rep, ids, dist, t_vertex = stage1_parity(fg, m, cfg, X, graphs, form, st["L_used"], nodes, deq)
            f["parity"] = {"stage1": rep}
            if form == "fp32":
                f["oracle_stage1_ms_per_vertex"] = t_vertex * 1e3
                f["parity"].update(stage23_parity(fg, m, cfg, X, p, ids, dist, nodes))
                ids = dist = None
            log(f"{cfg.name} {form} parity: {f['parity']}")
        if with_recall:
            Q, knodes, kd, qd = gt
            if ids is None:
                ids, dist, _ = fg.cross_query(m, fg.params(k=cfg.k, L=st["L_used"], precision=form))
            fg.refine(m, p, ids, dist)
            knn = fg.as_uint32(ids)
            sr = {}
            Qd = torch.from_numpy(Q).to(dev)
            for Ls in (16, 32, 64, 128):
                found, _ = fg.search(Xd, pg, entry, Qd, Ls, 10, cfg.metric)
                sr[str(Ls)] = round(tie_recall(X, Q, fg.as_uint32(found), qd[:, -1], 10, cfg.metric), 5)
            f["quality"] = {"knng_recall": round(tie_recall(X, X[knodes], knn[knodes], kd[:, -1], cfg.k,
                                                            cfg.metric), 5),
                            "search_recall@10": sr}
        out["forms"][form] = f
        del m, lowp, lows
        torch.cuda.empty_cache()
        log(f"{cfg.name} {form} done in {time.time() - t0:.1f}s")
    if with_recall:
        out["quality_setup"] = {"knng_recall_nodes": len(gt[1]), "queries": int(gt[0].shape[0]),
                                "search_L_headline": 64,
                                "ground_truth": "FP64 direct form, FP32 GPU shortlist proved complete"}
    base = out["forms"].get("fp32")
    if base is not None:
        for form, f in out["forms"].items():
            if form == "fp32":
                continue
            f["speedup_vs_fp32"] = round(f["value"] / base["value"], 4)
            if "quality" in f and "quality" in base:
                f["search_recall_gap_pp_L64"] = round(
                    (base["quality"]["search_recall@10"]["64"] - f["quality"]["search_recall@10"]["64"]) * 100, 3)
                f["knng_recall_gap_pp"] = round((base["quality"]["knng_recall"] - f["quality"]["knng_recall"]) * 100, 3)
    return out, X, graphs


def cpu_baseline(cfg, X, graphs, t_s1_vertex, nodes_used):
    """The oracle timed on this host: stage 1 on the seeded vertices of the
    full workload that the parity check ran (its time per vertex), one
    thread on 500 of them, and stages 2-3 in full on a 2 x 20,000 draw of
    the same distribution and parameters.  Returns vectors/s of the summed
    per-vertex cost."""
    import oracle
    from workloads import build_input_pg, make_vectors, split_sizes
    threads = oracle.default_threads()
    nodes = sample_nodes(X.shape[0], nodes_used, 12345)
    if t_s1_vertex is None:
        t0 = time.perf_counter()
        oracle.cross_query(X, graphs, cfg.k, cfg.L, cfg.metric, nodes=nodes, threads=threads)
        t_s1_vertex = (time.perf_counter() - t0) / len(nodes)
    one = nodes[:500]
    t0 = time.perf_counter()
    oracle.cross_query(X, graphs, cfg.k, cfg.L, cfg.metric, nodes=one, threads=1)
    t_s1_one = (time.perf_counter() - t0) / len(one)
    small = cfg.scaled(tuple(min(s, 20000) for s in cfg.sizes[:2]) if cfg.h > 2 else (20000,) * cfg.h)
    Xs = make_vectors(small)
    gs = []
    for off, n in split_sizes(small):
        pg = build_input_pg(Xs[off:off + n], small.r_in, small.metric)
        gs.append((off, pg.adj, pg.entry))
    ids, dd, _ = oracle.cross_query(Xs, gs, small.k, small.L, small.metric, threads=threads)
    t0 = time.perf_counter()
    i2, d2, _, T, _ = oracle.refine(Xs, gs, ids, dd, small.rounds, small.metric, threads=threads)
    oracle.prune(Xs, i2, d2, T, small.R, small.metric, threads=threads)
    t_s23 = (time.perf_counter() - t0) / Xs.shape[0]
    per_vec = t_s1_vertex + t_s23
    return {"value": 1.0 / per_vec, "unit": "vectors/s", "cores": threads, "kind": "oracle",
            "sample": (f"stage 1 on {len(nodes)} seeded vertices of the full workload "
                       f"({t_s1_vertex * 1e3:.3f} ms/vertex); stages 2-3 in full on a "
                       f"{'+'.join(str(s) for s in small.sizes)} draw of the same distribution "
                       f"({t_s23 * 1e3:.3f} ms/vertex)"),
            "host_nproc": os.cpu_count(), "threads": threads,
            "threads_note": "one GPU's share of the host is 16 cores; the oracle uses min(16, nproc) threads",
            "cpu": cpu_model(),
            "stage1_ms_per_vertex_1thread": round(t_s1_one * 1e3, 4)}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="cfg4")
    ap.add_argument("--also", default="cfg3", help="comma-separated extra workloads, or 'none'")
    ap.add_argument("--forms", default="fp32,bf16,fp8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--queries", type=int, default=10000)
    ap.add_argument("--parity-nodes", type=int, default=10000)
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--no-ndc-count", action="store_true",
                    help="take the distance count from the timed launch (re-scored ids included) "
                         "instead of an extra counting launch; for the largest workloads")
    ap.add_argument("--refine-study", default="",
                    help="comma-separated workloads: compare synchronous and streamlined refinement "
                         "(k-NNG recall and stage-2 time per round) instead of the merge benchmark")
    ap.add_argument("--study-batches", default="1,4,16,64")
    ap.add_argument("--study-rounds", type=int, default=6)
    ap.add_argument("--study-nodes", type=int, default=5000)
    ap.add_argument("--rows-study", default="",
                    help="comma-separated workloads: time the selection rules, MIPS transform, validity "
                         "and HNSW layers instead of the merge benchmark")
    ap.add_argument("--study-queries", type=int, default=10000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the merge is built and measured on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import paper_2603_21710_amd as fg
    from workloads import get_config

    forms = [f for f in args.forms.split(",") if f]
    if not forms or any(f not in ROW_BYTES for f in forms):
        print(f"--forms must list fp32, bf16 and/or fp8, got {args.forms!r}", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.rows_study:
        res = {"study": "follow-on rows", "results": []}
        for name in args.rows_study.split(","):
            res["results"].append(rows_study(fg, get_config(name), args.study_queries, dev))
        print(json.dumps(res), flush=True)
        return
    if args.refine_study:
        batches = [int(b) for b in args.study_batches.split(",") if b]
        res = {"study": "refinement schedule", "unit": "vectors/s", "steps": args.steps, "results": []}
        for name in args.refine_study.split(","):
            res["results"].append(refine_study(fg, get_config(name), batches, args.study_rounds, args.study_nodes,
                                               args.steps, dev))
        print(json.dumps(res), flush=True)
        return
    peak = copy_peak_gbs(dev)
    log(f"copy kernel: {peak:.1f} GB/s (read + write)")
    rpeak = read_peak_gbs(fg, dev)
    log(f"read stream: {rpeak:.1f} GB/s")

    cfg = get_config(args.config)
    head, X, graphs = measure(fg, cfg, forms, args, dev, rpeak, not args.no_parity, not args.no_recall)
    lead = forms[0]
    hf = head["forms"][lead]
    out = {"metric": METRIC, "value": hf["value"], "unit": "vectors/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": hf["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": hf["dtype"], "data": "synthetic (seeded; stands in for the paper's datasets)",
           "config": {"workload": cfg.name, "sizes": list(cfg.sizes), "dim": cfg.dim,
                      "metric": cfg.metric, "r_in": cfg.r_in, "k": cfg.k, "L": hf["L_used"],
                      "rounds": cfg.rounds, "R": cfg.R, "precision": lead, "forms": forms,
                      "parallelism": "1 GPU"},
           "stages_ms": hf["stages_ms"], "roofline": hf["roofline"], "copy_peak_gbs": round(peak, 1),
           "read_peak_gbs": round(rpeak, 1),
           "forms": head["forms"]}
    for key in ("input_build_s", "input_reach", "quality_setup"):
        if key in head:
            out[key] = head[key]
    also = [] if args.also in ("", "none") else [a for a in args.also.split(",") if a]
    out["also"] = {}
    for name in also:
        o, _, _ = measure(fg, get_config(name), forms, args, dev, rpeak, not args.no_parity,
                          not args.no_recall)
        out["also"][name] = o
    if not args.no_cpu_baseline:
        t0 = time.time()
        t_v = hf.get("oracle_stage1_ms_per_vertex")
        out["cpu_baseline"] = cpu_baseline(cfg, X, graphs, None if t_v is None else t_v / 1e3,
                                           args.parity_nodes)
        log(f"cpu baseline: {out['cpu_baseline']} ({time.time() - t0:.1f}s)")
    bad = []
    for wl, fs in [(cfg.name, head["forms"])] + [(n, o["forms"]) for n, o in out["also"].items()]:
        for form, f in fs.items():
            par = f.get("parity", {})
            if par.get("stage1", {}).get("mismatched_vertices", 0) or par.get("stage3_mismatched_vertices", 0) \
                    or par.get("stage2_bad_vertices", 0) or par.get("stage2_indegree_recount_ok") is False:
                bad.append(f"{wl}/{form}")
    out["parity_ok"] = not bad
    print(json.dumps(out), flush=True)
    if bad:
        log(f"PARITY MISMATCH in {bad}")
        sys.exit(3)


if __name__ == "__main__":
    main()
