"""GPU parity of streamlined refinement (Section 4.2.1): each round visits
consecutive vertex ranges in turn, each range's Visit and Update on the
lists the earlier ranges left.  The oracle runs the same schedule; ids,
distance bits, indegrees and the proposal and repair counts must agree."""
import numpy as np
import pytest
import torch

import oracle
from helpers import golden, line_points, pad_adj
from wl import CFG5_SMALL, to_gpu, workload

pytestmark = pytest.mark.gpu

fg = pytest.importorskip("paper_2603_21710_amd")

CASES = [
    ("cfg1", None),
    ("cfg1ov", None),
    ("cfg2", (2500, 2000)),
    ("cfg3", (300, 500, 700, 150, 900, 400, 1200, 650)),
    ("cfg4", (1200, 1000)),
    ("cfg5", CFG5_SMALL),
]
IDS = [c[0] for c in CASES]


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _stage1(name, sizes):
    cfg, X, graphs, _ = workload(name, sizes)
    m = to_gpu(X, graphs, cfg.metric)
    ids, dist, _ = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L))
    return cfg, X, graphs, m, ids, dist


def _check(ids, dist, T, st, oi, od, oT, ost, repair=True):
    gi = _u32(ids)
    bad = np.argwhere(gi != oi)
    assert bad.size == 0, f"{len(bad)} id mismatches, first {bad[:3].tolist()}"
    assert (dist.cpu().numpy().view(np.uint32) == od.view(np.uint32)).all()
    assert (_u32(T) == oT).all()
    assert st["proposals"] == ost["proposals"]
    if repair:
        assert st["repaired"] == ost["repaired"]


@pytest.mark.parametrize("name,sizes", CASES, ids=IDS)
@pytest.mark.parametrize("batches,join,repair", [(2, "mfma", True), (7, "mfma", True), (5, "fp32", True),
                                                 (3, "mfma", False)])
def test_streamlined_refine_matches_oracle(name, sizes, batches, join, repair):
    cfg, X, graphs, m, ids, dist = _stage1(name, sizes)
    print(f"case {name} N={X.shape[0]} batches={batches} join={join} repair={repair}", flush=True)
    oi, od, of, oT, ost = oracle.refine(X, graphs, _u32(ids), dist.cpu().numpy(), cfg.rounds, cfg.metric,
                                        do_repair=repair, batches=batches)
    flags = (0 if repair else fg.FGIM_FLAG_NO_REPAIR) | (fg.FGIM_FLAG_NO_MFMA_SCREEN if join == "fp32" else 0)
    T, st = fg.refine(m, fg.params(k=cfg.k, L=cfg.L, rounds=cfg.rounds, flags=flags, stream_batches=batches),
                      ids, dist, stats=True)
    _check(ids, dist, T, st, oi, od, oT, ost, repair)


def test_many_small_ranges_and_empty_ranges():
    # 64 ranges on 4,500 vertices, and more ranges than vertices on the
    # hand example (most ranges empty)
    cfg, X, graphs, m, ids, dist = _stage1("cfg2", (2500, 2000))
    print("case cfg2 batches=64", flush=True)
    oi, od, of, oT, ost = oracle.refine(X, graphs, _u32(ids), dist.cpu().numpy(), 2, cfg.metric, batches=64)
    T, st = fg.refine(m, fg.params(k=cfg.k, L=cfg.L, rounds=2, stream_batches=64), ids, dist, stats=True)
    _check(ids, dist, T, st, oi, od, oT, ost)

    g = golden("e2e_tiny.json")
    X = line_points(g["points"])
    subs = [(s["off"], pad_adj(s["adj"]), s["entry"]) for s in g["subs"]]
    m = to_gpu(X, subs, "l2")
    ids, dist, _ = fg.cross_query(m, fg.params(k=g["k"], L=g["L"]))
    print(f"case hand example N={X.shape[0]} batches=4096", flush=True)
    oi, od, of, oT, ost = oracle.refine(X, subs, _u32(ids), dist.cpu().numpy(), 2, k_rev=g["k_rev"],
                                        batches=4096)
    T, st = fg.refine(m, fg.params(k=g["k"], L=g["L"], rounds=2, k_rev=g["k_rev"], stream_batches=4096), ids,
                      dist, stats=True)
    _check(ids, dist, T, st, oi, od, oT, ost)


def test_streamlined_graph_capture_matches_eager():
    cfg, X, graphs, m, ids, dist = _stage1("cfg3", (300, 500, 700, 150, 900, 400, 1200, 650))
    runs = []
    for flags in (0, fg.FGIM_FLAG_NO_GRAPH_CAPTURE):
        print(f"case cfg3 batches=4 flags={flags}", flush=True)
        a_ids, a_d = ids.clone(), dist.clone()
        T, _ = fg.refine(m, fg.params(k=cfg.k, L=cfg.L, rounds=3, flags=flags, stream_batches=4), a_ids, a_d)
        runs.append((a_ids, a_d, T))
    assert all(torch.equal(x, y) for x, y in zip(runs[0], runs[1]))


def test_streamlined_buffer_overflow_reruns_to_the_same_result():
    cfg, X, graphs, m, ids, dist = _stage1("cfg1", None)
    runs = []
    for flags in (0, fg.FGIM_FLAG_MIN_BUFFERS):
        print(f"case cfg1 batches=2 flags={flags}", flush=True)
        a_ids, a_d = ids.clone(), dist.clone()
        T, st = fg.refine(m, fg.params(k=cfg.k, L=cfg.L, rounds=cfg.rounds, flags=flags, stream_batches=2),
                          a_ids, a_d, stats=True)
        runs.append((a_ids, a_d, T, st))
    assert runs[1][3]["refine_attempts"] >= 2
    assert all(torch.equal(x, y) for x, y in zip(runs[0][:3], runs[1][:3]))
    assert runs[0][3]["proposals"] == runs[1][3]["proposals"]


@pytest.mark.parametrize("name,sizes", [("cfg1ov", None), ("cfg3", (300, 500, 700, 150, 900, 400, 1200, 650))])
def test_streamlined_merge_matches_oracle(name, sizes):
    cfg, X, graphs, _ = workload(name, sizes)
    m = to_gpu(X, graphs, cfg.metric)
    print(f"case merge {name} batches=6", flush=True)
    pg, deg, entry, st = fg.merge(m, fg.params(k=cfg.k, L=cfg.L, R=cfg.R, rounds=cfg.rounds, stream_batches=6),
                                  stats=True)
    oi, odeg, oent = oracle.merge(X, graphs, cfg.k, cfg.L, cfg.rounds, cfg.R, cfg.metric, batches=6)
    assert (_u32(pg) == oi).all()
    assert (_u32(deg) == odeg).all()
    assert entry == oent
