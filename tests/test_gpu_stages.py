"""GPU parity of stage 2 (refinement rounds with indegree repair,
Algorithms 3-4), stage 3 (neighbour selection + reverse fill, Algorithm 5)
and the full merge against the oracle.  Each stage gets identical inputs on
both sides, so a mismatch points at that stage."""
import numpy as np
import pytest
import torch

import oracle
from helpers import NONE, golden, line_points, pad_adj, pad_ids
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


@pytest.mark.parametrize("name,sizes", CASES, ids=IDS)
@pytest.mark.parametrize("rounds,repair,join", [(1, True, "mfma"), (2, False, "mfma"), (None, True, "mfma"),
                                                (None, True, "fp32")])
def test_refine_matches_oracle(name, sizes, rounds, repair, join):
    cfg, X, graphs, m, ids, dist = _stage1(name, sizes)
    rounds = cfg.rounds if rounds is None else rounds
    print(f"case {name} rounds={rounds} repair={repair}", flush=True)
    oi, od, of, oT, ost = oracle.refine(X, graphs, _u32(ids), dist.cpu().numpy(), rounds,
                                        cfg.metric, do_repair=repair)
    flags = (0 if repair else fg.FGIM_FLAG_NO_REPAIR) | (fg.FGIM_FLAG_NO_MFMA_SCREEN if join == "fp32" else 0)
    T, st = fg.refine(m, fg.params(k=cfg.k, L=cfg.L, rounds=rounds, flags=flags), ids, dist,
                      stats=True)
    if join == "mfma":
        # the screen re-scores a fraction of the pairs and never misses a proposal
        assert 0 < st["rechecked"]
    gi = _u32(ids)
    bad = np.argwhere(gi != oi)
    assert bad.size == 0, f"{len(bad)} id mismatches, first {bad[:3].tolist()}"
    assert (dist.cpu().numpy().view(np.uint32) == od.view(np.uint32)).all()
    assert (_u32(T) == oT).all()
    if repair:
        assert st["repaired"] == ost["repaired"]
    assert st["proposals"] == ost["proposals"]


@pytest.mark.parametrize("k_rev", [4, 64])
def test_refine_reverse_cap(k_rev):
    cfg, X, graphs, m, ids, dist = _stage1("cfg1ov", None)
    oi, od, of, oT, _ = oracle.refine(X, graphs, _u32(ids), dist.cpu().numpy(), 2, cfg.metric,
                                      k_rev=k_rev)
    T, _ = fg.refine(m, fg.params(k=cfg.k, L=cfg.L, rounds=2, k_rev=k_rev), ids, dist)
    assert (_u32(ids) == oi).all() and (_u32(T) == oT).all()


def test_graph_capture_matches_eager():
    cfg, X, graphs, m, ids, dist = _stage1("cfg3", (300, 500, 700, 150, 900, 400, 1200, 650))
    a_ids, a_d = ids.clone(), dist.clone()
    Ta, _ = fg.refine(m, fg.params(k=cfg.k, L=cfg.L, rounds=3), a_ids, a_d)
    b_ids, b_d = ids.clone(), dist.clone()
    Tb, _ = fg.refine(m, fg.params(k=cfg.k, L=cfg.L, rounds=3, flags=fg.FGIM_FLAG_NO_GRAPH_CAPTURE),
                      b_ids, b_d)
    assert torch.equal(a_ids, b_ids) and torch.equal(a_d, b_d) and torch.equal(Ta, Tb)
    for _ in range(2):
        c_ids, c_d = ids.clone(), dist.clone()
        fg.refine(m, fg.params(k=cfg.k, L=cfg.L, rounds=3), c_ids, c_d)
        assert torch.equal(a_ids, c_ids)


@pytest.mark.parametrize("name,sizes", CASES, ids=IDS)
def test_prune_matches_oracle(name, sizes):
    cfg, X, graphs, m, ids, dist = _stage1(name, sizes)
    oi, od, of, oT, _ = oracle.refine(X, graphs, _u32(ids), dist.cpu().numpy(), cfg.rounds,
                                      cfg.metric)
    pi, pd, pdeg = oracle.prune(X, oi, od, oT, cfg.R, cfg.metric)
    dev = torch.device("cuda")
    gids = torch.from_numpy(oi.view(np.int32)).to(dev)
    gd = torch.from_numpy(od).to(dev)
    gT = torch.from_numpy(oT.view(np.int32)).to(dev)
    for R in (cfg.R, 8):
        pi, pd, pdeg = oracle.prune(X, oi, od, oT, R, cfg.metric)
        # the MFMA-screened selection (k <= 64, dim <= 256) and the FP32 one
        for flags in (0, fg.FGIM_FLAG_NO_MFMA_SCREEN):
            pg, deg = fg.prune(m, fg.params(k=cfg.k, L=cfg.L, R=R, flags=flags), gids, gd, gT)
            assert (_u32(pg) == pi).all(), f"R={R} flags={flags}"
            assert (_u32(deg) == pdeg).all()


def test_prune_rejects_list_holes():
    cfg, X, graphs, m, ids, dist = _stage1("cfg1", None)
    T, _ = fg.refine(m, fg.params(k=cfg.k, L=cfg.L, rounds=1), ids, dist)
    bad = ids.clone()
    bad[3, 2] = -1  # a free slot before occupied ones
    with pytest.raises(fg.FgimError) as ei:
        fg.prune(m, fg.params(k=cfg.k, L=cfg.L, R=cfg.R), bad, dist, T)
    assert ei.value.name == "FGIM_ERR_GRAPH"


def test_scratch_arena_reuse_and_release():
    """Calls reuse the library's scratch arena (grown after the first call);
    releasing it, or running on another stream, changes no result."""
    cfg, X, graphs, _ = workload("cfg1", (700, 500))
    m = to_gpu(X, graphs, cfg.metric)
    p = fg.params(k=cfg.k, L=cfg.L, R=cfg.R, rounds=cfg.rounds)
    fg.release_scratch()
    ref, rdeg, rent, _ = fg.merge(m, p)  # spills to the memory pool, then sizes the arena
    for _ in range(2):
        pg, deg, ent, _ = fg.merge(m, p)  # from the arena
        assert torch.equal(pg, ref) and torch.equal(deg, rdeg) and ent == rent
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        pg, deg, ent, _ = fg.merge(m, p)
    side.synchronize()
    assert torch.equal(pg, ref) and ent == rent
    fg.release_scratch()
    pg, _, _, _ = fg.merge(m, p)
    assert torch.equal(pg, ref)


def test_buffer_overflow_reruns_to_the_same_result():
    """Refinement buffers that start too small overflow; the rounds run again
    with larger ones and give the result of a run that never overflowed."""
    cfg, X, graphs, _ = workload("cfg1", None)
    m = to_gpu(X, graphs, cfg.metric)
    p = fg.params(k=cfg.k, L=cfg.L, R=cfg.R, rounds=cfg.rounds)
    ref, rdeg, rent, st0 = fg.merge(m, p, stats=True)
    small = fg.params(k=cfg.k, L=cfg.L, R=cfg.R, rounds=cfg.rounds, flags=fg.FGIM_FLAG_MIN_BUFFERS)
    pg, deg, ent, st = fg.merge(m, small, stats=True)
    print(f"attempts {st['refine_attempts']} (normal {st0['refine_attempts']})", flush=True)
    assert st["refine_attempts"] >= 2
    assert torch.equal(pg, ref) and torch.equal(deg, rdeg) and ent == rent
    assert st["proposals"] == st0["proposals"] and st["rechecked"] == st0["rechecked"]


@pytest.mark.parametrize("name,sizes", [("cfg1", None), ("cfg3", (300, 500, 700, 150, 900, 400, 1200, 650))])
def test_update_chunks_change_no_result(name, sizes):
    """The Update of a synchronous round split into vertex chunks that share
    one pair buffer (every chunk against the same snapshot) gives the
    unsplit result, chunk boundaries included."""
    cfg, X, graphs, m, ids, dist = _stage1(name, sizes)
    oi, od, of, oT, ost = oracle.refine(X, graphs, _u32(ids), dist.cpu().numpy(), cfg.rounds, cfg.metric)
    for chunks in (1, 7, 64):
        print(f"case {name} update_chunks={chunks}", flush=True)
        a_ids, a_d = ids.clone(), dist.clone()
        T, st = fg.refine(m, fg.params(k=cfg.k, L=cfg.L, rounds=cfg.rounds, update_chunks=chunks), a_ids, a_d,
                          stats=True)
        assert (_u32(a_ids) == oi).all()
        assert (a_d.cpu().numpy().view(np.uint32) == od.view(np.uint32)).all()
        assert (_u32(T) == oT).all()
        assert st["proposals"] == ost["proposals"]


def test_refine_rejects_out_of_range_ids():
    cfg, X, graphs, m, ids, dist = _stage1("cfg1", None)
    bad = ids.clone()
    bad[5, 1] = X.shape[0] + 7  # an id past n_total
    keep = bad.clone()
    with pytest.raises(fg.FgimError) as ei:
        fg.refine(m, fg.params(k=cfg.k, L=cfg.L, rounds=1), bad, dist)
    assert ei.value.name == "FGIM_ERR_GRAPH"
    assert torch.equal(bad, keep)  # rejected before any list was changed


@pytest.mark.parametrize("name,sizes", CASES, ids=IDS)
def test_merge_matches_oracle(name, sizes):
    cfg, X, graphs, _ = workload(name, sizes)
    m = to_gpu(X, graphs, cfg.metric)
    p = fg.params(k=cfg.k, L=cfg.L, R=cfg.R, rounds=cfg.rounds)
    pg, deg, entry, st = fg.merge(m, p, stats=True)
    oi, odeg, oent = oracle.merge(X, graphs, cfg.k, cfg.L, cfg.rounds, cfg.R, cfg.metric)
    assert (_u32(pg) == oi).all()
    assert (_u32(deg) == odeg).all()
    assert entry == oent
    assert all(t > 0 for t in st["ms_stage"])
    pg2, _, _, _ = fg.merge(m, p)
    assert torch.equal(pg, pg2)


def test_hand_example_on_gpu():
    # The hand-derived example of Algorithms 2-5 (tests/golden/e2e_tiny.json).
    g = golden("e2e_tiny.json")
    X = line_points(g["points"])
    graphs = [(s["off"], pad_adj(s["adj"]), s["entry"]) for s in g["subs"]]
    m = to_gpu(X, graphs, "l2")
    p = fg.params(k=g["k"], L=g["L"], R=g["R"], rounds=g["rounds"], k_rev=g["k_rev"])
    ids, dist, _ = fg.cross_query(m, p)
    assert _u32(ids).tolist() == g["stage1"]["ids"]
    T, _ = fg.refine(m, p, ids, dist)
    assert _u32(ids).tolist() == g["stage2"]["ids"]
    assert _u32(T).tolist() == g["stage2"]["T"]
    pg, deg = fg.prune(m, p, ids, dist, T)
    assert _u32(pg).tolist() == pad_ids(g["stage3"]["ids"], g["R"]).tolist()
    pg2, deg2, entry, _ = fg.merge(m, p)
    assert torch.equal(pg, pg2) and entry == g["entry"]


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_precision_form_merge_matches_oracle(prec):
    # cfg5's form at test size: 20 uneven sub-indexes, low-precision beam with
    # the FP32 re-rank of 64 per search, then FP32 refinement and prune.  The
    # oracle runs the same stages on its own decoded copy.
    cfg, X, graphs, _ = workload("cfg5", CFG5_SMALL)
    deq = oracle.quantize_bf16(X)[1] if prec == "bf16" else oracle.quantize_fp8(X)[2]
    rerank = min(cfg.L, 2 * cfg.k)
    m = to_gpu(X, graphs, cfg.metric)
    p = fg.params(k=cfg.k, L=cfg.L, R=cfg.R, rounds=cfg.rounds, precision=prec)
    pg, deg, entry, st = fg.merge(m, p, stats=True)
    oi, od, _ = oracle.cross_query(X, graphs, cfg.k, cfg.L, cfg.metric, Xs=deq, rerank=rerank)
    i2, d2, _, T, _ = oracle.refine(X, graphs, oi, od, cfg.rounds, cfg.metric)
    pi, pd, pdeg = oracle.prune(X, i2, d2, T, cfg.R, cfg.metric)
    assert (_u32(pg) == pi).all() and (_u32(deg) == pdeg).all()
    assert entry == oracle.merged_entry(graphs)
    assert st["searches"] == X.shape[0] * (len(graphs) - 1)
