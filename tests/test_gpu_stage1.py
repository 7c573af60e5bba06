"""GPU parity of stage 1 (PGs -> k-NNG by cross-querying, Algorithm 2 with
Algorithm 1) and of the batched search against the oracle: ids bit-exact,
FP32 distances within 1e-5 relative."""
import numpy as np
import pytest
import torch

import oracle
from helpers import NONE
from wl import CFG5_SMALL, to_gpu, workload

pytestmark = pytest.mark.gpu

fg = pytest.importorskip("paper_2603_21710_amd")


def _cmp(gi, gd, oi, od, label=""):
    gi = gi.cpu().numpy().view(np.uint32)
    gd = gd.cpu().numpy()
    bad = np.argwhere(gi != oi)
    assert bad.size == 0, f"{label}: {len(bad)} id mismatches, first at {bad[:3].tolist()}"
    fin = np.isfinite(od)
    assert (np.isfinite(gd) == fin).all()
    assert np.allclose(gd[fin], od[fin], rtol=1e-5, atol=0), label
    return bool((gd.view(np.uint32) == od.view(np.uint32)).all())


CASES = [
    ("cfg1", None),
    ("cfg1ov", None),
    ("cfg2", (2500, 2000)),
    ("cfg3", (300, 500, 700, 150, 900, 400, 1200, 650)),
    ("cfg4", (1200, 1000)),
    ("cfg5", CFG5_SMALL),
]


@pytest.mark.parametrize("name,sizes", CASES, ids=[c[0] for c in CASES])
def test_cross_query_matches_oracle(name, sizes):
    cfg, X, graphs, _ = workload(name, sizes)
    print(f"case {name} N={X.shape[0]} d={X.shape[1]} h={len(graphs)}", flush=True)
    m = to_gpu(X, graphs, cfg.metric)
    ids, dist, st = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L), stats=True)
    oi, od, ost = oracle.cross_query(X, graphs, cfg.k, cfg.L, cfg.metric)
    bitwise = _cmp(ids, dist, oi, od, name)
    assert bitwise, "FP32 distances are expected to be bit-identical"
    assert st["expansions"] == ost["expansions"]
    assert st["ndc"] >= ost["ndc"]
    assert st["searches"] == X.shape[0] * (len(graphs) - 1)


def test_launch_shape_does_not_change_bits():
    cfg, X, graphs, _ = workload("cfg2", (2500, 2000))
    m = to_gpu(X, graphs, cfg.metric)
    ref, refd, _ = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L))
    for P, waves, slots in [(4, 1, 64), (8, 4, 256), (16, 16, 4096), (32, 8, 1024), (8, 32, 16384)]:
        ids, dist, st = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L, lanes_per_dist=P,
                                                    waves_per_cu=waves, visited_slots=slots),
                                       stats=True)
        assert torch.equal(ids, ref) and torch.equal(dist.view(torch.int32), refd.view(torch.int32)), (P, waves, slots)
    for _ in range(3):
        ids, dist, _ = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L))
        assert torch.equal(ids, ref)


def _random_graphs(X, sizes, degree, seed):
    """Sub-indexes whose rows hold `degree` random distinct other local ids."""
    rng = np.random.default_rng(seed)
    graphs, off = [], 0
    for n in sizes:
        adj = np.full((n, 24), NONE, np.uint32)
        for u in range(n):
            adj[u, :degree] = rng.choice(np.delete(np.arange(n), u), degree, replace=False)
        graphs.append((off, adj, 0))
        off += n
    return graphs


@pytest.mark.parametrize("degree,P,slots", [(6, 16, 1024), (20, 8, 2048)])
def test_sparse_graphs_take_the_two_chunk_shape(degree, P, slots):
    # d = 128: the default shape has four chunks per lane (P = 8) and, at
    # L = 64, 2048 visited slots; graphs of mean out-degree <= 12 take two
    # chunks per lane and 1024 slots.  Either way the result is the oracle's.
    cfg, X, _, _ = workload("cfg2", (1500, 1200))
    graphs = _random_graphs(X, (1500, 1200), degree, 40 + degree)
    m = to_gpu(X, graphs, cfg.metric)
    ids, dist, st = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L), stats=True)
    assert (st["lanes_per_dist"], st["visited_slots"]) == (P, slots)
    oi, od, _ = oracle.cross_query(X, graphs, cfg.k, cfg.L, cfg.metric)
    assert _cmp(ids, dist, oi, od, f"degree {degree}")


@pytest.mark.parametrize("k,L", [(16, 1), (16, 5), (100, 64), (24, 128), (32, 200), (128, 256)])
def test_pool_and_topk_sizes(k, L):
    cfg, X, graphs, _ = workload("cfg3", (300, 500, 700, 150, 900, 400, 1200, 650))
    m = to_gpu(X, graphs, cfg.metric)
    ids, dist, _ = fg.cross_query(m, fg.params(k=k, L=L))
    oi, od, _ = oracle.cross_query(X, graphs, k, L, cfg.metric)
    _cmp(ids, dist, oi, od, f"k={k} L={L}")


def test_degenerate_inputs():
    # single sub-index (no cross-queries), tiny sub-indexes, L larger than a
    # graph, k larger than every candidate set (padding), wide adjacency rows.
    rng = np.random.default_rng(0)
    X = rng.normal(size=(300, 32)).astype(np.float32)
    def adj_of(n, stride, deg):
        a = np.full((n, stride), NONE, np.uint32)
        for u in range(n):
            nb = [v for v in rng.permutation(n)[:deg + 1] if v != u][:deg]
            a[u, :len(nb)] = nb
        return a
    cases = [
        [(0, adj_of(300, 16, 10), 5)],
        [(0, adj_of(1, 4, 0), 0), (1, adj_of(2, 4, 1), 1), (3, adj_of(297, 100, 70), 7)],
        [(0, adj_of(150, 8, 3), 0), (150, adj_of(150, 8, 3), 149)],
    ]
    for graphs in cases:
        m = to_gpu(X, graphs, "l2")
        for k, L in [(8, 4), (64, 200), (120, 3)]:
            ids, dist, _ = fg.cross_query(m, fg.params(k=k, L=L))
            oi, od, _ = oracle.cross_query(X, graphs, k, L, "l2")
            _cmp(ids, dist, oi, od, f"k={k} L={L} h={len(graphs)}")


def test_malformed_graph_is_rejected():
    cfg, X, graphs, _ = workload("cfg1", (200, 200))
    for mutate in ("range", "self", "dup"):
        g = [(o, a.copy(), e) for o, a, e in graphs]
        a = g[1][1]
        if mutate == "range":
            a[5, 0] = 200
        elif mutate == "self":
            a[7, 0] = 7
        else:
            a[9, 1] = a[9, 0]
        m = to_gpu(X, g, cfg.metric)
        with pytest.raises(fg.FgimError) as ei:
            fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L))
        assert ei.value.name == "FGIM_ERR_GRAPH"


@pytest.mark.parametrize("name,sizes", [("cfg1ov", None), ("cfg3", (300, 500, 700, 150, 900, 400, 1200, 650))])
def test_search_matches_oracle(name, sizes):
    cfg, X, graphs, Q = workload(name, sizes)
    off, adj, entry = graphs[-1]
    Xs = X[off:off + adj.shape[0]]
    dev = torch.device("cuda")
    for L, topk in [(16, 10), (64, 10), (100, 100)]:
        ids, dist = fg.search(torch.from_numpy(Xs).to(dev), torch.from_numpy(adj.view(np.int32)).to(dev),
                              entry, torch.from_numpy(Q).to(dev), L, topk, cfg.metric)
        gi = ids.cpu().numpy().view(np.uint32)
        gd = dist.cpu().numpy()
        for q in range(0, Q.shape[0], 7):
            oi, od, _, _ = oracle.knn_search(Q[q], Xs, adj, entry, L, cfg.metric)
            n = min(topk, len(oi))
            assert gi[q, :n].tolist() == oi[:n].tolist()
            assert (gd[q, :n] == od[:n]).all()
            assert (gi[q, n:] == NONE).all()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_quantize_matches_oracle(prec):
    rng = np.random.default_rng(1)
    X = np.concatenate([rng.normal(size=(500, 96)) * 10.0 ** rng.integers(-3, 3, (500, 1)),
                        np.zeros((1, 96)), rng.uniform(-1, 1, (3, 96)) * 1e-30]).astype(np.float32)
    codes, scales = fg.quantize(torch.from_numpy(X).cuda(), prec)
    if prec == "bf16":
        oc, od = oracle.quantize_bf16(X)
        assert (codes.cpu().numpy().view(np.uint16) == oc).all()
    else:
        oc, osc, od = oracle.quantize_fp8(X)
        assert (scales.cpu().numpy() == osc).all()
        assert (codes.cpu().numpy() == oc).all()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("name,sizes", [("cfg4", (1200, 1000)), ("cfg2", (2500, 2000)),
                                        ("cfg3", (300, 500, 700, 150, 900, 400, 1200, 650)),
                                        ("cfg5", CFG5_SMALL)])
def test_precision_form_stage1_matches_oracle(prec, name, sizes):
    # The low-precision beam scores the FP32 query against decoded rows
    # (BF16 exactly, FP8 as scale * decode in one FP32 rounding) in the
    # canonical order, so the oracle reproduces it by searching the decoded
    # copy and re-scoring each search's first `rerank` results on FP32 rows.
    cfg, X, graphs, _ = workload(name, sizes)
    if prec == "bf16":
        _, deq = oracle.quantize_bf16(X)
    else:
        _, _, deq = oracle.quantize_fp8(X)
    rerank = min(cfg.L, 2 * cfg.k)
    m = to_gpu(X, graphs, cfg.metric)
    ids, dist, _ = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L, precision=prec))
    oi, od, _ = oracle.cross_query(X, graphs, cfg.k, cfg.L, cfg.metric, Xs=deq, rerank=rerank)
    _cmp(ids, dist, oi, od, f"{name} {prec}")
    # the same with a caller-provided copy from fgim_quantize
    codes, scales = fg.quantize(m.X, prec)
    m2 = to_gpu(X, graphs, cfg.metric, codes, scales)
    ids2, dist2, _ = fg.cross_query(m2, fg.params(k=cfg.k, L=cfg.L, precision=prec))
    assert torch.equal(ids, ids2) and torch.equal(dist, dist2)
