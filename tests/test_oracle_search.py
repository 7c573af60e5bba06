"""Pins of the oracle's Algorithm 1 (KNNSearch, Section 2.1)."""
import numpy as np
import pytest

import oracle
from helpers import golden, line_points, pad_adj, NONE


def _brute(X, q, L):
    d = ((X.astype(np.int64) - q.astype(np.int64)) ** 2).sum(1)
    order = np.lexsort((np.arange(len(X)), d))
    return order[:L], d[order[:L]]


def test_hand_trace(golden_dir):
    g = golden("alg1_trace.json")
    X = line_points(g["points"])
    adj = pad_adj(g["adj"])
    q = line_points([g["query"]])[0]
    for c in g["cases"]:
        ids, dd, ndc, nexp = oracle.knn_search(q, X, adj, g["entry"], c["L"])
        assert ids.tolist() == c["ids"]
        assert dd.tolist() == c["dists"]
        assert ndc == c["ndc"] and nexp == c["expansions"]


@pytest.mark.parametrize("L", [1, 5, 17, 40])
def test_complete_graph_is_exact_top_L(L):
    # Expanding the entry of a complete graph inserts every vertex, so the
    # pool is the exact top-L (integer data: FP32 distances are exact).
    rng = np.random.default_rng(L)
    n = 40
    X = rng.integers(0, 256, (n, 16)).astype(np.float32)
    adj = np.array([[j for j in range(n) if j != i] for i in range(n)], np.uint32)
    q = rng.integers(0, 256, 16).astype(np.float32)
    ids, dd, ndc, nexp = oracle.knn_search(q, X, adj, 3, L)
    bi, bd = _brute(X, q, L)
    assert ids.tolist() == bi.tolist()
    assert dd.tolist() == bd.astype(np.float32).tolist()
    assert ndc == n


def test_large_pool_on_connected_graph_reaches_everything():
    # With L >= n nothing is ever evicted, so the search reaches every vertex
    # reachable from ep; on a strongly connected graph the result is all of V.
    rng = np.random.default_rng(5)
    n = 60
    X = rng.integers(0, 256, (n, 8)).astype(np.float32)
    rows = []
    for i in range(n):
        nb = {(i + 1) % n}
        nb |= set(rng.integers(0, n, 3).tolist()) - {i}
        rows.append(sorted(nb))
    adj = pad_adj(rows, 4)
    q = rng.integers(0, 256, 8).astype(np.float32)
    ids, dd, ndc, _ = oracle.knn_search(q, X, adj, 0, n)
    bi, bd = _brute(X, q, n)
    assert ids.tolist() == bi.tolist()
    assert ndc == n


def test_greedy_on_path_finds_nearest():
    # 1-D sorted points joined as a path: the distance to q is unimodal along
    # the path, so even L=1 walks to the true nearest neighbour.
    xs = np.sort(np.random.default_rng(9).choice(1000, 50, replace=False))
    X = line_points(xs)
    rows = [[j for j in (i - 1, i + 1) if 0 <= j < 50] for i in range(50)]
    adj = pad_adj(rows, 2)
    for qv in (-5, 3, 500, 999, 1200):
        q = line_points([qv])[0]
        ids, _, _, _ = oracle.knn_search(q, X, adj, 25, 1)
        true = int(np.argmin((xs - qv) ** 2))
        assert ids[0] == true


def test_output_sorted_unique_and_ndc_bounded():
    rng = np.random.default_rng(21)
    n = 500
    X = rng.normal(size=(n, 32)).astype(np.float32)
    adj = rng.integers(0, n, (n, 8)).astype(np.uint32)
    adj[adj == np.arange(n)[:, None]] = NONE
    adj[:, 7] = NONE   # padding is skipped
    for L in (4, 16, 64):
        q = rng.normal(size=32).astype(np.float32)
        ids, dd, ndc, nexp = oracle.knn_search(q, X, adj, 0, L)
        assert len(set(ids.tolist())) == len(ids)
        keys = list(zip(dd.tolist(), ids.tolist()))
        assert keys == sorted(keys)
        assert ndc <= n and nexp <= ndc
        for i, v in enumerate(ids):
            assert dd[i] == oracle.distance(q, X[v])


def test_bad_graph_rejected():
    X = line_points([0, 1])
    with pytest.raises(ValueError):
        oracle.knn_search(X[0], X, np.array([[1], [5]], np.uint32), 0, 2)
