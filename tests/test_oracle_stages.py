"""Pins of the oracle's three stages (Algorithms 2-5) against hand-derived
examples, special cases with exact answers and invariants the paper states."""
import numpy as np
import pytest

import oracle
from helpers import NONE, golden, line_points, pad_adj, pad_dists, pad_ids
from workloads import build_input_pg, get_config, make_queries, make_vectors, split_sizes


def _tiny():
    g = golden("e2e_tiny.json")
    X = line_points(g["points"])
    subs = [(s["off"], pad_adj(s["adj"]), s["entry"]) for s in g["subs"]]
    return g, X, subs


def test_e2e_hand_example_stage1():
    g, X, subs = _tiny()
    ids, dd, _ = oracle.cross_query(X, subs, g["k"], g["L"])
    assert ids.tolist() == g["stage1"]["ids"]
    assert dd.tolist() == g["stage1"]["dists"]


@pytest.mark.parametrize("stage,rounds", [("round1", 1), ("stage2", 2)])
def test_e2e_hand_example_refine(stage, rounds):
    g, X, subs = _tiny()
    ids, dd, _ = oracle.cross_query(X, subs, g["k"], g["L"])
    i2, d2, f2, T, st = oracle.refine(X, subs, ids, dd, rounds, k_rev=g["k_rev"])
    exp = g[stage]
    assert i2.tolist() == exp["ids"]
    assert d2.tolist() == exp["dists"]
    assert f2.tolist() == exp["flags"]
    assert T.tolist() == exp["T"]
    if "repaired" in exp:
        assert st["repaired"] == exp["repaired"]


def test_e2e_hand_example_prune_and_merge():
    g, X, subs = _tiny()
    s2 = g["stage2"]
    oi, od, deg = oracle.prune(X, np.array(s2["ids"], np.uint32),
                               np.array(s2["dists"], np.float32),
                               np.array(s2["T"], np.uint32), g["R"])
    assert oi.tolist() == pad_ids(g["stage3"]["ids"], g["R"]).tolist()
    assert deg.tolist() == g["stage3"]["deg"]
    mi, mdeg, ent = oracle.merge(X, subs, g["k"], g["L"], g["rounds"], g["R"],
                                 k_rev=g["k_rev"])
    assert mi.tolist() == oi.tolist() and ent == g["entry"]


@pytest.mark.parametrize("case", golden("repair_cases.json")["cases"], ids=lambda c: c["name"])
def test_repair_hand_examples(case):
    k = case["k"]
    ids = pad_ids(case["ids"], k)
    dd = pad_dists(case["dists"], k)
    flags = np.zeros_like(ids, dtype=np.uint8)
    oi, od, of, T, nr = oracle.repair(ids, dd, flags)
    assert oi.tolist() == pad_ids(case["out_ids"], k).tolist()
    assert od.tolist() == pad_dists(case["out_dists"], k).tolist()
    assert (of & 1).tolist() == case["out_new"]
    assert T.tolist() == case["T"]
    assert nr == case["repaired"]


def _rand_lists(rng, N, k, fill=1.0):
    ids = np.full((N, k), NONE, np.uint32)
    dd = np.full((N, k), np.inf, np.float32)
    for u in range(N):
        m = k if rng.random() < fill else int(rng.integers(1, k + 1))
        cand = rng.choice(np.setdiff1d(np.arange(N), [u]), m, replace=False)
        d = rng.integers(1, 50, m).astype(np.float32)
        order = np.lexsort((cand, d))
        ids[u, :m] = cand[order]
        dd[u, :m] = d[order]
    return ids, dd


@pytest.mark.parametrize("seed", range(6))
def test_repair_invariants(seed):
    # The outdegree bound is kept and full lists keep their degree (Section
    # 4.2.2; a list with a free slot may take v*), T equals a recount, the number of
    # zero-indegree vertices never grows, a repaired vertex gains exactly one
    # in-edge and no vertex that had in-edges loses its last one.
    rng = np.random.default_rng(seed)
    N, k = 300, 4
    ids, dd = _rand_lists(rng, N, k, fill=0.8 if seed % 2 else 1.0)
    T0 = np.bincount(ids[ids != NONE].astype(np.int64), minlength=N)
    oi, od, of, T, nr = oracle.repair(ids, dd)
    deg0 = (ids != NONE).sum(1)
    deg1 = (oi != NONE).sum(1)
    assert (deg1 <= k).all() and (deg1 >= deg0).all()
    assert (deg1[deg0 == k] == k).all()
    assert (deg1 - deg0).sum() <= nr
    recount = np.bincount(oi[oi != NONE].astype(np.int64), minlength=N)
    assert (recount == T).all()
    assert (T == 0).sum() <= (T0 == 0).sum()
    assert nr == (T0 == 0).sum() - (T == 0).sum()
    assert (T[T0 == 0] <= 1).all()
    assert (T[T0 > 0] >= 1).all()
    for u in range(N):
        row = [(od[u, t], oi[u, t]) for t in range(k) if oi[u, t] != NONE]
        assert row == sorted(row) and len({v for _, v in row}) == len(row)


def test_min_L_closed_form():
    # L >= ceil((k - min |C+|) / (h - 1)) (Section 4.1.2); worst case ceil(k/(h-1)).
    assert oracle.min_L(16, 0, 2) == 16
    assert oracle.min_L(24, 3, 8) == 3
    assert oracle.min_L(32, 10, 5) == 6
    assert oracle.min_L(32, 0, 20) == 2
    assert oracle.min_L(8, 9, 3) == 1


def _complete_subs(sizes):
    subs, off = [], 0
    for n in sizes:
        adj = np.array([[j for j in range(n) if j != i] for i in range(n)], np.uint32)
        subs.append((off, adj, 0))
        off += n
    return subs


@pytest.mark.parametrize("sizes,k,L", [((20, 30), 8, 8), ((15, 25, 10), 12, 20),
                                       ((30, 30), 16, 40)])
def test_stage1_complete_graphs_give_exact_knng(sizes, k, L):
    # With complete input graphs every search returns the exact top-L of its
    # graph and C+ is the whole own sub-index, so top-k of the union is the
    # exact k-NN (integer data: FP32 distances are exact, ties by id).
    rng = np.random.default_rng(sum(sizes))
    X = rng.integers(0, 256, (sum(sizes), 16)).astype(np.float32)
    ids, dd, _ = oracle.cross_query(X, _complete_subs(sizes), k, L)
    gi, gd = oracle.bruteforce(X, X, k, exclude=np.arange(sum(sizes)))
    assert ids.tolist() == gi.tolist()
    assert dd.astype(np.float64).tolist() == gd.tolist()


def _cfg_small(name="cfg1ov", sizes=(1500, 1500)):
    cfg = get_config(name).scaled(sizes)
    X = make_vectors(cfg)
    subs = []
    for off, n in split_sizes(cfg):
        pg = build_input_pg(X[off:off + n], cfg.r_in, cfg.metric)
        subs.append((off, pg.adj, pg.entry))
    return cfg, X, subs


def test_stage1_candidate_sources_and_sampling():
    cfg, X, subs = _cfg_small(sizes=(700, 500, 300))
    ids, dd, st = oracle.cross_query(X, subs, cfg.k, cfg.L, cfg.metric, threads=1)
    ids8, dd8, st8 = oracle.cross_query(X, subs, cfg.k, cfg.L, cfg.metric, threads=8)
    assert (ids == ids8).all() and (dd == dd8).all() and st == st8
    nodes = np.array([5, 699, 700, 1499, 1000], np.uint64)
    si, sd, _ = oracle.cross_query(X, subs, cfg.k, cfg.L, cfg.metric, nodes=nodes)
    assert (si == ids[nodes.astype(np.int64)]).all()
    offs = [s[0] for s in subs]
    for u in range(X.shape[0]):
        g = np.searchsorted(offs, u, side="right") - 1
        own = {offs[g] + int(v) for v in subs[g][1][u - offs[g]] if v != NONE}
        for v in ids[u]:
            if v == NONE:
                continue
            gv = np.searchsorted(offs, v, side="right") - 1
            assert gv != g or int(v) in own
            assert v != u


def test_stage1_single_subindex_is_sorted_local_list():
    cfg, X, subs = _cfg_small(sizes=(800,))
    ids, dd, _ = oracle.cross_query(X, subs, cfg.k, cfg.L, cfg.metric)
    adj = subs[0][1]
    for u in range(0, 800, 37):
        loc = [int(v) for v in adj[u] if v != NONE]
        keys = sorted((oracle.distance(X[u], X[v]), v) for v in loc)[:cfg.k]
        assert [v for _, v in keys] == [int(v) for v in ids[u] if v != NONE]


def test_stage1_rerank_with_identical_copy_matches_fp32():
    cfg, X, subs = _cfg_small(sizes=(600, 600))
    a, ad, _ = oracle.cross_query(X, subs, cfg.k, cfg.L, cfg.metric)
    b, bd, _ = oracle.cross_query(X, subs, cfg.k, cfg.L, cfg.metric, Xs=X.copy(),
                                  rerank=cfg.k)
    assert (a == b).all() and (ad == bd).all()


def _stage1_from_parts(X, Xs, subs, u, k, L, keep, metric, score_on):
    """Stage 1 of vertex u rebuilt from its parts: C+(u) scored on X, plus the
    first `keep` results of Algorithm 1 (oracle.knn_search, pinned by the
    hand trace) run on the copy Xs in every other sub-index, each re-scored
    on `score_on`; sorted by (delta, id) and cut to k."""
    offs = [s[0] for s in subs]
    g = int(np.searchsorted(offs, u, side="right") - 1)
    off, adj, _ = subs[g]
    cand = [(oracle.distance(X[u], X[off + int(v)], metric), off + int(v))
            for v in adj[u - off] if v != NONE]
    for j, (offj, adjj, ej) in enumerate(subs):
        if j == g:
            continue
        n = adjj.shape[0]
        ids, _, _, _ = oracle.knn_search(X[u], Xs[offj:offj + n], adjj, ej, L, metric)
        for v in ids[:keep]:
            gv = offj + int(v)
            cand.append((oracle.distance(X[u], score_on[gv], metric), gv))
    cand.sort()
    return cand[:k]


@pytest.mark.parametrize("metric,k,L,rerank", [("l2", 16, 32, 8), ("l2", 16, 32, 20),
                                               ("ip", 12, 24, 12)])
def test_stage1_rerank_branch_with_a_distinct_copy(metric, k, L, rerank):
    # The low-precision form: the beam scores a copy Xs that differs from X,
    # each search keeps its first `rerank` results, and those are re-scored
    # on the FP32 rows before the union (rerank < L; the first case also has
    # rerank < k).  Xs = X + noise comparable to the spread of a cluster, so
    # that the copy's search order differs from X's.
    name = "cfg1ov" if metric == "l2" else "cfg3ov"
    cfg, X, subs = _cfg_small(name, sizes=(500, 400, 300))
    rng = np.random.default_rng(31)
    scale = 0.5 if metric == "l2" else 0.05
    Xs = (X + rng.normal(0, scale, X.shape)).astype(np.float32)
    nodes = np.arange(0, X.shape[0], 23, dtype=np.uint64)
    ids, dd, _ = oracle.cross_query(X, subs, k, L, metric, nodes=nodes, Xs=Xs, rerank=rerank)
    wrong_count = wrong_rows = 0
    for r, u in enumerate(nodes.astype(np.int64)):
        want = _stage1_from_parts(X, Xs, subs, u, k, L, rerank, metric, X)
        got = [(float(dd[r, t]), int(ids[r, t])) for t in range(k) if ids[r, t] != NONE]
        assert got == want, f"vertex {u}"
        # every distance is the FP32 distance of its id on the FP32 rows
        for d, v in got:
            assert d == oracle.distance(X[u], X[v], metric)
        # the two plausible mistakes give other lists on this input
        wrong_count += _stage1_from_parts(X, Xs, subs, u, k, L, L, metric, X) != want
        wrong_rows += _stage1_from_parts(X, Xs, subs, u, k, L, rerank, metric, Xs) != want
    assert wrong_count > 0 and wrong_rows > 0


def test_merged_entry_on_unequal_subindexes():
    # The merged entry is the entry of the largest sub-index, the lowest
    # index among equal sizes, as a global id.
    def subs(sizes, entries):
        out, off = [], 0
        for n, e in zip(sizes, entries):
            out.append((off, np.zeros((n, 1), np.uint32), e))
            off += n
        return out
    assert oracle.merged_entry(subs((300, 700, 700, 200), (5, 11, 17, 3))) == 311
    assert oracle.merged_entry(subs((100, 50, 400), (1, 2, 7))) == 157
    assert oracle.merged_entry(subs((90, 40), (89, 0))) == 89
    assert oracle.merged_entry(subs((40, 90), (0, 89))) == 129


def test_join_keeps_exact_knng():
    # An exact k-NNG is a fixed point of Update: no pair can beat an entry of
    # a true k-NN list (repair off, so only the join acts).
    rng = np.random.default_rng(4)
    X = rng.integers(0, 256, (400, 8)).astype(np.float32)
    subs = [(0, np.zeros((200, 1), np.uint32), 0), (200, np.zeros((200, 1), np.uint32), 0)]
    gi, gd = oracle.bruteforce(X, X, 10, exclude=np.arange(400))
    i2, d2, f2, T, st = oracle.refine(X, subs, gi, gd.astype(np.float32), 3,
                                      do_repair=False)
    assert (i2 == gi).all() and (d2 == gd.astype(np.float32)).all()


def test_join_needs_two_subindexes():
    # Pairs must come from different sub-indexes (Algorithm 3): with h = 1 no
    # pair qualifies and the lists are unchanged.
    cfg, X, subs = _cfg_small(sizes=(900,))
    ids, dd, _ = oracle.cross_query(X, subs, cfg.k, cfg.L, cfg.metric)
    i2, d2, f2, T, st = oracle.refine(X, subs, ids, dd, 2, cfg.metric, do_repair=False)
    assert st["proposals"] == 0 and (i2 == ids).all() and (f2 == 0).all()


def test_join_keys_monotone_and_recall_up():
    cfg, X, subs = _cfg_small()
    ids, dd, _ = oracle.cross_query(X, subs, cfg.k, cfg.L, cfg.metric)
    i1, d1, _, _, _ = oracle.refine(X, subs, ids, dd, 1, cfg.metric, do_repair=False)
    assert (d1 <= dd).all()
    for u in range(X.shape[0]):
        row = list(zip(d1[u].tolist(), i1[u].tolist()))
        assert row == sorted(row)
        assert len(set(i1[u].tolist())) == len(row)
    nodes = np.arange(0, X.shape[0], 7)
    r0 = oracle.knng_recall(X, ids[nodes], nodes, cfg.k)
    i2, d2, _, T, _ = oracle.refine(X, subs, ids, dd, cfg.rounds, cfg.metric)
    r2 = oracle.knng_recall(X, i2[nodes], nodes, cfg.k)
    assert r2 >= r0
    recount = np.bincount(i2[i2 != NONE].astype(np.int64), minlength=X.shape[0])
    assert (recount == T).all()


def _path_knng(n, k):
    X = line_points(np.arange(n) * 3)
    gi, gd = oracle.bruteforce(X, X, k, exclude=np.arange(n))
    return X, gi, gd.astype(np.float32)


def test_prune_on_line_gives_path():
    # Equally spaced points on a line: u's nearer neighbour on either side
    # occludes every farther point on that side, so the RNG selection over
    # the exact k-NNG is the path graph, which reverse filling keeps.
    n, k = 30, 6
    X, gi, gd = _path_knng(n, k)
    T = np.full(n, 2, np.uint32)
    oi, od, deg = oracle.prune(X, gi, gd, T, 8)
    for u in range(n):
        want = [v for v in (u - 1, u + 1) if 0 <= v < n]
        assert [int(v) for v in oi[u] if v != NONE] == want


def test_prune_keeps_only_in_edge():
    # A neighbour with T = 1 is kept even when occluded (Algorithm 5).
    n, k = 30, 6
    X, gi, gd = _path_knng(n, k)
    T = np.full(n, 2, np.uint32)
    T[14] = 1
    oi, od, deg = oracle.prune(X, gi, gd, T, 8)
    # 14 is in the 6-NN lists of 11 and 12, occluded there by 13.
    assert 14 in oi[11].tolist() and 14 in oi[12].tolist()
    T[14] = 2
    oi2, _, _ = oracle.prune(X, gi, gd, T, 8)
    assert 14 not in oi2[11].tolist() and 14 not in oi2[12].tolist()


def test_prune_degree_bound_and_rule():
    cfg, X, subs = _cfg_small()
    ids, dd, _ = oracle.cross_query(X, subs, cfg.k, cfg.L, cfg.metric)
    i2, d2, _, T, _ = oracle.refine(X, subs, ids, dd, cfg.rounds, cfg.metric)
    for R in (4, 16):
        oi, od, deg = oracle.prune(X, i2, d2, T, R, cfg.metric)
        assert (deg <= R).all()
        assert ((oi != NONE).sum(1) == deg).all()
        for u in range(0, X.shape[0], 11):
            row = [(od[u, t], oi[u, t]) for t in range(deg[u])]
            assert row == sorted(row) and u not in oi[u].tolist()


def test_merge_end_to_end_quality():
    cfg, X, subs = _cfg_small()
    pg, deg, ent = oracle.merge(X, subs, cfg.k, cfg.L, cfg.rounds, cfg.R, cfg.metric)
    N = X.shape[0]
    assert (deg <= cfg.R).all() and (deg >= 1).all()
    for u in range(N):
        row = pg[u, :deg[u]]
        assert u not in row.tolist() and len(set(row.tolist())) == deg[u]
    from workloads import reach_fraction
    assert reach_fraction(pg, ent) >= 0.99
    Q = make_queries(cfg, 100)
    assert oracle.search_recall(X, pg, ent, Q, 64, cfg.metric) >= 0.9


def test_evaluation_ground_truth_matches_oracle():
    # The benchmark's FP64 ground truth (torch, Gram form) agrees with the
    # oracle's direct FP64 brute force, and tie-aware recall of the truth is 1.
    from workloads.evaluate import exact_knn_fp64, tie_recall
    rng = np.random.default_rng(8)
    X = rng.integers(0, 256, (3000, 32)).astype(np.float32)
    Q = rng.integers(0, 256, (50, 32)).astype(np.float32)
    for metric in ("l2", "ip"):
        gi, gd = exact_knn_fp64(X, Q, 10, metric)
        oi, od = oracle.bruteforce(X, Q, 10, metric)
        assert np.array_equal(gd, od)
        assert tie_recall(X, Q, oi, od[:, -1], 10, metric) == 1.0
        assert tie_recall(X, Q, gi.astype(np.uint32), od[:, -1], 10, metric) == 1.0
    wrong = np.full((50, 10), 0xFFFFFFFF, np.uint32)
    assert tie_recall(X, Q, wrong, od[:, -1], 10, "ip") == 0.0


@pytest.mark.parametrize("metric", ["l2", "ip", "cos"])
def test_recall_of_the_exact_answer_is_one_on_float_data(metric):
    # On float data the Gram form (|q|^2 + |x|^2 - 2<q,x>) and the direct
    # form of a distance differ in the last bits.  The ground truth is
    # re-ranked by the direct form that scores returned ids, so the exact
    # answer -- the oracle's FP64 brute force, an independent loop -- scores
    # exactly 1.0 and the truth's ids are the oracle's.
    from workloads.evaluate import exact_knn_fp64, tie_recall
    rng = np.random.default_rng(11)
    X = rng.normal(size=(4000, 96)).astype(np.float32)
    Q = rng.normal(size=(300, 96)).astype(np.float32)
    if metric == "cos":
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    gi, gd = exact_knn_fp64(X, Q, 10, metric)
    oi, od = oracle.bruteforce(X, Q, 10, metric)
    assert (gi == oi.astype(np.int64)).all()
    assert np.allclose(gd, od, rtol=1e-12, atol=1e-12)
    assert tie_recall(X, Q, oi, gd[:, -1], 10, metric) == 1.0
    assert tie_recall(X, Q, gi.astype(np.uint32), gd[:, -1], 10, metric) == 1.0
    # one wrong id per query costs exactly 1/10
    worse = oi.copy()
    worse[:, 0] = oracle.bruteforce(X, Q, 40, metric)[0][:, 39]
    assert tie_recall(X, Q, worse, gd[:, -1], 10, metric) == pytest.approx(0.9)
    # the k-NNG form (each point's own id excluded)
    nodes = np.arange(0, 4000, 50)
    ki, kd = exact_knn_fp64(X, X[nodes], 10, metric, exclude=nodes)
    bi, bd = oracle.bruteforce(X, X[nodes], 10, metric, exclude=nodes)
    assert (ki == bi.astype(np.int64)).all()
    assert tie_recall(X, X[nodes], bi, kd[:, -1], 10, metric) == 1.0


def test_prune_rows_equals_full_prune_on_its_rows():
    # Algorithm 5 for a sample of vertices (selection of u and of every
    # vertex whose list holds u, then the reverse fill of u) equals the
    # rows of the full prune, including vertices that only reverse edges
    # fill and the degree bound R < k.
    cfg, X, subs = _cfg_small()
    ids, dd, _ = oracle.cross_query(X, subs, cfg.k, cfg.L, cfg.metric)
    i2, d2, _, T, _ = oracle.refine(X, subs, ids, dd, cfg.rounds, cfg.metric)
    rows = np.array([0, 1, 17, 1499, 1500, 2999, 2000, 2001, 777], np.uint64)
    for R in (cfg.R, 8):
        fi, fd, fdeg = oracle.prune(X, i2, d2, T, R, cfg.metric)
        ri, rd, rdeg = oracle.prune_rows(X, i2, d2, T, R, rows, cfg.metric)
        r = rows.astype(np.int64)
        assert (ri == fi[r]).all() and (rdeg == fdeg[r]).all()
        assert (rd.view(np.uint32) == fd[r].view(np.uint32)).all()


@pytest.mark.parametrize("metric", ["l2", "ip", "cos"])
def test_screened_ground_truth_equals_oracle_bruteforce(metric):
    # The FP32-screened ground truth (shortlist proved complete by the FP32
    # error bound, else widened, else a direct FP64 pass) returns the
    # oracle's FP64 brute-force answer; a shortlist of one row forces both
    # fallbacks and still gives the same answer.
    import torch
    from workloads.evaluate import exact_knn_screened
    rng = np.random.default_rng(12)
    X = rng.normal(size=(3000, 64)).astype(np.float32)
    Q = rng.normal(size=(200, 64)).astype(np.float32)
    if metric != "l2":
        X /= np.linalg.norm(X, axis=1, keepdims=True)
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    oi, od = oracle.bruteforce(X, Q, 10, metric)
    for margin, widen in ((48, 16), (-9, 1)):
        gi, gd, fb = exact_knn_screened(X, Q, 10, metric, Xdev=torch.from_numpy(X), margin=margin,
                                        widen=widen, block=64)
        assert (gi == oi.astype(np.int64)).all(), margin
        assert np.allclose(gd, od, rtol=1e-12, atol=1e-12)
        if margin < 0:
            assert fb["longer_shortlist"] == 200 and fb["direct_pass"] == 200
    nodes = np.arange(0, 3000, 40)
    gi, gd, _ = exact_knn_screened(X, X[nodes], 10, metric, exclude=nodes, Xdev=torch.from_numpy(X))
    bi, bd = oracle.bruteforce(X, X[nodes], 10, metric, exclude=nodes)
    assert (gi == bi.astype(np.int64)).all()


def _line_knng(n, k, spacing=3):
    X = line_points(np.arange(n) * spacing)
    gi, gd = oracle.bruteforce(X, X, k, exclude=np.arange(n))
    return X, gi, gd.astype(np.float32)


def _sel_offsets(oi, u, spacing=3):
    return sorted(int(v) - u for v in oi[u] if v != NONE)


def test_alpha_rng_on_a_line():
    # Points 3i on a line, exact 16-NN (8 per side inside), T = 2 so the T = 1
    # exemption never applies.  alpha-RNG keeps v at j hops past a kept w at
    # 1 hop on the same side when |u - v| < alpha |w - v|: 3j < 1.25 * 3(j - 1)
    # holds first for j = 6 (j = 5 is the tie 15 = 15, which strict < drops);
    # after that the next survivor would need j > 30.  A neighbour on the other
    # side is always farther from v than u is.  alpha = 1.25 is exact in
    # binary, so the hand result is exact.  The selection stops at R = 8, the
    # reverse fill adds the mirror edges.
    n, k = 40, 16
    X, gi, gd = _line_knng(n, k)
    T = np.full(n, 2, np.uint32)
    sel, _, _ = oracle.prune(X, gi, gd, T, 8, rule="alpha", param=1.25)
    assert _sel_offsets(sel, 20) == [-6, -1, 1, 6]
    assert _sel_offsets(sel, 0) == [1, 6]
    # alpha = 1 is Algorithm 5's rule exactly (alpha^2 * delta = delta)
    a1, _, _ = oracle.prune(X, gi, gd, T, 8, rule="alpha", param=1.0)
    r1, _, _ = oracle.prune(X, gi, gd, T, 8)
    assert (a1 == r1).all() and _sel_offsets(r1, 20) == [-1, 1]


def test_tau_mng_on_a_line():
    # tau-MNG: w occludes v when |w - v| < |u - v| - 3 tau.  On the same line
    # v at j hops survives the kept w at i hops iff 3j < 3(j - i) + 3 tau, i.e.
    # i < tau.  tau = 1: only the first hop per side (the path graph, like
    # RNG); tau = 1.5: hops 1 and 2 survive hop 1, hop 3 is occluded by hop 2,
    # and so is every later one.  Distances are perfect squares, so every
    # square root is exact.
    n, k = 40, 16
    X, gi, gd = _line_knng(n, k)
    T = np.full(n, 2, np.uint32)
    t1, _, _ = oracle.prune(X, gi, gd, T, 8, rule="tau", param=1.0)
    assert _sel_offsets(t1, 20) == [-1, 1]
    t15, _, _ = oracle.prune(X, gi, gd, T, 8, rule="tau", param=1.5)
    assert _sel_offsets(t15, 20) == [-2, -1, 1, 2]
    # a tau larger than every distance occludes nothing: the first R of the
    # list, then the reverse fill truncated to R
    big, _, _ = oracle.prune(X, gi, gd, T, 16, rule="tau", param=1000.0)
    assert sorted(big[20].tolist()) == sorted(gi[20].tolist())


def test_selection_rules_keep_the_only_in_edge_and_reject_inner_product():
    n, k = 30, 6
    X, gi, gd = _line_knng(n, k)
    T = np.full(n, 2, np.uint32)
    T[14] = 1   # 14 is occluded in the lists of 11 and 12 under every rule here
    for rule, param in (("alpha", 1.2), ("tau", 0.5)):
        oi, _, _ = oracle.prune(X, gi, gd, T, 8, rule=rule, param=param)
        assert 14 in oi[11].tolist() and 14 in oi[12].tolist()
    with pytest.raises(ValueError):
        oracle.prune(X, gi, gd, T, 8, metric="ip", rule="alpha", param=1.2)
    with pytest.raises(ValueError):
        oracle.prune(X, gi, gd, T, 8, rule="alpha", param=0.9)


def test_mips_to_l2_transform():
    # x' = (x, sqrt(M - |x|^2)): every row has squared length M (up to FP32
    # rounding of the extra coordinate), the longest row gets 0, and with
    # q' = (q, 0) squared L2 equals |q|^2 + M - 2<q, x>, so the exact L2 k-NN
    # on the transformed rows are the exact inner-product k-NN.
    rng = np.random.default_rng(21)
    X = (rng.normal(size=(3000, 32)) * rng.uniform(0.2, 3.0, (3000, 1))).astype(np.float32)
    Q = rng.normal(size=(100, 32)).astype(np.float32)
    Xt, M = oracle.mips_to_l2(X)
    assert Xt.shape == (3000, 36) and (Xt[:, 33:] == 0).all() and (Xt[:, :32] == X).all()
    n2 = (X.astype(np.float64) ** 2).sum(1)
    assert M == pytest.approx(n2.max(), rel=1e-5)
    assert Xt[np.argmax(n2), 32] == 0.0
    assert np.allclose((Xt.astype(np.float64) ** 2).sum(1), M, rtol=2e-6)
    Qt = np.zeros((100, 36), np.float32)
    Qt[:, :32] = Q
    li, _ = oracle.bruteforce(Xt, Qt, 10, "l2")
    ii, _ = oracle.bruteforce(X, Q, 10, "ip")
    agree = (li == ii).mean()
    assert agree > 0.99, agree


def _complete_valid_subs(sizes, valid):
    """Complete input graphs over all vertices, and the same graphs over only
    the valid vertices (local ids renumbered in order)."""
    full, comp, off, coff = [], [], 0, 0
    for n in sizes:
        full.append((off, np.array([[j for j in range(n) if j != i] for i in range(n)], np.uint32), 0))
        keep = [i for i in range(n) if valid[off + i]]
        m = len(keep)
        adj = np.full((max(m, 1), max(m - 1, 1)), NONE, np.uint32)
        for a in range(m):
            row = [b for b in range(m) if b != a]
            adj[a, :len(row)] = row
        comp.append((coff, adj, 0))
        off += n
        coff += m
    return full, comp


def test_validity_all_ones_is_no_mask():
    cfg, X, subs = _cfg_small(sizes=(700, 500, 300))
    ones = np.ones(X.shape[0], np.uint8)
    a, ad, _ = oracle.cross_query(X, subs, cfg.k, cfg.L, cfg.metric)
    b, bd, _ = oracle.cross_query(X, subs, cfg.k, cfg.L, cfg.metric, valid=ones)
    assert (a == b).all() and (ad == bd).all()
    m1 = oracle.merge(X, subs, cfg.k, cfg.L, cfg.rounds, cfg.R, cfg.metric)
    m2 = oracle.merge(X, subs, cfg.k, cfg.L, cfg.rounds, cfg.R, cfg.metric, valid=ones)
    assert (m1[0] == m2[0]).all() and m1[2] == m2[2]


def test_deleted_vertices_equal_removed_vertices_on_complete_graphs():
    # phi keeps only valid vertices (Section 4.1.3).  With complete input
    # graphs and L >= every graph, each search returns its whole graph, so
    # merging with some vertices marked invalid must give, up to the
    # order-preserving renumbering, the merge of the data without them:
    # stage 1 is then the exact k-NN among valid vertices, and refinement
    # and prune see the same lists.
    rng = np.random.default_rng(17)
    sizes = (40, 55, 30)
    X = rng.integers(0, 256, (sum(sizes), 8)).astype(np.float32)
    valid = (rng.random(sum(sizes)) > 0.3).astype(np.uint8)
    full, comp = _complete_valid_subs(sizes, valid)
    keep = np.nonzero(valid)[0]
    k, L, R = 8, 64, 10
    ids, dd, _ = oracle.cross_query(X, full, k, L, valid=valid)
    assert (ids[valid == 0] == NONE).all()
    gi, gd = oracle.bruteforce(X[keep], X[keep], k, exclude=np.arange(len(keep)))
    assert (ids[keep] == keep[gi]).all() and (dd[keep].astype(np.float64) == gd).all()
    pg, deg, _ = oracle.merge(X, full, k, L, 2, R, valid=valid)
    cpg, cdeg, _ = oracle.merge(X[keep], comp, k, L, 2, R)
    mapped = np.where(cpg == NONE, NONE, keep[np.minimum(cpg, len(keep) - 1)]).astype(np.uint32)
    assert (pg[keep] == mapped).all() and (deg[keep] == cdeg).all()
    assert (pg[valid == 0] == NONE).all() and (deg[valid == 0] == 0).all()


def test_deletion_and_overlap_invariants():
    # A deletion (random 30 % of one sub-index) and an overlap (a second copy
    # of vertices of another sub-index, marked invalid in one of them): no
    # invalid vertex is a neighbour anywhere, invalid rows are empty, the
    # merged entry is valid.
    cfg, X, subs = _cfg_small(sizes=(900, 600))
    rng = np.random.default_rng(3)
    valid = np.ones(X.shape[0], np.uint8)
    valid[rng.choice(900, 270, replace=False)] = 0
    valid[900:1000] = 0
    pg, deg, ent = oracle.merge(X, subs, cfg.k, cfg.L, cfg.rounds, cfg.R, cfg.metric, valid=valid)
    used = pg[pg != NONE]
    assert valid[used].all()
    assert (deg[valid == 0] == 0).all() and (deg[valid == 1] >= 1).all()
    assert valid[ent] == 1


def test_merged_entry_with_invalid_entries():
    def subs(sizes, entries):
        out, off = [], 0
        for n, e in zip(sizes, entries):
            out.append((off, np.zeros((n, 1), np.uint32), e))
            off += n
        return out
    s = subs((30, 70, 50), (4, 9, 2))
    valid = np.ones(150, np.uint8)
    assert oracle.merged_entry(s, valid) == 39
    valid[39] = 0
    valid[30:35] = 0
    assert oracle.merged_entry(s, valid) == 35          # smallest valid id of sub-index 1
    valid[30:100] = 0
    assert oracle.merged_entry(s, valid) == 102          # next largest: sub-index 2's entry
    valid[:] = 0
    assert oracle.merged_entry(s, valid) == NONE


def test_rerank_takes_the_first_valid_results():
    # low-precision copy and validity together: each search's first `rerank`
    # valid results, re-scored on the FP32 rows
    cfg, X, subs = _cfg_small("cfg1ov", sizes=(500, 400, 300))
    rng = np.random.default_rng(32)
    Xs = (X + rng.normal(0, 0.5, X.shape)).astype(np.float32)
    valid = (rng.random(X.shape[0]) > 0.4).astype(np.uint8)
    nodes = np.nonzero(valid)[0][::19].astype(np.uint64)
    k, L, rr = 16, 32, 10
    ids, dd, _ = oracle.cross_query(X, subs, k, L, "l2", nodes=nodes, Xs=Xs, rerank=rr, valid=valid)
    offs = [s[0] for s in subs]
    for r, u in enumerate(nodes.astype(np.int64)):
        g = int(np.searchsorted(offs, u, side="right") - 1)
        off, adj, _ = subs[g]
        cand = [(oracle.distance(X[u], X[off + int(v)]), off + int(v)) for v in adj[u - off]
                if v != NONE and valid[off + int(v)]]
        for j, (offj, adjj, ej) in enumerate(subs):
            if j == g:
                continue
            res, _, _, _ = oracle.knn_search(X[u], Xs[offj:offj + adjj.shape[0]], adjj, ej, L, "l2")
            good = [offj + int(v) for v in res if valid[offj + int(v)]][:rr]
            cand += [(oracle.distance(X[u], X[v]), v) for v in good]
        cand.sort()
        got = [(float(dd[r, t]), int(ids[r, t])) for t in range(k) if ids[r, t] != NONE]
        assert got == cand[:k], u


def test_hnsw_layers_on_a_line():
    # Section 4.3.3: points 3i on a line; every 4th point reaches layer 1 and
    # every 16th layer 2.  Within a layer the heuristic keeps the nearest
    # member on each side (the next one further out is closer to that
    # member than to u), the reverse edges are the same edges, and pruning
    # again keeps them: each layer is the path over its members.  The top
    # entry is the smallest id of the highest layer.
    n = 64
    X = line_points(np.arange(n) * 3)
    lv = np.zeros(n, np.uint8)
    lv[::4] = 1
    lv[::16] = 2
    ids, adj, cnt, top = oracle.hnsw_layers(X, lv, M=4, ef=8)
    assert cnt.tolist() == [16, 4] and top == 0
    l1, a1 = ids[:16], adj[:16]
    assert l1.tolist() == list(range(0, 64, 4))
    for r, u in enumerate(l1.astype(np.int64)):
        want = [v for v in (u - 4, u + 4) if 0 <= v < n]
        assert [int(v) for v in a1[r] if v != NONE] == want
    l2, a2 = ids[16:], adj[16:]
    assert l2.tolist() == [0, 16, 32, 48]
    assert [int(v) for v in a2[1] if v != NONE] == [0, 32]


def test_hnsw_layers_invariants_and_search():
    # members are exactly the vertices with level >= l; rows are sorted by
    # distance, unique, without self-loops, at most M; searching the
    # hierarchy over a 1-D path base graph finds the true nearest point
    rng = np.random.default_rng(9)
    cfg, X, subs = _cfg_small()
    N = X.shape[0]
    M = 8
    lv = np.minimum(np.floor(-np.log(rng.random(N)) / np.log(M)), 5).astype(np.uint8)
    ids, adj, cnt, top = oracle.hnsw_layers(X, lv, M=M, ef=32, metric=cfg.metric)
    off = 0
    for l in range(1, len(cnt) + 1):
        mem = ids[off:off + cnt[l - 1]]
        assert mem.tolist() == np.nonzero(lv >= l)[0].tolist()
        for r in range(len(mem)):
            row = [int(v) for v in adj[off + r] if v != NONE]
            assert len(row) <= M and int(mem[r]) not in row and len(set(row)) == len(row)
            assert all(lv[v] >= l for v in row)
            d = [oracle.distance(X[mem[r]], X[v], cfg.metric) for v in row]
            assert d == sorted(d)
        off += int(cnt[l - 1])
    assert lv[top] == len(cnt)
    xs = rng.permutation(200).astype(np.float32) * 2.0
    P = line_points(xs)
    order = np.argsort(xs)
    base = np.full((200, 2), NONE, np.uint32)
    for i, v in enumerate(order):
        nb = [order[j] for j in (i - 1, i + 1) if 0 <= j < 200]
        base[v, :len(nb)] = nb
    plv = np.minimum(np.floor(-np.log(rng.random(200)) / np.log(4)), 3).astype(np.uint8)
    layers = oracle.hnsw_layers(P, plv, M=4, ef=16)
    for qx in (-5.0, 17.3, 201.0, 398.9, 1000.0):
        q = np.array([qx, 0, 0, 0], np.float32)
        got, _ = oracle.hnsw_search(q, P, base, layers, 4, 1)
        assert got[0] == int(np.argmin(np.abs(xs - qx)))
