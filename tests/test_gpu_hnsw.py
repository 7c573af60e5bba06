"""GPU parity of HNSW-adaptive merging (Section 4.3.3): the upper layers
rebuilt over a merged base graph, and the search over the hierarchy, against
the oracle bit for bit.  Levels are drawn on the host with a seeded
generator and passed to both sides."""
import numpy as np
import pytest
import torch

import oracle
from helpers import NONE, line_points
from wl import to_gpu, workload

pytestmark = pytest.mark.gpu

fg = pytest.importorskip("paper_2603_21710_amd")


def _levels(n, M, seed, cap=6):
    rng = np.random.default_rng(seed)
    return np.minimum(np.floor(-np.log(rng.random(n)) / np.log(M)), cap).astype(np.uint8)


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("name,sizes,M,ef", [("cfg1ov", None, 16, 48), ("cfg2", (2500, 2000), 32, 64),
                                             ("cfg4", (1200, 1000), 48, 96), ("cfg3", (300, 500, 700, 150, 900,
                                                                                      400, 1200, 650), 8, 24)])
def test_layers_match_oracle(name, sizes, M, ef):
    cfg, X, graphs, _ = workload(name, sizes)
    lv = _levels(X.shape[0], 4, 5)
    print(f"case {name} N={X.shape[0]} M={M} ef={ef} layers={int(lv.max())}", flush=True)
    Xd = torch.from_numpy(X).cuda()
    ids, adj, counts, top = fg.hnsw_layers(Xd, torch.from_numpy(lv).cuda(), M, ef, cfg.metric)
    oi, oa, oc, otop = oracle.hnsw_layers(X, lv, M, ef, cfg.metric)
    assert counts == oc.tolist() and top == otop
    assert (_u32(ids) == oi).all()
    bad = np.argwhere(_u32(adj) != oa)
    assert bad.size == 0, f"{len(bad)} mismatches, first {bad[:3].tolist()}"


def test_layers_on_a_line():
    n = 64
    X = line_points(np.arange(n) * 3)
    lv = np.zeros(n, np.uint8)
    lv[::4] = 1
    lv[::16] = 2
    ids, adj, counts, top = fg.hnsw_layers(torch.from_numpy(X).cuda(), torch.from_numpy(lv).cuda(), 4, 8)
    assert counts == [16, 4] and top == 0
    a = _u32(adj)
    for r, u in enumerate(range(0, 64, 4)):
        assert [int(v) for v in a[r] if v != NONE] == [v for v in (u - 4, u + 4) if 0 <= v < n]


@pytest.mark.parametrize("name,sizes", [("cfg1ov", None), ("cfg2", (2500, 2000))])
def test_search_over_layers_matches_oracle(name, sizes):
    cfg, X, graphs, Q = workload(name, sizes)
    pg, deg, entry = oracle.merge(X, graphs, cfg.k, cfg.L, cfg.rounds, cfg.R, cfg.metric)
    M = cfg.R
    lv = _levels(X.shape[0], M, 11)
    layers = oracle.hnsw_layers(X, lv, M, 64, cfg.metric)
    Xd = torch.from_numpy(X).cuda()
    gl = fg.hnsw_layers(Xd, torch.from_numpy(lv).cuda(), M, 64, cfg.metric)
    Qd = torch.from_numpy(Q).cuda()
    for L in (10, 64):
        print(f"case {name} N={X.shape[0]} nq={Q.shape[0]} L={L} layers={int(lv.max())}", flush=True)
        ids, dist = fg.search_layers(Xd, torch.from_numpy(pg.view(np.int32)).cuda(), gl, M, Qd, L, 10, cfg.metric)
        gi, gd = _u32(ids), dist.cpu().numpy()
        for qi in range(0, Q.shape[0], 5):
            oi, od = oracle.hnsw_search(Q[qi], X, pg, layers, M, L, cfg.metric)
            nn = min(10, len(oi))
            assert gi[qi, :nn].tolist() == oi[:nn].tolist(), (L, qi)
            assert (gd[qi, :nn].view(np.uint32) == od[:nn].view(np.uint32)).all()


def test_layer_count_mismatch_is_rejected():
    cfg, X, graphs, _ = workload("cfg1", (600, 400))
    lv = _levels(X.shape[0], 4, 1)
    Xd = torch.from_numpy(X).cuda()
    counts = [int((lv >= l).sum()) for l in range(1, int(lv.max()) + 1)]
    counts[0] += 1
    import ctypes
    cnt = (ctypes.c_uint64 * len(counts))(*counts)
    ids = torch.empty(sum(counts), dtype=torch.int32, device="cuda")
    adj = torch.empty((sum(counts), 8), dtype=torch.int32, device="cuda")
    top = ctypes.c_uint32()
    rc = fg.lib().fgim_hnsw_layers(Xd.data_ptr(), X.shape[0], X.shape[1], X.shape[1], 0,
                                   torch.from_numpy(lv).cuda().data_ptr(), len(counts), 8, 16, cnt,
                                   ids.data_ptr(), adj.data_ptr(), ctypes.byref(top), None)
    assert rc == 1
