"""GPU parity at the full size of the 2 x 500,000, d = 128 workload, in the
launch configuration the benchmark times.  Each stage gets identical inputs
on both sides: stage 1 on 20,000 sampled vertices (the oracle computes them
one by one), stage 2 on the GPU's stage-1 lists in full (every round, the
repair and the indegrees), stage 3 on the oracle's stage-2 lists in full.
At this size the refinement's prefix scans span more than 1,024 blocks and
the join's pair buffer is claimed by thousands of workgroups, paths that
the small cases never reach."""
import numpy as np
import pytest
import torch

import oracle
from helpers import NONE
from wl import to_gpu, workload

pytestmark = pytest.mark.gpu

fg = pytest.importorskip("paper_2603_21710_amd")


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _same(g_ids, g_d, o_ids, o_d, label):
    bad = np.argwhere(g_ids != o_ids)
    assert bad.size == 0, f"{label}: {len(bad)} id mismatches, first {bad[:3].tolist()}"
    assert (g_d.view(np.uint32) == o_d.view(np.uint32)).all(), f"{label}: distance bits differ"


@pytest.mark.timeout(900)
def test_full_size_stage_isolated_parity():
    cfg, X, graphs, _ = workload("cfg2")
    N = X.shape[0]
    print(f"full size: N={N} d={X.shape[1]} h={len(graphs)}", flush=True)
    m = to_gpu(X, graphs, cfg.metric)
    p = fg.params(k=cfg.k, L=cfg.L, R=cfg.R, rounds=cfg.rounds)

    ids, dist, st = fg.cross_query(m, p, stats=True)
    gi, gd = _u32(ids), dist.cpu().numpy()
    assert st["searches"] == N
    nodes = np.sort(np.random.default_rng(2024).choice(N, 20000, replace=False))
    oi, od, _ = oracle.cross_query(X, graphs, cfg.k, cfg.L, cfg.metric, nodes=nodes)
    _same(gi[nodes], gd[nodes], oi, od, "stage 1 (sampled)")
    print("stage 1: 20000 sampled vertices bit-exact", flush=True)

    ri, rd, _, rT, rst = oracle.refine(X, graphs, gi, gd, cfg.rounds, cfg.metric)
    T, st2 = fg.refine(m, p, ids, dist, stats=True)
    _same(_u32(ids), dist.cpu().numpy(), ri, rd, "stage 2")
    assert (_u32(T) == rT).all()
    assert st2["proposals"] == rst["proposals"] and st2["repaired"] == rst["repaired"]
    print(f"stage 2: bit-exact, {rst['proposals']} proposals, {rst['repaired']} repaired", flush=True)

    pi, pd, pdeg = oracle.prune(X, ri, rd, rT, cfg.R, cfg.metric)
    dev = torch.device("cuda")
    pg, deg = fg.prune(m, p, torch.from_numpy(ri.view(np.int32)).to(dev), torch.from_numpy(rd).to(dev),
                       torch.from_numpy(rT.view(np.int32)).to(dev))
    assert (_u32(pg) == pi).all() and (_u32(deg) == pdeg).all()
    print("stage 3: bit-exact", flush=True)


def _integer_lists(seed, N, k, dim, partial=0.1):
    """Rows of small integers (every squared L2 distance exact in FP32) and
    sorted (delta, id) lists of k random other vertices, a tenth of them cut
    short."""
    rng = np.random.default_rng(seed)
    X = rng.integers(-6, 7, (N, dim)).astype(np.float32)
    ids = rng.integers(0, N - 1, (N, k), dtype=np.int64)
    ids += ids >= np.arange(N)[:, None]
    s = np.sort(ids, axis=1)
    for u in np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0]:
        ids[u] = rng.choice(np.delete(np.arange(N), u), k, replace=False)
    Xi = X.astype(np.int64)
    d = np.stack([((Xi - Xi[ids[:, j]]) ** 2).sum(1) for j in range(k)], axis=1)
    key = np.sort((d << 32) | ids, axis=1)
    out_i = (key & 0xFFFFFFFF).astype(np.uint32)
    out_d = (key >> 32).astype(np.float32)
    cut = (rng.random(N) < partial)[:, None] & (np.arange(k)[None, :] >= rng.integers(1, k, N)[:, None])
    out_i[cut] = NONE
    out_d[cut] = np.inf
    return X, out_i, out_d


@pytest.mark.timeout(900)
def test_refine_parity_with_more_segments_than_one_placing_pass_counts():
    # 8.5 M vertices: the reverse lists' 17 M segments make each coarse
    # bucket wider than the 8,192 segments a placing workgroup counts at a
    # time, so every bucket is placed in two passes; 1.3e8 proposals
    N, k = 8_500_000, 4
    X, ids0, d0 = _integer_lists(11, N, k, 4)
    subs = [(0, np.zeros((N // 2, 1), np.uint32), 0), (N // 2, np.zeros((N - N // 2, 1), np.uint32), 0)]
    print(f"wide buckets: N={N} k={k}", flush=True)
    ri, rd, _, rT, rst = oracle.refine(X, subs, ids0, d0, 1, "l2")
    m = to_gpu(X, subs, "l2")
    dev = torch.device("cuda")
    ids = torch.from_numpy(ids0.view(np.int32)).to(dev)
    dist = torch.from_numpy(d0).to(dev)
    T, st = fg.refine(m, fg.params(k=k, L=8, rounds=1), ids, dist, stats=True)
    _same(_u32(ids), dist.cpu().numpy(), ri, rd, "stage 2")
    assert (_u32(T) == rT).all()
    assert st["proposals"] == rst["proposals"] and st["repaired"] == rst["repaired"]
    print(f"bit-exact, {rst['proposals']} proposals, {rst['repaired']} repaired", flush=True)
