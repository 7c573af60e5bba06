"""GPU parity of phi's validity flags (Section 4.1.3; deletion and overlap,
Exp. 8) against the oracle: dropped vertices get empty rows and never appear
as neighbours, the searches still route through them, and the merged entry
is a retained vertex."""
import numpy as np
import pytest
import torch

import oracle
from wl import CFG5_SMALL, to_gpu, workload

pytestmark = pytest.mark.gpu

fg = pytest.importorskip("paper_2603_21710_amd")

NONE = 0xFFFFFFFF


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _mask(n, frac, seed, overlap=None):
    rng = np.random.default_rng(seed)
    v = (rng.random(n) >= frac).astype(np.uint8)
    if overlap is not None:
        v[overlap[0]:overlap[1]] = 0
    return v


CASES = [("cfg1ov", None, 0.3), ("cfg2", (2500, 2000), 0.5),
         ("cfg3", (300, 500, 700, 150, 900, 400, 1200, 650), 0.1), ("cfg5", CFG5_SMALL, 0.3)]


@pytest.mark.parametrize("name,sizes,frac", CASES, ids=[c[0] for c in CASES])
def test_stage1_with_deletions_matches_oracle(name, sizes, frac):
    cfg, X, graphs, _ = workload(name, sizes)
    valid = _mask(X.shape[0], frac, 7)
    print(f"case {name} N={X.shape[0]} dropped={int((valid == 0).sum())}", flush=True)
    m = to_gpu(X, graphs, cfg.metric, valid=valid)
    ids, dist, _ = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L))
    oi, od, _ = oracle.cross_query(X, graphs, cfg.k, cfg.L, cfg.metric, valid=valid)
    assert (_u32(ids) == oi).all()
    assert (dist.cpu().numpy().view(np.uint32) == od.view(np.uint32)).all()
    assert (oi[valid == 0] == NONE).all() and valid[oi[oi != NONE]].all()
    # the entry point that allocates nothing takes the same flags
    ids2 = torch.empty_like(ids)
    dist2 = torch.empty_like(dist)
    fg.cross_query_noalloc(m, fg.params(k=cfg.k, L=cfg.L), ids2, dist2)
    assert torch.equal(ids2, ids) and torch.equal(dist2, dist)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_precision_form_with_deletions_matches_oracle(prec):
    cfg, X, graphs, _ = workload("cfg2", (2500, 2000))
    valid = _mask(X.shape[0], 0.4, 11)
    deq = oracle.quantize_bf16(X)[1] if prec == "bf16" else oracle.quantize_fp8(X)[2]
    rerank = min(cfg.L, 2 * cfg.k)
    m = to_gpu(X, graphs, cfg.metric, valid=valid)
    ids, dist, _ = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L, precision=prec))
    oi, od, _ = oracle.cross_query(X, graphs, cfg.k, cfg.L, cfg.metric, Xs=deq, rerank=rerank, valid=valid)
    assert (_u32(ids) == oi).all()
    assert (dist.cpu().numpy().view(np.uint32) == od.view(np.uint32)).all()


@pytest.mark.parametrize("scenario", ["deletion", "overlap", "entry_dropped"])
def test_merge_with_validity_matches_oracle(scenario):
    cfg, X, graphs, _ = workload("cfg2", (2500, 2000))
    N = X.shape[0]
    if scenario == "deletion":
        valid = _mask(N, 0.3, 3)
    elif scenario == "overlap":
        # the second sub-index repeats the first 600 vertices of the first
        # one (a copy in an overlapping index); phi keeps one copy
        X = X.copy()
        X[2500:3100] = X[:600]
        valid = np.ones(N, np.uint8)
        valid[2500:3100] = 0
    else:
        valid = _mask(N, 0.2, 4)
        valid[graphs[0][0] + graphs[0][2]] = 0       # the largest sub-index's entry
        valid[:40] = 0
    m = to_gpu(X, graphs, cfg.metric, valid=valid)
    p = fg.params(k=cfg.k, L=cfg.L, R=cfg.R, rounds=cfg.rounds)
    pg, deg, entry, _ = fg.merge(m, p)
    oi, odeg, oent = oracle.merge(X, graphs, cfg.k, cfg.L, cfg.rounds, cfg.R, cfg.metric, valid=valid)
    assert (_u32(pg) == oi).all() and (_u32(deg) == odeg).all()
    assert entry == oent and valid[entry] == 1
    assert (odeg[valid == 0] == 0).all() and valid[oi[oi != NONE]].all()


@pytest.mark.parametrize("name,sizes,batches", [("cfg1ov", None, 5),
                                                ("cfg3", (300, 500, 700, 150, 900, 400, 1200, 650), 3)])
def test_streamlined_merge_with_deletions_matches_oracle(name, sizes, batches):
    # validity, streamlined refinement and the prune together: the dropped
    # vertices stay out of every list through the ranges as well
    cfg, X, graphs, _ = workload(name, sizes)
    valid = _mask(X.shape[0], 0.25, 11)
    print(f"case {name} N={X.shape[0]} dropped={int((valid == 0).sum())} batches={batches}", flush=True)
    m = to_gpu(X, graphs, cfg.metric, valid=valid)
    p = fg.params(k=cfg.k, L=cfg.L, R=cfg.R, rounds=cfg.rounds, stream_batches=batches)
    pg, deg, entry, _ = fg.merge(m, p, stats=True)
    oi, odeg, oent = oracle.merge(X, graphs, cfg.k, cfg.L, cfg.rounds, cfg.R, cfg.metric, valid=valid,
                                  batches=batches)
    assert (_u32(pg) == oi).all()
    assert (_u32(deg) == odeg).all()
    assert entry == oent
    gone = np.nonzero(valid == 0)[0]
    assert (odeg[gone] == 0).all() and not np.isin(oi[oi != NONE], gone).any()
