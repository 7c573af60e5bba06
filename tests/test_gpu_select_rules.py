"""GPU parity of the swap-in neighbour-selection rules of stage 3 (alpha-RNG
and tau-MNG, Section 4.3.1) and of the MIPS -> L2 transformation against the
oracle.  Each selection kernel (the MFMA-screened one and the all-FP32 one)
gets the oracle's refined lists as input; ids must match bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from wl import to_gpu, workload

pytestmark = pytest.mark.gpu

fg = pytest.importorskip("paper_2603_21710_amd")

CASES = [("cfg1ov", None), ("cfg2", (2500, 2000)), ("cfg4", (1200, 1000))]
RULES = [("alpha", 1.2), ("alpha", 1.25), ("tau", 0.0), ("tau", 0.3), ("tau", 2.0)]


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _refined(name, sizes):
    cfg, X, graphs, _ = workload(name, sizes)
    m = to_gpu(X, graphs, cfg.metric)
    oi, od, _ = oracle.cross_query(X, graphs, cfg.k, cfg.L, cfg.metric)
    ri, rd, _, rT, _ = oracle.refine(X, graphs, oi, od, cfg.rounds, cfg.metric)
    return cfg, X, graphs, m, ri, rd, rT


def _tau_for(cfg, tau):
    # tau in the units of the Euclidean distance: the cosine workload's unit
    # vectors sit about 1.3 apart, the others' about 10 (cfg1ov) and 250 (cfg2)
    scale = {"cos": 0.05, "l2": 1.0}[cfg.metric] * (50.0 if cfg.name.startswith("cfg2") else 1.0)
    return tau * scale


@pytest.mark.parametrize("name,sizes", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("rule,param", RULES, ids=[f"{r}{p}" for r, p in RULES])
def test_selection_rule_matches_oracle(name, sizes, rule, param):
    cfg, X, graphs, m, ri, rd, rT = _refined(name, sizes)
    if rule == "tau":
        param = _tau_for(cfg, param)
    dev = torch.device("cuda")
    gids = torch.from_numpy(ri.view(np.int32)).to(dev)
    gd = torch.from_numpy(rd).to(dev)
    gT = torch.from_numpy(rT.view(np.int32)).to(dev)
    print(f"case {name} rule={rule} param={param}", flush=True)
    for R in (cfg.R, 8):
        pi, _, pdeg = oracle.prune(X, ri, rd, rT, R, cfg.metric, rule=rule, param=param)
        for flags in (0, fg.FGIM_FLAG_NO_MFMA_SCREEN):
            pg, deg = fg.prune(m, fg.params(k=cfg.k, L=cfg.L, R=R, flags=flags, select_rule=rule,
                                            select_param=param), gids, gd, gT)
            bad = np.argwhere(_u32(pg) != pi)
            assert bad.size == 0, f"R={R} flags={flags}: {len(bad)} mismatches, first {bad[:3].tolist()}"
            assert (_u32(deg) == pdeg).all()


def test_alpha_rng_merge_matches_oracle():
    cfg, X, graphs, _ = workload("cfg2", (2500, 2000))
    m = to_gpu(X, graphs, cfg.metric)
    p = fg.params(k=cfg.k, L=cfg.L, R=cfg.R, rounds=cfg.rounds, select_rule="alpha", select_param=1.2)
    pg, deg, entry, _ = fg.merge(m, p)
    oi, od, _ = oracle.cross_query(X, graphs, cfg.k, cfg.L, cfg.metric)
    ri, rd, _, rT, _ = oracle.refine(X, graphs, oi, od, cfg.rounds, cfg.metric)
    pi, _, pdeg = oracle.prune(X, ri, rd, rT, cfg.R, cfg.metric, rule="alpha", param=1.2)
    assert (_u32(pg) == pi).all() and (_u32(deg) == pdeg).all()


def test_rules_need_a_metric_distance():
    cfg, X, graphs, _ = workload("cfg3", (300, 500, 700, 150, 900, 400, 1200, 650))
    m = to_gpu(X, graphs, cfg.metric)
    ids, dist, _ = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L))
    T, _ = fg.refine(m, fg.params(k=cfg.k, L=cfg.L, rounds=1), ids, dist)
    for rule, param in (("alpha", 1.2), ("tau", 0.1), ("alpha", 0.5)):
        with pytest.raises(fg.FgimError) as ei:
            fg.prune(m, fg.params(k=cfg.k, L=cfg.L, R=cfg.R, select_rule=rule, select_param=param), ids, dist, T)
        assert ei.value.name == "FGIM_ERR_INVALID_ARG"


def test_mips_to_l2_matches_oracle_and_merges_under_l2():
    # 2 M rows of widely spread lengths: every row's square root is checked
    # against the oracle's correctly rounded sqrtf.
    rng = np.random.default_rng(5)
    X = (rng.normal(size=(2_000_000, 32)) * np.exp(rng.uniform(-4, 4, (2_000_000, 1)))).astype(np.float32)
    Xt, M = fg.mips_to_l2(torch.from_numpy(X).cuda())
    ot, oM = oracle.mips_to_l2(X)
    assert float(M.item()) == oM
    assert (Xt.cpu().numpy().view(np.uint32) == ot.view(np.uint32)).all()
    # the batching workload's inner-product data, transformed, merged under L2
    cfg, Xi, graphs, _ = workload("cfg3", (300, 500, 700, 150, 900, 400, 1200, 650))
    Xl, _ = oracle.mips_to_l2(Xi)
    m = to_gpu(Xl, graphs, "l2")
    p = fg.params(k=cfg.k, L=cfg.L, R=cfg.R, rounds=cfg.rounds, select_rule="alpha", select_param=1.2)
    pg, deg, entry, _ = fg.merge(m, p)
    oi, od, _ = oracle.cross_query(Xl, graphs, cfg.k, cfg.L, "l2")
    ri, rd, _, rT, _ = oracle.refine(Xl, graphs, oi, od, cfg.rounds, "l2")
    pi, _, pdeg = oracle.prune(Xl, ri, rd, rT, cfg.R, "l2", rule="alpha", param=1.2)
    assert (_u32(pg) == pi).all() and (_u32(deg) == pdeg).all()


@pytest.mark.parametrize("n,d", [(100_003, 96), (20_001, 300), (9_999, 768), (1_003, 4096), (7, 8)])
def test_mips_to_l2_every_row_shape(n, d):
    # one chunk per lane (d <= 256) and 2, 4 and 16 per lane (d = 300, 768,
    # 4096), with row counts that leave the last step of row groups partial
    rng = np.random.default_rng(d)
    X = (rng.normal(size=(n, d)) * np.exp(rng.uniform(-3, 3, (n, 1)))).astype(np.float32)
    print(f"case n={n} d={d}", flush=True)
    Xt, M = fg.mips_to_l2(torch.from_numpy(X).cuda())
    ot, oM = oracle.mips_to_l2(X)
    assert float(M.item()) == oM
    assert (Xt.cpu().numpy().view(np.uint32) == ot.view(np.uint32)).all()
