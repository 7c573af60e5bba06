"""GPU tests of the stage-1 tuner: launch-shape tuning keeps every FP32 bit,
a lowered beam width stays at or above the minimum-querying bound (Section
4.1.2) and the run at that width is exactly stage 1 at that L, and decisions
persist in the cache file."""
import numpy as np
import pytest
import torch

import oracle
from helpers import NONE
from wl import to_gpu, workload

pytestmark = pytest.mark.gpu

fg = pytest.importorskip("paper_2603_21710_amd")

CFG3_SMALL = (300, 500, 700, 150, 900, 400, 1200, 650)


def _min_local(graphs):
    return min(int((a != NONE).sum(1).min()) for _, a, _ in graphs)


@pytest.fixture
def cache(tmp_path, monkeypatch):
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("FGIM_TUNE_CACHE", str(path))
    return path


def test_shape_tuning_keeps_bits_and_persists(cache, monkeypatch):
    cfg, X, graphs, _ = workload("cfg2", (2500, 2000))
    m = to_gpu(X, graphs, cfg.metric)
    ref, refd, _ = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L))
    ids, dist, st = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L, autotune=True), stats=True)
    # FP32 with two sub-indexes: the tuner may only pick the launch shape
    assert st["L_used"] == cfg.L
    assert st["ms_tune"] > 0
    assert torch.equal(ids, ref) and torch.equal(dist.view(torch.int32), refd.view(torch.int32))
    lines = cache.read_text().splitlines()
    assert any(l.startswith("shape/") for l in lines), lines
    P, w, v = (int(t) for t in lines[-1].split(" ")[1:])
    assert (st["lanes_per_dist"], st["waves_per_cu"], st["visited_slots"]) == (P, w, v)
    # the second call is a cache hit and launches the same shape
    ids2, _, st2 = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L, autotune=True), stats=True)
    assert st2["ms_tune"] == 0 and torch.equal(ids2, ref)
    assert (st2["lanes_per_dist"], st2["waves_per_cu"], st2["visited_slots"]) == (P, w, v)
    # a fresh read of the file (another path, then back) still hits
    monkeypatch.setenv("FGIM_TUNE_CACHE", "")
    monkeypatch.setenv("FGIM_TUNE_CACHE", str(cache))
    _, _, st3 = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L, autotune=True), stats=True)
    assert st3["ms_tune"] == 0


def test_fixed_launch_fields_are_kept(cache):
    cfg, X, graphs, _ = workload("cfg2", (2500, 2000))
    m = to_gpu(X, graphs, cfg.metric)
    _, _, st = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L, autotune=True, lanes_per_dist=8,
                                           visited_slots=256), stats=True)
    assert st["lanes_per_dist"] == 8 and st["visited_slots"] == 256


def test_batched_form_width_is_bounded_and_exact(cache):
    cfg, X, graphs, _ = workload("cfg3", CFG3_SMALL)
    m = to_gpu(X, graphs, cfg.metric)
    ids, dist, st = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L, autotune=True), stats=True)
    lo = oracle.min_L(cfg.k, _min_local(graphs), len(graphs))
    Lu = st["L_used"]
    print(f"cfg3 small: L_used={Lu} lower bound={lo} configured={cfg.L}", flush=True)
    assert lo <= Lu <= cfg.L
    assert any(l.startswith("width/") for l in cache.read_text().splitlines())
    # after tuning, stage 1 is Algorithm 2 at width L_used, bit for bit
    oi, od, _ = oracle.cross_query(X, graphs, cfg.k, Lu, cfg.metric)
    gi = ids.cpu().numpy().view(np.uint32)
    assert (gi == oi).all()
    assert (dist.cpu().numpy().view(np.uint32) == od.view(np.uint32)).all()
    # the tuned lists keep most of what the configured width finds
    ri, _, _ = oracle.cross_query(X, graphs, cfg.k, cfg.L, cfg.metric)
    keep = np.mean([len(set(a[a != NONE]) & set(b[b != NONE])) / max(1, (a != NONE).sum())
                    for a, b in zip(ri, gi)])
    assert keep >= 0.97, keep


def test_precision_form_width_respects_rerank(cache):
    cfg, X, graphs, _ = workload("cfg4", (1200, 1000))
    m = to_gpu(X, graphs, cfg.metric)
    _, _, st = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L, precision="bf16", rerank=48,
                                           autotune=True), stats=True)
    assert 48 <= st["L_used"] <= cfg.L
    _, _, st = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L, precision="fp8", autotune=True),
                              stats=True)
    lo = oracle.min_L(cfg.k, _min_local(graphs), len(graphs))
    assert lo <= st["L_used"] <= cfg.L


def test_memory_only_cache(monkeypatch):
    monkeypatch.setenv("FGIM_TUNE_CACHE", "")
    cfg, X, graphs, _ = workload("cfg1", None)
    m = to_gpu(X, graphs, cfg.metric)
    ref, _, _ = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L))
    ids, _, st = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L, autotune=True), stats=True)
    assert torch.equal(ids, ref)
    _, _, st2 = fg.cross_query(m, fg.params(k=cfg.k, L=cfg.L, autotune=True), stats=True)
    assert st2["ms_tune"] == 0
