"""The entry point that allocates nothing (fgim_cross_query_noalloc) gives
the bits of fgim_cross_query, over two calls in a row on one GPU, the second
with a smaller input (fewer vertices, fewer sub-indexes), so that state left
in the shared scratch array by the first call must not leak into the second."""
import numpy as np
import pytest
import torch

from wl import to_gpu, workload

pytestmark = pytest.mark.gpu

fg = pytest.importorskip("paper_2603_21710_amd")


def _both(name, sizes, precision="fp32", drop=0.0):
    cfg, X, graphs, _ = workload(name, sizes)
    lowp = lows = None
    if precision != "fp32":
        Xd = torch.from_numpy(X).cuda()
        lowp, lows = fg.quantize(Xd, precision)
    valid = None
    if drop:
        valid = (np.random.default_rng(3).random(X.shape[0]) >= drop).astype(np.uint8)
    m = to_gpu(X, graphs, cfg.metric, lowp, lows, valid=valid)
    p = fg.params(k=cfg.k, L=cfg.L, precision=precision)
    ref_ids, ref_d, _ = fg.cross_query(m, p)
    ids = torch.full_like(ref_ids, 7)
    dist = torch.full_like(ref_d, 3.0)
    print(f"noalloc {name} {sizes} {precision}: N={X.shape[0]} h={len(graphs)}", flush=True)
    fg.cross_query_noalloc(m, p, ids, dist)
    torch.cuda.synchronize()
    return ref_ids, ref_d, ids, dist


@pytest.mark.parametrize("first,second,precision", [
    (("cfg3", (300, 500, 700, 150, 900, 400, 1200, 650)), ("cfg1", (600, 400)), "fp32"),
    (("cfg2", (2500, 2000)), ("cfg2", (900, 700)), "fp32"),
    (("cfg4", (1200, 1000)), ("cfg4", (500, 300)), "bf16"),
    (("cfg2", (2500, 2000)), ("cfg2", (900, 700)), "fp8"),
])
def test_noalloc_matches_cross_query_twice(first, second, precision):
    for name, sizes in (first, second):
        ref_ids, ref_d, ids, dist = _both(name, sizes, precision)
        assert torch.equal(ids, ref_ids), f"{name} {sizes}: ids differ"
        assert torch.equal(dist.view(torch.int32), ref_d.view(torch.int32)), f"{name} {sizes}: distances differ"


def test_noalloc_with_validity_matches_cross_query_twice():
    # dropped vertices (the ID mapping's validity flags) on the first call,
    # none on the second, smaller one
    for (name, sizes), drop in ((("cfg2", (2500, 2000)), 0.3), (("cfg1", (600, 400)), 0.0)):
        ref_ids, ref_d, ids, dist = _both(name, sizes, drop=drop)
        assert torch.equal(ids, ref_ids), f"{name} {sizes}: ids differ"
        assert torch.equal(dist.view(torch.int32), ref_d.view(torch.int32)), f"{name} {sizes}: distances differ"


def test_noalloc_rejects_what_it_cannot_do_without_memory():
    cfg, X, graphs, _ = workload("cfg1", (600, 400))
    m = to_gpu(X, graphs, cfg.metric)
    ids = torch.empty((m.n, cfg.k), dtype=torch.int32, device="cuda")
    dist = torch.empty((m.n, cfg.k), dtype=torch.float32, device="cuda")
    for p in (fg.params(k=cfg.k, L=cfg.L, autotune=True), fg.params(k=cfg.k, L=cfg.L, precision="bf16")):
        with pytest.raises(fg.FgimError) as ei:
            fg.cross_query_noalloc(m, p, ids, dist)
        assert ei.value.name == "FGIM_ERR_INVALID_ARG"
