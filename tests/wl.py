"""Workload fixtures shared by the GPU tests: seeded inputs at test sizes."""
import functools

import numpy as np
import torch

from workloads import build_input_pg, get_config, make_queries, make_vectors, split_sizes

# cfg5's parameter set (h = 20 uneven sub-indexes, d = 128, R_in = 48, k = 32,
# L = 96: two pool registers, R = 48) at a size the oracle finishes in seconds
CFG5_SMALL = (900, 700, 650, 800, 120, 60, 300, 210, 95, 150, 400, 70, 250, 180, 110, 330, 90,
              140, 75, 170)


@functools.lru_cache(maxsize=None)
def workload(name, sizes=None, device=None):
    """(cfg, X float32 [N, d], [(off, adj uint32, entry)], queries)."""
    cfg = get_config(name)
    if sizes is not None:
        cfg = cfg.scaled(tuple(sizes))
    X = make_vectors(cfg)
    graphs = []
    for off, n in split_sizes(cfg):
        pg = build_input_pg(X[off:off + n], cfg.r_in, cfg.metric, device=device)
        graphs.append((off, pg.adj, pg.entry))
    Q = make_queries(cfg, min(cfg.n_queries, 1000))
    return cfg, X, graphs, Q


def to_gpu(X, graphs, metric, lowp=None, lowp_scale=None, valid=None):
    import paper_2603_21710_amd as fg
    dev = torch.device("cuda")
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(dev)
    g = [(torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(dev), int(e))
         for _, a, e in graphs]
    vd = None if valid is None else torch.from_numpy(np.ascontiguousarray(valid, np.uint8)).to(dev)
    return fg.Merge(Xd, g, metric, lowp, lowp_scale, vd)
