"""Builder for the pre-built input proximity graphs G_i.

The merge consumes h pre-built PGs over disjoint vector sets (the problem
definition "Merging Graph-based Indexes", Section 2.1).  This module makes
them: for each sub-index, the exact R_in-nearest-neighbour list of every
point (self excluded, ties by id), then the relative-neighbourhood (RNG)
occlusion heuristic that HNSW uses (Section 2.2: a candidate v of u is kept
when it is strictly closer to u than to every kept neighbour), and the
medoid -- the point closest to the mean, ties to the lowest id -- as the
entry point ep_i.

Small graphs are built in float64 on the CPU with exact (distance, id)
ordering; large graphs are built in float32 with torch on whatever device
the tensors live on (the input graph only has to be a valid PG; its exact
edges are not under test).  Adjacency rows hold local ids in ascending
distance order, padded with 0xFFFFFFFF.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

NONE = 0xFFFFFFFF


@dataclasses.dataclass
class InputPG:
    adj: np.ndarray        # uint32 [n, r_in], local ids, NONE-padded
    entry: int             # local id of the medoid
    mean_degree: float


def _pair_dist(G: torch.Tensor, sq_a: torch.Tensor, sq_b: torch.Tensor,
               metric: str) -> torch.Tensor:
    if metric == "l2":
        return (sq_a[..., :, None] + sq_b[..., None, :] - 2.0 * G).clamp_min_(0.0)
    if metric == "ip":
        return -G
    if metric == "cos":
        return 1.0 - G
    raise ValueError(metric)


def _knn(X: torch.Tensor, r: int, metric: str, exact: bool):
    """(ids [n, r], dists [n, r]) of the r nearest other points."""
    n = X.shape[0]
    sq = (X * X).sum(1)
    ids = torch.empty((n, r), dtype=torch.int64, device=X.device)
    dd = torch.empty((n, r), dtype=X.dtype, device=X.device)
    budget = (1 << 30) if X.device.type == "cuda" else (1 << 27)
    block = max(1, min(n, budget // max(1, n)))
    col = torch.arange(n, device=X.device)
    for s in range(0, n, block):
        e = min(n, s + block)
        D = _pair_dist(X[s:e] @ X.T, sq[s:e], sq, metric)
        D[torch.arange(e - s, device=X.device), col[s:e]] = float("inf")
        if exact:
            # Stable sort keeps ascending id order among equal distances.
            dv, di = torch.sort(D, dim=1, stable=True)
            ids[s:e], dd[s:e] = di[:, :r], dv[:, :r]
        else:
            dv, di = torch.topk(D, r, dim=1, largest=False, sorted=True)
            ids[s:e], dd[s:e] = di, dv
    return ids, dd


def _rng_prune(X: torch.Tensor, ids: torch.Tensor, du: torch.Tensor,
               metric: str) -> torch.Tensor:
    """Keep candidate v of u iff delta(u, v) < delta(w, v) for every kept w."""
    n, r = ids.shape
    keep = torch.zeros((n, r), dtype=torch.bool, device=X.device)
    block = max(1, ((1 << 26) if X.device.type == "cuda" else (1 << 24)) // max(1, r * r))
    for s in range(0, n, block):
        e = min(n, s + block)
        Xc = X[ids[s:e]]                                  # [b, r, d]
        sq = (Xc * Xc).sum(-1)
        G = torch.bmm(Xc, Xc.transpose(1, 2).contiguous())
        Dcc = _pair_dist(G, sq, sq, metric)               # [b, r, r]
        kb = torch.zeros((e - s, r), dtype=torch.bool, device=X.device)
        dub = du[s:e]
        finite = torch.isfinite(dub)
        for p in range(r):
            occl = (kb[:, :p] & (Dcc[:, :p, p] <= dub[:, p:p + 1])).any(1)
            kb[:, p] = finite[:, p] & ~occl
        keep[s:e] = kb
    return keep


def build_input_pg(X_sub: np.ndarray | torch.Tensor, r_in: int, metric: str,
                   device: Optional[str] = None,
                   exact: Optional[bool] = None) -> InputPG:
    """Exact r_in-NN + RNG prune + medoid entry for one sub-index."""
    if isinstance(X_sub, np.ndarray):
        Xt = torch.from_numpy(np.ascontiguousarray(X_sub))
    else:
        Xt = X_sub
    n = Xt.shape[0]
    if device is None:
        device = "cpu" if n <= 20000 else ("cuda" if torch.cuda.is_available() else "cpu")
    if exact is None:
        exact = n <= 20000
    dtype = torch.float64 if (exact and device == "cpu") else torch.float32
    X = Xt.to(device=device, dtype=dtype)
    r = min(r_in, n - 1)
    adj = np.full((n, r_in), NONE, dtype=np.uint32)
    if r <= 0:
        return InputPG(adj=adj, entry=0, mean_degree=0.0)
    ids, dd = _knn(X, r, metric, exact)
    keep = _rng_prune(X, ids, dd, metric)
    # Compact the kept ids to the front of each row, preserving order.
    order = torch.argsort((~keep).to(torch.int8), dim=1, stable=True)
    kid = torch.gather(ids, 1, order)
    kcnt = keep.sum(1)
    pos = torch.arange(r, device=X.device)[None, :]
    kid = torch.where(pos < kcnt[:, None], kid, torch.full_like(kid, NONE))
    adj[:, :r] = kid.cpu().numpy().astype(np.uint32)
    Xd = X.to(torch.float64)
    mean = Xd.mean(0)
    entry = int(torch.argmin(((Xd - mean) ** 2).sum(1)).item())
    return InputPG(adj=adj, entry=entry,
                   mean_degree=float(kcnt.to(torch.float64).mean().item()))


def reach_fraction(adj: np.ndarray, entry: int) -> float:
    """Fraction of vertices reachable from entry along out-edges."""
    n = adj.shape[0]
    seen = np.zeros(n, dtype=bool)
    seen[entry] = True
    frontier = np.array([entry], dtype=np.int64)
    while frontier.size:
        nb = adj[frontier].reshape(-1)
        nb = nb[nb != NONE].astype(np.int64)
        nb = np.unique(nb)
        nb = nb[~seen[nb]]
        seen[nb] = True
        frontier = nb
    return float(seen.mean())
