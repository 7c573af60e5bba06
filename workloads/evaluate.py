"""Quality measurement: exact FP64 k-NN ground truth and tie-aware recall.

Recall@k = |R ∩ R~| / k (Section 2.1).  A returned id counts as correct when
its FP64 distance to the query is at most the FP64 distance of the true k-th
neighbour, so ties at the k-th place are not penalised (integer-valued data
has real ties).  The ground truth runs on the CPU in float64 with torch's
multi-threaded matmul; it is evaluation arithmetic, not part of the merge.
"""

from __future__ import annotations

import numpy as np
import torch

NONE = 0xFFFFFFFF


def _dist64(Xb: torch.Tensor, sqb: torch.Tensor, Q: torch.Tensor, metric: str) -> torch.Tensor:
    G = Q @ Xb.T
    if metric == "l2":
        return (Q * Q).sum(1)[:, None] + sqb[None, :] - 2.0 * G
    if metric == "ip":
        return -G
    return 1.0 - G


def exact_knn_fp64(X: np.ndarray, Q: np.ndarray, k: int, metric: str = "l2",
                   exclude: np.ndarray | None = None, block: int = 256):
    """(ids int64 [nq, k], dists float64 [nq, k]) of the exact k-NN in FP64.
    exclude[i] (optional) is a base id removed from query i's candidates."""
    Xt = torch.from_numpy(np.ascontiguousarray(X)).to(torch.float64)
    sq = (Xt * Xt).sum(1)
    Qt = torch.from_numpy(np.ascontiguousarray(Q)).to(torch.float64)
    nq = Qt.shape[0]
    ids = np.empty((nq, k), np.int64)
    dd = np.empty((nq, k), np.float64)
    for s in range(0, nq, block):
        e = min(nq, s + block)
        D = _dist64(Xt, sq, Qt[s:e], metric)
        if exclude is not None:
            ex = torch.from_numpy(np.asarray(exclude[s:e], np.int64))
            D[torch.arange(e - s), ex] = float("inf")
        v, i = torch.topk(D, k, dim=1, largest=False, sorted=True)
        ids[s:e], dd[s:e] = i.numpy(), v.numpy()
    return ids, dd


def dist64_rows(X: np.ndarray, Q: np.ndarray, ids: np.ndarray, metric: str) -> np.ndarray:
    """FP64 distance of query i to base rows ids[i, :] (NONE -> +inf)."""
    valid = ids != NONE
    safe = np.where(valid, ids, 0).astype(np.int64)
    Xs = X[safe].astype(np.float64)
    Qd = Q.astype(np.float64)[:, None, :]
    if metric == "l2":
        d = ((Xs - Qd) ** 2).sum(-1)
    elif metric == "ip":
        d = -(Xs * Qd).sum(-1)
    else:
        d = 1.0 - (Xs * Qd).sum(-1)
    return np.where(valid, d, np.inf)


def tie_recall(X: np.ndarray, Q: np.ndarray, found: np.ndarray, kth: np.ndarray, k: int,
               metric: str, block: int = 2048) -> float:
    """Tie-aware Recall@k of found[:, :k] (uint32 ids) against kth = the
    FP64 distance of each query's true k-th neighbour."""
    hit = 0
    for s in range(0, found.shape[0], block):
        e = min(found.shape[0], s + block)
        d = dist64_rows(X, Q[s:e], found[s:e, :k], metric)
        hit += int((d <= kth[s:e, None]).sum())
    return hit / float(found.shape[0] * k)
