"""Quality measurement: exact FP64 k-NN ground truth and tie-aware recall.

Recall@k = |R ∩ R~| / k (Section 2.1).  A returned id counts as correct when
its FP64 distance to the query is at most the FP64 distance of the true k-th
neighbour, so ties at the k-th place are not penalised (integer-valued data
has real ties).  The ground truth runs on the CPU in float64: torch's
multi-threaded matmul (Gram form |q|^2 + |x|^2 - 2<q,x>) picks a shortlist,
which is re-ranked by the direct form that dist64_rows also uses to score
returned ids.  Both sides of the comparison "distance <= k-th distance" are
then the same function of the same rows, so the exact answer scores 1.0 on
float data too (the Gram and direct forms differ in the last bits).  It is
evaluation arithmetic, not part of the merge.
"""

from __future__ import annotations

import time

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
                   exclude: np.ndarray | None = None, block: int = 256, margin: int = 16):
    """(ids int64 [nq, k], dists float64 [nq, k]) of the exact k-NN in FP64,
    ordered by (distance, id); the distances are dist64_rows' direct form.
    exclude[i] (optional) is a base id removed from query i's candidates.

    The Gram form picks the k + margin closest candidates; they are re-scored
    in the direct form and the first k kept.  The Gram form's error is below
    tol = 1e-9 (|q|^2 + max|x|^2) (its rounding is ~1e-16 of those terms),
    so a true k-th neighbour can only be missed when the shortlist's last
    Gram distance lies within 2 tol of the direct k-th distance; such queries
    are recomputed directly over every base row."""
    Xt = torch.from_numpy(np.ascontiguousarray(X)).to(torch.float64)
    sq = (Xt * Xt).sum(1)
    Qt = torch.from_numpy(np.ascontiguousarray(Q)).to(torch.float64)
    nq, n = Qt.shape[0], Xt.shape[0]
    m = min(n, k + margin)
    ids = np.empty((nq, k), np.int64)
    dd = np.empty((nq, k), np.float64)
    sqmax = float(sq.max()) if n else 0.0
    for s in range(0, nq, block):
        e = min(nq, s + block)
        D = _dist64(Xt, sq, Qt[s:e], metric)
        if exclude is not None:
            ex = torch.from_numpy(np.asarray(exclude[s:e], np.int64))
            D[torch.arange(e - s), ex] = float("inf")
        v, i = torch.topk(D, m, dim=1, largest=False, sorted=True)
        cand = i.numpy()
        dc = dist64_rows(X, Q[s:e], cand.astype(np.uint32), metric)
        if exclude is not None:
            dc[cand == np.asarray(exclude[s:e], np.int64)[:, None]] = np.inf
        order = np.lexsort((cand, dc), axis=1)
        cs = np.take_along_axis(cand, order, 1)[:, :k]
        ds = np.take_along_axis(dc, order, 1)[:, :k]
        tol = 1e-9 * ((Qt[s:e] * Qt[s:e]).sum(1).numpy() + sqmax + 1.0)
        last = v.numpy()[:, -1]
        for r in np.nonzero((m < n) & (last <= ds[:, -1] + 2 * tol))[0]:
            ex = None if exclude is None else int(exclude[s + r])
            cs[r], ds[r] = _direct_knn_one(X, Q[s + r], k, metric, ex)
        ids[s:e], dd[s:e] = cs, ds
    return ids, dd


def exact_knn_screened(X: np.ndarray, Q: np.ndarray, k: int, metric: str = "l2",
                       exclude: np.ndarray | None = None, Xdev: torch.Tensor | None = None,
                       block: int | None = None, margin: int = 48, widen: int = 16, progress=None):
    """exact_knn_fp64 with the shortlist screened in FP32 on the GPU (torch
    matmul: evaluation arithmetic, not the merge).  Every shortlist is
    re-ranked by the direct FP64 form on the CPU, and its completeness is
    proved per query: an FP32 Gram-form distance of d products is within
    B = 4 gamma_d (|q|^2 + max|x|^2) of the exact value (gamma_d =
    d u / (1 - d u), u = 2^-24, covering any summation order, doubled), so
    when the shortlist's last FP32 distance minus B exceeds the direct k-th
    distance, no row outside it can be among the k nearest.  Queries that
    fail the test get a 16x longer shortlist, then the direct FP64 pass over
    every row.  Returns what exact_knn_fp64 returns, and the count of
    queries that needed each fallback.  margin and widen set the two shortlist
    lengths, k + margin and widen (k + margin).  block (queries per GPU
    pass) defaults to what keeps one distance block near 2^30 entries;
    progress(done, total), if given, is called every ten seconds or so."""
    dev = Xdev.device if Xdev is not None else torch.device("cuda")
    Xg = Xdev if Xdev is not None else torch.from_numpy(np.ascontiguousarray(X)).to(dev)
    n, d = Xg.shape
    sqx = (Xg * Xg).sum(1)
    sqmax = max(float((Xg[c:c + (1 << 20)].to(torch.float64) ** 2).sum(1).max()) for c in range(0, n, 1 << 20))
    u = 2.0 ** -24
    gamma = d * u / (1.0 - d * u)
    nq = Q.shape[0]
    if block is None:
        block = max(32, min(1024, (1 << 30) // max(1, n)))
    ids = np.empty((nq, k), np.int64)
    dd = np.empty((nq, k), np.float64)
    fallback = [0, 0]
    t_last = time.time()
    for s in range(0, nq, block):
        if progress is not None and time.time() - t_last > 10.0:
            progress(s, nq)
            t_last = time.time()
        e = min(nq, s + block)
        Qg = torch.from_numpy(np.ascontiguousarray(Q[s:e])).to(dev)
        G = Qg @ Xg.T
        if metric == "l2":
            D = (Qg * Qg).sum(1)[:, None] + sqx[None, :] - 2.0 * G
        elif metric == "ip":
            D = -G
        else:
            D = 1.0 - G
        if exclude is not None:
            ex = torch.from_numpy(np.asarray(exclude[s:e], np.int64)).to(dev)
            D[torch.arange(e - s, device=dev), ex] = float("inf")
        qsq = (Q[s:e].astype(np.float64) ** 2).sum(1)
        bound = 4.0 * gamma * (qsq + sqmax)
        todo = np.arange(e - s)
        for tier, m in enumerate((min(n, k + margin), min(n, widen * (k + margin)))):
            v, i = torch.topk(D[torch.from_numpy(todo).to(dev)], m, dim=1, largest=False, sorted=True)
            cand = i.cpu().numpy()
            last = v[:, -1].double().cpu().numpy()
            dc = dist64_rows(X, Q[s + todo], cand.astype(np.uint32), metric)
            if exclude is not None:
                dc[cand == np.asarray(exclude, np.int64)[s + todo][:, None]] = np.inf
            order = np.lexsort((cand, dc), axis=1)
            cs = np.take_along_axis(cand, order, 1)[:, :k]
            ds = np.take_along_axis(dc, order, 1)[:, :k]
            ok = (m >= n) | (last - bound[todo] > ds[:, -1])
            ids[s + todo[ok]], dd[s + todo[ok]] = cs[ok], ds[ok]
            todo = todo[~ok]
            if todo.size == 0:
                break
            fallback[tier] += int(todo.size)
        for r in todo:
            ex = None if exclude is None else int(exclude[s + r])
            ids[s + r], dd[s + r] = _direct_knn_one(X, Q[s + r], k, metric, ex)
    return ids, dd, {"longer_shortlist": fallback[0], "direct_pass": fallback[1]}


def _direct_knn_one(X: np.ndarray, q: np.ndarray, k: int, metric: str, exclude=None,
                    chunk: int = 1 << 18):
    """Exact k-NN of one query by the direct FP64 form over every base row,
    in chunks of rows: (ids int64 [k], dists float64 [k])."""
    best_i = np.empty(0, np.int64)
    best_d = np.empty(0, np.float64)
    for c0 in range(0, X.shape[0], chunk):
        c1 = min(X.shape[0], c0 + chunk)
        idx = np.arange(c0, c1, dtype=np.int64)
        d = dist64_rows(X, q[None, :], idx[None, :].astype(np.uint32), metric)[0]
        if exclude is not None and c0 <= exclude < c1:
            d[exclude - c0] = np.inf
        ai = np.concatenate([best_i, idx])
        ad = np.concatenate([best_d, d])
        o = np.lexsort((ai, ad))[:k]
        best_i, best_d = ai[o], ad[o]
    return best_i, best_d


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
