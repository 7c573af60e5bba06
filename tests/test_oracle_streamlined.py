"""Pins of the oracle's streamlined refinement (Section 4.2.1, Algorithm 3):
each round visits consecutive vertex ranges in turn, and a range's Visit and
Update read the lists as the ranges before it left them.

With one vertex per range the oracle must equal a plain one-vertex-at-a-time
pass written here from the algorithm, which inserts every proposal into its
list at once.  The data are small integers, so every distance is exact and
this reference needs no part of the oracle's arithmetic."""
import numpy as np
import pytest

import oracle
from helpers import NONE


def _exact(X, a, b, metric):
    xa, xb = X[a].astype(np.int64), X[b].astype(np.int64)
    if metric == "l2":
        return int(((xa - xb) ** 2).sum())
    return -int((xa * xb).sum())


def _inputs(seed, N, k, dim, sizes, metric, partial=0.2):
    """Integer rows, h sub-indexes of the given sizes, and sorted (delta, id)
    lists of up to k random other vertices, some lists not full."""
    rng = np.random.default_rng(seed)
    X = rng.integers(-6, 7, (N, dim)).astype(np.float32)
    offs = np.cumsum([0] + list(sizes))[:-1]
    subs = [(int(o), np.zeros((n, 1), np.uint32), 0) for o, n in zip(offs, sizes)]
    gsub = np.repeat(np.arange(len(sizes)), sizes)
    ids = np.full((N, k), NONE, np.uint32)
    dd = np.full((N, k), np.inf, np.float32)
    for u in range(N):
        m = k if rng.random() > partial else int(rng.integers(1, k))
        others = rng.choice(np.delete(np.arange(N), u), m, replace=False)
        row = sorted((_exact(X, u, int(v), metric), int(v)) for v in others)
        ids[u, :m] = [v for _, v in row]
        dd[u, :m] = [d for d, _ in row]
    return X, subs, gsub, ids, dd


def _sequential(X, gsub, ids, dd, rounds, k_rev, metric):
    """Algorithm 3 one vertex at a time in ascending id, with its updates
    applied in place.  An entry carries two marks: new (not yet seen by a
    Visit of its owner) and a recorded reverse link (set when its owner's
    Visit sees it new, moved into Cn by the next Visit of its target).
    Reverse lists are read from the current lists, the first k_rev by
    (stored delta, id).  Returns (ids, dist, flags) with flags bit 0 = new
    and bit 2 = recorded reverse link."""
    N, k = ids.shape
    # entries [delta, id, new, rlink]
    lists = [[[int(d), int(v), True, False] for d, v in zip(dd[u], ids[u]) if v != NONE] for u in range(N)]

    def insert(t, v, d):
        L = lists[t]
        if any(e[1] == v for e in L):
            return
        if len(L) == k and (d, v) >= (L[-1][0], L[-1][1]):
            return
        L.append([d, v, True, False])
        L.sort(key=lambda e: (e[0], e[1]))
        del L[k:]

    for _ in range(rounds):
        for u in range(N):
            inn = [(e[0], w, e[3]) for w in range(N) for e in lists[w] if e[1] == u]
            rn = sorted((d, w) for d, w, rl in inn if rl)[:k_rev]
            ro = sorted((d, w) for d, w, rl in inn if not rl)[:k_rev]
            fwd_new = [e[1] for e in lists[u] if e[2]]
            fwd_old = [e[1] for e in lists[u] if not e[2]]
            Cn = sorted(set(fwd_new) | {w for _, w in rn})
            Co = sorted((set(fwd_old) | {w for _, w in ro}) - set(Cn))
            for w in range(N):             # u consumes its reverse links
                for e in lists[w]:
                    if e[1] == u:
                        e[3] = False
            for e in lists[u]:             # and records its new entries as links
                if e[2]:
                    e[2], e[3] = False, True
            pairs = [(Cn[i], Cn[j]) for i in range(len(Cn)) for j in range(i + 1, len(Cn))]
            pairs += [(a, b) for a in Cn for b in Co]
            for a, b in pairs:
                if gsub[a] == gsub[b]:
                    continue
                d = _exact(X, a, b, metric)
                insert(a, b, d)
                insert(b, a, d)
    oi = np.full((N, k), NONE, np.uint32)
    od = np.full((N, k), np.inf, np.float32)
    of = np.zeros((N, k), np.uint8)
    for u in range(N):
        for j, (d, v, f, rl) in enumerate(lists[u]):
            oi[u, j], od[u, j], of[u, j] = v, d, int(f) | (4 if rl else 0)
    return oi, od, of


@pytest.mark.parametrize("seed,metric,sizes,k,k_rev,rounds", [
    (1, "l2", (14, 12, 10), 5, 5, 2),
    (2, "l2", (20, 16), 6, 3, 2),
    (3, "ip", (9, 11, 8, 10), 4, 4, 3),
    # small k: a proposal that duplicates a list's last entry is common
    (7, "l2", (12, 12), 2, 2, 3),
    (8, "l2", (10, 9, 11), 3, 2, 3),
    (9, "ip", (15, 15), 3, 3, 2),
])
def test_one_vertex_batches_equal_the_sequential_pass(seed, metric, sizes, k, k_rev, rounds):
    N = sum(sizes)
    X, subs, gsub, ids, dd = _inputs(seed, N, k, 8, sizes, metric)
    si, sd, sf = _sequential(X, gsub, ids, dd, rounds, k_rev, metric)
    oi, od, of, T, st = oracle.refine(X, subs, ids, dd, rounds, metric, k_rev=k_rev, do_repair=False,
                                      batches=N)
    assert st["proposals"] > 0
    assert (oi == si).all()
    assert (od == sd).all()
    assert (of == sf).all()


def test_one_batch_is_the_synchronous_round():
    X, subs, gsub, ids, dd = _inputs(4, 40, 5, 8, (22, 18), "l2")
    a = oracle.refine(X, subs, ids, dd, 3, "l2")
    b = oracle.refine(X, subs, ids, dd, 3, "l2", batches=1)
    for x, y in zip(a[:4], b[:4]):
        assert (x == y).all()
    # a synchronous round records and consumes every reverse link at once
    assert not (a[2] & 4).any()


def test_streamlined_differs_from_synchronous():
    # the second range reads lists that the first range's proposals changed
    X, subs, gsub, ids, dd = _inputs(5, 60, 6, 8, (30, 30), "l2")
    si, sd, sf, _, _ = oracle.refine(X, subs, ids, dd, 1, "l2", do_repair=False)
    bi, bd, bf, _, _ = oracle.refine(X, subs, ids, dd, 1, "l2", do_repair=False, batches=2)
    assert not ((si == bi).all() and (sf == bf).all())


@pytest.mark.parametrize("batches", [2, 3, 7, 64])
def test_streamlined_invariants(batches):
    N, k = 64, 6
    X, subs, gsub, ids, dd = _inputs(6 + batches, N, k, 8, (25, 20, 19), "l2")
    oi, od, of, T, st = oracle.refine(X, subs, ids, dd, 2, "l2", batches=batches)
    for u in range(N):
        row = [(float(d), int(v)) for d, v in zip(od[u], oi[u]) if v != NONE]
        assert row == sorted(row)
        assert len({v for _, v in row}) == len(row)
        assert u not in {v for _, v in row}
        for d, v in row:
            assert d == _exact(X, u, v, "l2")
        assert (oi[u, len(row):] == NONE).all()
    assert (np.bincount(oi[oi != NONE].astype(np.int64), minlength=N) == T).all()


@pytest.mark.parametrize("batches", [2, 5])
def test_streamlined_lists_only_improve_without_repair(batches):
    # without repair an entry leaves a list only for a closer one, so the
    # j-th key of every list can only fall
    N, k = 48, 5
    X, subs, gsub, ids, dd = _inputs(20 + batches, N, k, 8, (24, 24), "l2")
    oi, od, of, T, st = oracle.refine(X, subs, ids, dd, 2, "l2", do_repair=False, batches=batches)
    for u in range(N):
        n0 = int((ids[u] != NONE).sum())
        assert (oi[u, :n0] != NONE).all()
        for j in range(n0):
            assert (float(od[u, j]), int(oi[u, j])) <= (float(dd[u, j]), int(ids[u, j]))
