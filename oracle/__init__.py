"""CPU oracle of the FGIM merge -- TEST INFRASTRUCTURE ONLY.

A plain C implementation (fgim_oracle.c) of the paper's Algorithms 1-5 used
to check the GPU library.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the library and its
Python binding never do, and the two share no code.

All arrays are numpy; ids are uint32 with 0xFFFFFFFF padding.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fgim_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
NONE = 0xFFFFFFFF
METRICS = {"l2": 0, "ip": 1, "cos": 2}
RULES = {"rng": 0, "alpha": 1, "tau": 2}   # stage-3 neighbour selection (Section 4.3.1)
FLAG_NEW = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (strict IEEE: no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
             "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
             "-Wno-unused-parameter", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Sub(ctypes.Structure):
    _fields_ = [("off", ctypes.c_uint64), ("n", ctypes.c_uint32),
                ("stride", ctypes.c_uint32), ("adj", ctypes.c_void_p),
                ("entry", ctypes.c_uint32)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        u32, u64, i32, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        L.oracle_distance.restype = ctypes.c_float
        L.oracle_distance.argtypes = [vp, vp, u32, i32]
        L.oracle_distance64.restype = ctypes.c_double
        L.oracle_distance64.argtypes = [vp, vp, u32, i32]
        L.oracle_knn_search.restype = i32
        L.oracle_knn_search.argtypes = [vp, vp, u64, u32, i32, vp, u32, u32, u32, u32,
                                        vp, vp, vp, vp]
        L.oracle_cross_query.restype = i32
        L.oracle_cross_query.argtypes = [vp, vp, u64, u32, i32, vp, u32, u32, u32, u32,
                                         vp, u64, vp, vp, i32, vp, vp]
        L.oracle_min_L.restype = u32
        L.oracle_min_L.argtypes = [u32, u32, u32]
        L.oracle_repair.restype = i32
        L.oracle_repair.argtypes = [u64, u32, vp, vp, vp, vp, vp]
        L.oracle_refine.restype = i32
        L.oracle_refine.argtypes = [vp, u64, u32, i32, vp, u32, u64, u32, u32, u32, vp, vp,
                                    vp, vp, i32, i32, vp, u32]
        L.oracle_prune.restype = i32
        L.oracle_prune.argtypes = [vp, u64, u32, i32, u64, u32, vp, vp, vp, u32, vp, vp, vp,
                                   i32, i32, ctypes.c_float]
        L.oracle_hnsw_layers.restype = i32
        L.oracle_hnsw_layers.argtypes = [vp, u64, u32, i32, u64, vp, u32, u32, u32, vp, vp, vp, vp,
                                         i32]
        L.oracle_hnsw_search.restype = i32
        L.oracle_hnsw_search.argtypes = [vp, vp, u64, u32, i32, u64, vp, u32, vp, vp, vp, u32, u32,
                                         u32, u32, vp, vp]
        L.oracle_mips_to_l2.restype = i32
        L.oracle_mips_to_l2.argtypes = [vp, u64, u64, u32, vp, u64, vp]
        L.oracle_prune_rows.restype = i32
        L.oracle_prune_rows.argtypes = [vp, u64, u32, i32, u64, u32, vp, vp, vp, u32, vp, u64,
                                        vp, vp, vp, i32, i32, ctypes.c_float]
        L.oracle_merged_entry.restype = u64
        L.oracle_merged_entry.argtypes = [vp, u32, vp]
        L.oracle_merge.restype = i32
        L.oracle_merge.argtypes = [vp, u64, u32, i32, vp, u32, u32, u32, u32, u32, u32, vp,
                                   vp, vp, i32, vp, u32]
        L.oracle_bruteforce.restype = i32
        L.oracle_bruteforce.argtypes = [vp, u64, u64, u32, i32, vp, u64, u64, u32, vp, vp,
                                        vp, i32]
        L.oracle_bf16_from_f32.restype = ctypes.c_uint16
        L.oracle_bf16_from_f32.argtypes = [ctypes.c_float]
        L.oracle_bf16_to_f32.restype = ctypes.c_float
        L.oracle_bf16_to_f32.argtypes = [ctypes.c_uint16]
        L.oracle_fp8_from_f32.restype = ctypes.c_uint8
        L.oracle_fp8_from_f32.argtypes = [ctypes.c_float]
        L.oracle_fp8_to_f32.restype = ctypes.c_float
        L.oracle_fp8_to_f32.argtypes = [ctypes.c_uint8]
        L.oracle_quantize_fp8.restype = i32
        L.oracle_quantize_fp8.argtypes = [vp, u64, u64, u32, vp, vp, vp]
        L.oracle_quantize_bf16.restype = i32
        L.oracle_quantize_bf16.argtypes = [vp, u64, u64, u32, vp, vp]
        _lib = L
    return _lib


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


def _f32(X) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32)
    return X


def _subs(subs: Sequence[Tuple[int, np.ndarray, int]]):
    """subs: (offset, adj uint32 [n, stride], entry) per sub-index."""
    keep = []
    arr = (_Sub * len(subs))()
    for i, (off, adj, entry) in enumerate(subs):
        a = np.ascontiguousarray(adj, dtype=np.uint32)
        keep.append(a)
        arr[i] = _Sub(int(off), a.shape[0], a.shape[1], _p(a), int(entry))
    return arr, keep


def distance(a, b, metric: str = "l2") -> float:
    a, b = _f32(a), _f32(b)
    return float(lib().oracle_distance(_p(a), _p(b), a.shape[-1], METRICS[metric]))


def distance64(a, b, metric: str = "l2") -> float:
    a, b = _f32(a), _f32(b)
    return float(lib().oracle_distance64(_p(a), _p(b), a.shape[-1], METRICS[metric]))


def knn_search(q, Xj, adj, entry: int, L: int, metric: str = "l2"):
    """Algorithm 1 on one graph: (ids, dists, ndc, expansions)."""
    q, Xj = _f32(q), _f32(Xj)
    adj = np.ascontiguousarray(adj, dtype=np.uint32)
    ids = np.empty(L, np.uint32)
    dd = np.empty(L, np.float32)
    ndc = ctypes.c_uint64()
    nexp = ctypes.c_uint64()
    n = lib().oracle_knn_search(_p(q), _p(Xj), Xj.shape[1], Xj.shape[1], METRICS[metric],
                                _p(adj), adj.shape[0], adj.shape[1], entry, L, _p(ids),
                                _p(dd), ctypes.byref(ndc), ctypes.byref(nexp))
    if n < 0:
        raise ValueError("oracle_knn_search: bad graph or arguments")
    return ids[:n].copy(), dd[:n].copy(), ndc.value, nexp.value


def _valid(valid, n):
    if valid is None:
        return None
    v = np.ascontiguousarray(valid, dtype=np.uint8)
    if v.shape != (n,):
        raise ValueError(f"valid must have {n} flags")
    return v


def cross_query(X, subs, k: int, L: int, metric: str = "l2", nodes=None,
                Xs=None, rerank: int = 0, threads: Optional[int] = None, valid=None):
    """Stage 1 (Algorithm 2) for `nodes` (all when None): (ids, dists, stats).
    valid (uint8 [N], optional): phi's validity flag of every global id."""
    X = _f32(X)
    vf = _valid(valid, X.shape[0])
    Xs_ = None if Xs is None else _f32(Xs)
    arr, keep = _subs(subs)
    if nodes is None:
        nn = X.shape[0]
        nptr = None
    else:
        nodes = np.ascontiguousarray(nodes, dtype=np.uint64)
        nn = nodes.shape[0]
        nptr = _p(nodes)
    ids = np.empty((nn, k), np.uint32)
    dd = np.empty((nn, k), np.float32)
    st = np.zeros(2, np.uint64)
    rc = lib().oracle_cross_query(_p(X), None if Xs_ is None else _p(Xs_), X.shape[1],
                                  X.shape[1], METRICS[metric], ctypes.addressof(arr),
                                  len(subs), k, L, rerank, nptr, nn, _p(ids), _p(dd),
                                  threads or default_threads(), _p(st),
                                  None if vf is None else _p(vf))
    if rc:
        raise ValueError("oracle_cross_query failed")
    return ids, dd, {"ndc": int(st[0]), "expansions": int(st[1])}


def min_L(k: int, min_local: int, h: int) -> int:
    return int(lib().oracle_min_L(k, min_local, h))


def repair(ids, dist, flags=None):
    """Algorithm 4 on copies: (ids, dist, flags, T, n_repaired)."""
    ids = np.array(ids, dtype=np.uint32, order="C", copy=True)
    dist = np.array(dist, dtype=np.float32, order="C", copy=True)
    N, k = ids.shape
    if flags is None:
        flags = np.where(ids == NONE, 0, FLAG_NEW).astype(np.uint8)
    else:
        flags = np.array(flags, dtype=np.uint8, order="C", copy=True)
    T = np.empty(N, np.uint32)
    nr = ctypes.c_uint64()
    if lib().oracle_repair(N, k, _p(ids), _p(dist), _p(flags), _p(T), ctypes.byref(nr)):
        raise ValueError("oracle_repair failed")
    return ids, dist, flags, T, nr.value


def refine(X, subs, ids, dist, rounds: int, metric: str = "l2", k_rev: int = 0,
           flags=None, do_repair: bool = True, threads: Optional[int] = None,
           batches: int = 1):
    """Stage 2 on copies: (ids, dist, flags, T, stats).  batches > 1: the
    streamlined form, each round visiting `batches` consecutive vertex
    ranges in turn, each on the lists the ranges before it left."""
    X = _f32(X)
    arr, keep = _subs(subs)
    ids = np.array(ids, dtype=np.uint32, order="C", copy=True)
    dist = np.array(dist, dtype=np.float32, order="C", copy=True)
    N, k = ids.shape
    if flags is None:
        flags = np.where(ids == NONE, 0, FLAG_NEW).astype(np.uint8)
    else:
        flags = np.array(flags, dtype=np.uint8, order="C", copy=True)
    T = np.zeros(N, np.uint32)
    st = np.zeros(2, np.uint64)
    rc = lib().oracle_refine(_p(X), X.shape[1], X.shape[1], METRICS[metric],
                             ctypes.addressof(arr), len(subs), N, k, rounds, k_rev,
                             _p(ids), _p(dist), _p(flags), _p(T), int(do_repair),
                             threads or default_threads(), _p(st), int(batches))
    if rc:
        raise ValueError("oracle_refine failed")
    return ids, dist, flags, T, {"proposals": int(st[0]), "repaired": int(st[1])}


def prune(X, ids, dist, T, R: int, metric: str = "l2", threads: Optional[int] = None,
          rule: str = "rng", param: float = 0.0):
    """Stage 3 (Algorithm 5; rule "alpha" / "tau" swaps in alpha-RNG with
    alpha = param or tau-MNG with tau = param): (out_ids [N, R], out_dist, deg)."""
    X = _f32(X)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    dist = np.ascontiguousarray(dist, dtype=np.float32)
    T = np.ascontiguousarray(T, dtype=np.uint32)
    N, k = ids.shape
    oi = np.empty((N, R), np.uint32)
    od = np.empty((N, R), np.float32)
    deg = np.empty(N, np.uint32)
    rc = lib().oracle_prune(_p(X), X.shape[1], X.shape[1], METRICS[metric], N, k, _p(ids),
                            _p(dist), _p(T), R, _p(oi), _p(od), _p(deg),
                            threads or default_threads(), RULES[rule], float(param))
    if rc:
        raise ValueError("oracle_prune failed")
    return oi, od, deg


def prune_rows(X, ids, dist, T, R: int, rows, metric: str = "l2", threads: Optional[int] = None,
               rule: str = "rng", param: float = 0.0):
    """Stage 3 (Algorithm 5) for the listed vertices of the full lists:
    (out_ids [len(rows), R], out_dist, deg), row r as prune() gives rows[r]."""
    X = _f32(X)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    dist = np.ascontiguousarray(dist, dtype=np.float32)
    T = np.ascontiguousarray(T, dtype=np.uint32)
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    N, k = ids.shape
    nr = rows.shape[0]
    oi = np.empty((nr, R), np.uint32)
    od = np.empty((nr, R), np.float32)
    deg = np.empty(nr, np.uint32)
    rc = lib().oracle_prune_rows(_p(X), X.shape[1], X.shape[1], METRICS[metric], N, k, _p(ids),
                                 _p(dist), _p(T), R, _p(rows), nr, _p(oi), _p(od), _p(deg),
                                 threads or default_threads(), RULES[rule], float(param))
    if rc:
        raise ValueError("oracle_prune_rows failed")
    return oi, od, deg


def hnsw_layers(X, levels, M: int, ef: int, metric: str = "l2", threads: Optional[int] = None):
    """Upper layers of HNSW-adaptive merging (Section 4.3.3) for levels
    (uint8 [N]): (layer_ids, layer_adj [rows, M], counts [max_level], top)."""
    X = _f32(X)
    lv = np.ascontiguousarray(levels, dtype=np.uint8)
    N = X.shape[0]
    max_level = int(lv.max()) if N else 0
    rows = int(sum(int((lv >= l).sum()) for l in range(1, max_level + 1)))
    ids = np.empty(max(rows, 1), np.uint32)
    adj = np.empty((max(rows, 1), M), np.uint32)
    cnt = np.zeros(max(max_level, 1), np.uint64)
    top = ctypes.c_uint32()
    rc = lib().oracle_hnsw_layers(_p(X), X.shape[1], X.shape[1], METRICS[metric], N, _p(lv),
                                  max_level, M, ef, _p(ids), _p(adj), _p(cnt), ctypes.byref(top),
                                  threads or default_threads())
    if rc:
        raise ValueError("oracle_hnsw_layers failed")
    return ids[:rows], adj[:rows], cnt[:max_level], top.value


def hnsw_search(q, X, base_adj, layers, M: int, L: int, metric: str = "l2"):
    """Search over the hierarchy: (ids, dists) of the final pool."""
    ids, adj, cnt, top = layers
    q, X = _f32(q), _f32(X)
    base_adj = np.ascontiguousarray(base_adj, dtype=np.uint32)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    adj = np.ascontiguousarray(adj, dtype=np.uint32)
    cnt = np.ascontiguousarray(cnt, dtype=np.uint64)
    oi = np.empty(L, np.uint32)
    od = np.empty(L, np.float32)
    n = lib().oracle_hnsw_search(_p(q), _p(X), X.shape[1], X.shape[1], METRICS[metric], X.shape[0],
                                 _p(base_adj), base_adj.shape[1], _p(ids), _p(adj), _p(cnt),
                                 len(cnt), M, top, L, _p(oi), _p(od))
    if n < 0:
        raise ValueError("oracle_hnsw_search failed")
    return oi[:n].copy(), od[:n].copy()


def mips_to_l2(X):
    """MIPS -> L2 transform: (rows [n, d + 4] float32, M = max |x|^2)."""
    X = _f32(X)
    n, d = X.shape
    out = np.empty((n, d + 4), np.float32)
    M = ctypes.c_float()
    if lib().oracle_mips_to_l2(_p(X), n, d, d, _p(out), d + 4, ctypes.byref(M)):
        raise ValueError("oracle_mips_to_l2 failed")
    return out, M.value


def merged_entry(subs, valid=None) -> int:
    arr, keep = _subs(subs)
    n = sum(int(np.asarray(a).shape[0]) for _, a, _ in subs)
    vf = _valid(valid, n)
    return int(lib().oracle_merged_entry(ctypes.addressof(arr), len(subs),
                                         None if vf is None else _p(vf)))


def merge(X, subs, k: int, L: int, rounds: int, R: int, metric: str = "l2",
          k_rev: int = 0, threads: Optional[int] = None, valid=None, batches: int = 1):
    """All three stages: (pg_ids [N, R], deg, entry).  valid: as cross_query;
    batches: as refine."""
    X = _f32(X)
    arr, keep = _subs(subs)
    N = X.shape[0]
    vf = _valid(valid, N)
    oi = np.empty((N, R), np.uint32)
    deg = np.empty(N, np.uint32)
    ent = ctypes.c_uint64()
    rc = lib().oracle_merge(_p(X), X.shape[1], X.shape[1], METRICS[metric],
                            ctypes.addressof(arr), len(subs), k, L, rounds, k_rev, R,
                            _p(oi), _p(deg), ctypes.byref(ent), threads or default_threads(),
                            None if vf is None else _p(vf), int(batches))
    if rc:
        raise ValueError("oracle_merge failed")
    return oi, deg, ent.value


def bruteforce(X, Q, k: int, metric: str = "l2", exclude=None,
               threads: Optional[int] = None):
    """Exact FP64 k-NN of each query row: (ids uint32 [nq, k], dists float64)."""
    X, Q = _f32(X), _f32(Q)
    nq = Q.shape[0]
    ids = np.empty((nq, k), np.uint32)
    dd = np.empty((nq, k), np.float64)
    ex = None
    if exclude is not None:
        ex = np.ascontiguousarray(exclude, dtype=np.uint64)
    lib().oracle_bruteforce(_p(X), X.shape[0], X.shape[1], X.shape[1], METRICS[metric],
                            _p(Q), nq, Q.shape[1], k, None if ex is None else _p(ex),
                            _p(ids), _p(dd), threads or default_threads())
    return ids, dd


def bf16_from_f32(x: float) -> int:
    return int(lib().oracle_bf16_from_f32(float(x)))


def bf16_to_f32(b: int) -> float:
    return float(lib().oracle_bf16_to_f32(int(b)))


def fp8_from_f32(x: float) -> int:
    return int(lib().oracle_fp8_from_f32(float(x)))


def fp8_to_f32(c: int) -> float:
    return float(lib().oracle_fp8_to_f32(int(c)))


def quantize_bf16(X):
    """(codes uint16 [n, d], dequantised float32 [n, d])."""
    X = _f32(X)
    n, d = X.shape
    codes = np.empty((n, d), np.uint16)
    deq = np.empty((n, d), np.float32)
    lib().oracle_quantize_bf16(_p(X), n, d, d, _p(codes), _p(deq))
    return codes, deq


def quantize_fp8(X):
    """(codes uint8 [n, d], scales float32 [n], dequantised float32 [n, d])."""
    X = _f32(X)
    n, d = X.shape
    codes = np.empty((n, d), np.uint8)
    sc = np.empty(n, np.float32)
    deq = np.empty((n, d), np.float32)
    lib().oracle_quantize_fp8(_p(X), n, d, d, _p(codes), _p(sc), _p(deq))
    return codes, sc, deq


def knng_recall(X, ids, nodes, k: int, metric: str = "l2", threads=None) -> float:
    """Tie-aware k-NNG recall over `nodes` against FP64 brute force."""
    nodes = np.asarray(nodes, dtype=np.uint64)
    gt_ids, gt_d = bruteforce(X, np.asarray(X)[nodes.astype(np.int64)], k, metric,
                              exclude=nodes, threads=threads)
    return _tie_recall(X, X[nodes.astype(np.int64)], ids, gt_d[:, k - 1], k, metric)


def _tie_recall(X, Q, found, kth, k, metric) -> float:
    """Tie-aware recall: a found id counts when its FP64 distance, computed
    by the same loop as the brute force's (so equal ids give equal bits), is
    at most the true k-th distance."""
    X, Q = _f32(X), _f32(Q)
    f64 = lib().oracle_distance64
    m = METRICS[metric]
    hit = 0
    for i in range(found.shape[0]):
        q = Q[i]
        for v in found[i, :k]:
            if v == NONE:
                continue
            x = X[int(v)]
            hit += f64(_p(q), _p(x), X.shape[1], m) <= kth[i]
    return hit / float(found.shape[0] * k)


def search_recall(X, pg_ids, entry: int, Q, L: int, metric: str = "l2", at: int = 10,
                  threads=None) -> float:
    """Recall@at of Algorithm 1 on a merged graph from its entry, FP64 truth."""
    gt_ids, gt_d = bruteforce(X, Q, at, metric, threads=threads)
    found = np.full((Q.shape[0], at), NONE, np.uint32)
    for i in range(Q.shape[0]):
        ids, _, _, _ = knn_search(Q[i], X, pg_ids, entry, max(L, at), metric)
        found[i, :min(at, ids.size)] = ids[:at]
    return _tie_recall(X, Q, found, gt_d[:, at - 1], at, metric)
