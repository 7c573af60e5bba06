"""Python binding of libfgim, the MI355X (gfx950) FGIM merge library.

Thin ctypes marshalling over the C ABI in include/fgim.h: every step of the
merge runs in the library's HIP kernels.  Tensors must be CUDA (HIP) tensors
on the current device; torch provides device memory and the stream only.
Importing works without a GPU, but every call needs the built library
(python -m paper_2603_21710_amd.build) and raises if it is missing.
"""

from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfgim.so")
NONE = 0xFFFFFFFF

FGIM_L2, FGIM_IP, FGIM_COSINE = 0, 1, 2
FGIM_FP32, FGIM_BF16, FGIM_FP8_E4M3 = 0, 1, 2
FGIM_FLAG_NO_REPAIR = 1
FGIM_FLAG_NO_GRAPH_CAPTURE = 2
FGIM_FLAG_NO_MFMA_SCREEN = 4
FGIM_FLAG_MIN_BUFFERS = 8
METRICS = {"l2": FGIM_L2, "ip": FGIM_IP, "cos": FGIM_COSINE}
SELECT_RULES = {"rng": 0, "alpha": 1, "tau": 2}
PRECISIONS = {"fp32": FGIM_FP32, "bf16": FGIM_BF16, "fp8": FGIM_FP8_E4M3}

STATUS = {0: "FGIM_OK", 1: "FGIM_ERR_INVALID_ARG", 2: "FGIM_ERR_GRAPH",
          3: "FGIM_ERR_OUT_OF_MEMORY", 4: "FGIM_ERR_DEVICE", 5: "FGIM_ERR_UNSUPPORTED"}

EXPORTS = ["fgim_cross_query", "fgim_cross_query_noalloc", "fgim_refine", "fgim_repair", "fgim_prune",
           "fgim_merge", "fgim_search", "fgim_mips_to_l2", "fgim_hnsw_layers", "fgim_search_layers", "fgim_read_stream",
           "fgim_quantize", "fgim_min_beam_width", "fgim_release_scratch", "fgim_status_string",
           "fgim_last_error"]


class FgimError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Subindex(ctypes.Structure):
    _fields_ = [("row_offset", ctypes.c_uint64), ("n", ctypes.c_uint32),
                ("adj_stride", ctypes.c_uint32), ("adj", ctypes.c_void_p),
                ("entry", ctypes.c_uint32)]


class Dataset(ctypes.Structure):
    _fields_ = [("base", ctypes.c_void_p), ("n_total", ctypes.c_uint64),
                ("dim", ctypes.c_uint32), ("ld", ctypes.c_uint64), ("metric", ctypes.c_int),
                ("subs", ctypes.c_void_p), ("h", ctypes.c_uint32),
                ("base_lp", ctypes.c_void_p), ("base_lp_scale", ctypes.c_void_p),
                ("valid", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("L", ctypes.c_uint32), ("R", ctypes.c_uint32),
                ("rounds", ctypes.c_uint32), ("precision", ctypes.c_int),
                ("rerank", ctypes.c_uint32), ("k_rev", ctypes.c_uint32),
                ("autotune", ctypes.c_int), ("lanes_per_dist", ctypes.c_uint32),
                ("waves_per_cu", ctypes.c_uint32), ("visited_slots", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("select_rule", ctypes.c_uint32),
                ("select_param", ctypes.c_float), ("stream_batches", ctypes.c_uint32),
                ("update_chunks", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("ms_stage", ctypes.c_double * 3), ("ms_beam_kernel", ctypes.c_double),
                ("ndc", ctypes.c_uint64), ("expansions", ctypes.c_uint64),
                ("searches", ctypes.c_uint64), ("proposals", ctypes.c_uint64),
                ("repaired", ctypes.c_uint64), ("rechecked", ctypes.c_uint64),
                ("L_used", ctypes.c_uint32), ("lanes_per_dist", ctypes.c_uint32),
                ("waves_per_cu", ctypes.c_uint32), ("visited_slots", ctypes.c_uint32),
                ("ms_tune", ctypes.c_double), ("repair_batches", ctypes.c_uint64),
                ("repair_alone", ctypes.c_uint64), ("refine_attempts", ctypes.c_uint32)]

    def to_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "ms_stage"}
        d["ms_stage"] = list(self.ms_stage)
        return d


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libfgim.so; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2603_21710_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        for name, args in {
            "fgim_cross_query": [vp, vp, vp, vp, vp, vp],
            "fgim_cross_query_noalloc": [vp, vp, vp, vp, vp],
            "fgim_refine": [vp, vp, vp, vp, vp, vp, vp],
            "fgim_prune": [vp, vp, vp, vp, vp, vp, vp, vp],
            "fgim_merge": [vp, vp, vp, vp, vp, vp, vp],
            "fgim_search": [vp, u64, u32, u64, i32, vp, u32, u32, vp, u64, u64, u32, u32, vp,
                            vp, vp],
            "fgim_quantize": [vp, u64, u32, u64, i32, vp, vp, vp],
            "fgim_mips_to_l2": [vp, u64, u32, u64, vp, u64, vp, vp],
            "fgim_read_stream": [vp, u64, vp, vp],
            "fgim_hnsw_layers": [vp, u64, u32, u64, i32, vp, u32, u32, u32, vp, vp, vp, vp, vp],
            "fgim_search_layers": [vp, u64, u32, u64, i32, vp, u32, vp, vp, vp, u32, u32, u32, vp, u64,
                                   u64, u32, u32, vp, vp, vp],
            "fgim_repair": [vp, vp, u64, u32, vp, vp, vp],
        }.items():
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = args
        L.fgim_min_beam_width.restype = u32
        L.fgim_min_beam_width.argtypes = [u32, u32, u32]
        L.fgim_status_string.restype = ctypes.c_char_p
        L.fgim_status_string.argtypes = [i32]
        L.fgim_last_error.restype = ctypes.c_char_p
        L.fgim_last_error.argtypes = []
        L.fgim_release_scratch.restype = ctypes.c_int
        L.fgim_release_scratch.argtypes = []
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != 0:
        raise FgimError(rc, lib().fgim_last_error().decode(errors="replace"))


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _need_cuda(t: torch.Tensor, name: str, dtype=None) -> None:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype not in (dtype if isinstance(dtype, tuple) else (dtype,)):
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")


class Merge:
    """Inputs of one merge: base vectors X (float32 [N, d], CUDA) and h input
    graphs as (adj int32/uint32 [n_i, R_in] local ids, entry) in global-id
    order; sub-index i owns rows [off_i, off_i + n_i).  valid (uint8 [N],
    CUDA, optional): the ID mapping's validity flags (0 = dropped)."""

    def __init__(self, X: torch.Tensor, graphs: Sequence[Tuple[torch.Tensor, int]],
                 metric: str = "l2", lowp: Optional[torch.Tensor] = None,
                 lowp_scale: Optional[torch.Tensor] = None, valid: Optional[torch.Tensor] = None):
        _need_cuda(X, "X", torch.float32)
        if valid is not None:
            _need_cuda(valid, "valid", torch.uint8)
            if valid.shape != (X.shape[0],) or not valid.is_contiguous():
                raise ValueError(f"valid must be a contiguous uint8 tensor of {X.shape[0]} flags")
        self.valid = valid
        if X.dim() != 2 or X.stride(1) != 1:
            raise ValueError("X must be a row-major 2-D tensor")
        self.X = X
        self.metric = metric
        self.graphs = []
        subs = (Subindex * len(graphs))()
        off = 0
        for i, (adj, entry) in enumerate(graphs):
            _need_cuda(adj, f"graph {i} adjacency", (torch.int32,))
            adj = adj.contiguous()
            self.graphs.append(adj)
            subs[i] = Subindex(off, adj.shape[0], adj.shape[1], adj.data_ptr(), int(entry))
            off += adj.shape[0]
        if off != X.shape[0]:
            raise ValueError(f"graphs cover {off} rows, X has {X.shape[0]}")
        self._subs = subs
        self.lowp, self.lowp_scale = lowp, lowp_scale
        self.data = Dataset(X.data_ptr(), X.shape[0], X.shape[1], X.stride(0), METRICS[metric],
                            ctypes.addressof(subs), len(graphs), _ptr(lowp), _ptr(lowp_scale),
                            _ptr(valid))

    @property
    def n(self) -> int:
        return self.X.shape[0]


def params(k: int, L: int, R: int = 0, rounds: int = 0, precision: str = "fp32",
           rerank: int = 0, k_rev: int = 0, autotune: bool = False, lanes_per_dist: int = 0,
           waves_per_cu: int = 0, visited_slots: int = 0, flags: int = 0, select_rule: str = "rng",
           select_param: float = 0.0, stream_batches: int = 0, update_chunks: int = 0) -> Params:
    return Params(k, L, R, rounds, PRECISIONS[precision], rerank, k_rev, int(autotune),
                  lanes_per_dist, waves_per_cu, visited_slots, flags, SELECT_RULES[select_rule],
                  float(select_param), stream_batches, update_chunks)


def cross_query(m: Merge, p: Params, stats: bool = False):
    """Stage 1: (ids int32 [N, k] (uint32 bit patterns), dist float32, stats|None)."""
    ids = torch.empty((m.n, p.k), dtype=torch.int32, device=m.X.device)
    dist = torch.empty((m.n, p.k), dtype=torch.float32, device=m.X.device)
    st = Stats() if stats else None
    _check(lib().fgim_cross_query(ctypes.byref(m.data), ctypes.byref(p), ids.data_ptr(),
                                  dist.data_ptr(), ctypes.byref(st) if st else None, _stream()))
    return ids, dist, (st.to_dict() if st else None)


def cross_query_noalloc(m: Merge, p: Params, ids: torch.Tensor, dist: torch.Tensor) -> None:
    """Stage 1 into caller-given (ids int32 [N, k], dist float32 [N, k]),
    through the entry point that allocates no device memory (autotune off;
    the low-precision forms need m's lowp copy)."""
    _need_cuda(ids, "ids", torch.int32)
    _need_cuda(dist, "dist", torch.float32)
    if ids.shape != (m.n, p.k) or dist.shape != (m.n, p.k) or not ids.is_contiguous() \
            or not dist.is_contiguous():
        raise ValueError(f"ids and dist must be contiguous [{m.n}, {p.k}] tensors")
    _check(lib().fgim_cross_query_noalloc(ctypes.byref(m.data), ctypes.byref(p), ids.data_ptr(),
                                          dist.data_ptr(), _stream()))


def refine(m: Merge, p: Params, ids: torch.Tensor, dist: torch.Tensor, stats: bool = False):
    """Stage 2 in place on (ids, dist); returns (indegree int32 [N], stats|None)."""
    _need_cuda(ids, "ids", torch.int32)
    _need_cuda(dist, "dist", torch.float32)
    T = torch.empty(m.n, dtype=torch.int32, device=m.X.device)
    st = Stats() if stats else None
    _check(lib().fgim_refine(ctypes.byref(m.data), ctypes.byref(p), ids.data_ptr(),
                             dist.data_ptr(), T.data_ptr(), ctypes.byref(st) if st else None,
                             _stream()))
    return T, (st.to_dict() if st else None)


def repair(ids: torch.Tensor, dist: torch.Tensor):
    """Algorithm 4 alone, in place on (ids, dist) [N, k]; returns (indegree
    int32 [N], number of repaired vertices)."""
    _need_cuda(ids, "ids", torch.int32)
    _need_cuda(dist, "dist", torch.float32)
    if ids.dim() != 2 or ids.shape != dist.shape or not ids.is_contiguous() or not dist.is_contiguous():
        raise ValueError("ids and dist must be contiguous [N, k] tensors of one shape")
    T = torch.empty(ids.shape[0], dtype=torch.int32, device=ids.device)
    n = ctypes.c_uint64()
    _check(lib().fgim_repair(ids.data_ptr(), dist.data_ptr(), ids.shape[0], ids.shape[1], T.data_ptr(),
                             ctypes.byref(n), _stream()))
    return T, n.value


def release_scratch() -> None:
    """Free the current device's scratch arena (after its last call has
    finished on the device); the next call starts a new one."""
    _check(lib().fgim_release_scratch())


def prune(m: Merge, p: Params, ids: torch.Tensor, dist: torch.Tensor, T: torch.Tensor):
    """Stage 3: (pg_ids int32 [N, R], pg_deg int32 [N])."""
    pg = torch.empty((m.n, p.R), dtype=torch.int32, device=m.X.device)
    deg = torch.empty(m.n, dtype=torch.int32, device=m.X.device)
    _check(lib().fgim_prune(ctypes.byref(m.data), ctypes.byref(p), ids.data_ptr(),
                            dist.data_ptr(), T.data_ptr(), pg.data_ptr(), deg.data_ptr(),
                            _stream()))
    return pg, deg


def merge(m: Merge, p: Params, stats: bool = False):
    """All three stages: (pg_ids [N, R], pg_deg [N], entry, stats|None)."""
    pg = torch.empty((m.n, p.R), dtype=torch.int32, device=m.X.device)
    deg = torch.empty(m.n, dtype=torch.int32, device=m.X.device)
    entry = ctypes.c_uint32()
    st = Stats() if stats else None
    _check(lib().fgim_merge(ctypes.byref(m.data), ctypes.byref(p), pg.data_ptr(),
                            deg.data_ptr(), ctypes.byref(entry),
                            ctypes.byref(st) if st else None, _stream()))
    return pg, deg, entry.value, (st.to_dict() if st else None)


def search(X: torch.Tensor, adj: torch.Tensor, entry: int, Q: torch.Tensor, L: int, topk: int,
           metric: str = "l2"):
    """Algorithm 1 for every row of Q on graph adj: (ids [nq, topk], dist)."""
    _need_cuda(X, "X", torch.float32)
    _need_cuda(Q, "Q", torch.float32)
    _need_cuda(adj, "adj", torch.int32)
    adj = adj.contiguous()
    ids = torch.empty((Q.shape[0], topk), dtype=torch.int32, device=X.device)
    dist = torch.empty((Q.shape[0], topk), dtype=torch.float32, device=X.device)
    _check(lib().fgim_search(X.data_ptr(), X.shape[0], X.shape[1], X.stride(0), METRICS[metric],
                             adj.data_ptr(), adj.shape[1], int(entry), Q.data_ptr(), Q.shape[0],
                             Q.stride(0), L, topk, ids.data_ptr(), dist.data_ptr(), _stream()))
    return ids, dist


def quantize(X: torch.Tensor, precision: str):
    """Low-precision copy: BF16 -> (int16 codes [N, d], None);
    FP8 -> (uint8 codes [N, d], float32 scales [N])."""
    _need_cuda(X, "X", torch.float32)
    n, d = X.shape
    if precision == "bf16":
        codes = torch.empty((n, d), dtype=torch.int16, device=X.device)
        scales = None
    elif precision == "fp8":
        codes = torch.empty((n, d), dtype=torch.uint8, device=X.device)
        scales = torch.empty(n, dtype=torch.float32, device=X.device)
    else:
        raise ValueError(precision)
    _check(lib().fgim_quantize(X.data_ptr(), n, d, X.stride(0), PRECISIONS[precision],
                               codes.data_ptr(), _ptr(scales), _stream()))
    return codes, scales


def read_stream(buf: torch.Tensor) -> torch.Tensor:
    """Reads every byte of a contiguous device tensor once (a measurement
    aid: its duration gives the read-stream bandwidth); returns the XOR of
    its 32-bit words as an int32 tensor [1]."""
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous device tensor")
    out = torch.empty(1, dtype=torch.int32, device=buf.device)
    _check(lib().fgim_read_stream(buf.data_ptr(), buf.numel() * buf.element_size(), out.data_ptr(), _stream()))
    return out


def mips_to_l2(X: torch.Tensor):
    """MIPS -> L2 transform: (rows float32 [n, d + 4] CUDA, M float32 [1] CUDA)."""
    _need_cuda(X, "X", torch.float32)
    n, d = X.shape
    out = torch.empty((n, d + 4), dtype=torch.float32, device=X.device)
    M = torch.empty(1, dtype=torch.float32, device=X.device)
    _check(lib().fgim_mips_to_l2(X.data_ptr(), n, d, X.stride(0), out.data_ptr(), d + 4, M.data_ptr(),
                                 _stream()))
    return out, M


def hnsw_layers(X: torch.Tensor, levels: torch.Tensor, M: int, ef: int, metric: str = "l2"):
    """Upper layers over the base rows X for levels (uint8 [N], CUDA):
    (layer_ids int32 [rows], layer_adj int32 [rows, M], counts (list), top)."""
    _need_cuda(X, "X", torch.float32)
    _need_cuda(levels, "levels", torch.uint8)
    lv = levels.contiguous()
    max_level = int(lv.max().item()) if lv.numel() else 0
    counts = [int((lv >= l).sum().item()) for l in range(1, max_level + 1)]
    rows = sum(counts)
    ids = torch.empty(max(rows, 1), dtype=torch.int32, device=X.device)
    adj = torch.empty((max(rows, 1), M), dtype=torch.int32, device=X.device)
    cnt = (ctypes.c_uint64 * max(max_level, 1))(*counts)
    top = ctypes.c_uint32()
    _check(lib().fgim_hnsw_layers(X.data_ptr(), X.shape[0], X.shape[1], X.stride(0), METRICS[metric],
                                  lv.data_ptr(), max_level, M, ef, cnt, ids.data_ptr(), adj.data_ptr(),
                                  ctypes.byref(top), _stream()))
    return ids[:rows], adj[:rows], counts, top.value


def search_layers(X: torch.Tensor, base_adj: torch.Tensor, layers, M: int, Q: torch.Tensor, L: int,
                  topk: int, metric: str = "l2"):
    """Hierarchical search (descent through the layers, then Algorithm 1 on
    the base graph): (ids [nq, topk], dist)."""
    _need_cuda(X, "X", torch.float32)
    _need_cuda(Q, "Q", torch.float32)
    _need_cuda(base_adj, "base_adj", torch.int32)
    lids, ladj, counts, top = layers
    base_adj = base_adj.contiguous()
    cnt = (ctypes.c_uint64 * max(len(counts), 1))(*counts)
    ids = torch.empty((Q.shape[0], topk), dtype=torch.int32, device=X.device)
    dist = torch.empty((Q.shape[0], topk), dtype=torch.float32, device=X.device)
    _check(lib().fgim_search_layers(X.data_ptr(), X.shape[0], X.shape[1], X.stride(0), METRICS[metric],
                                    base_adj.data_ptr(), base_adj.shape[1], lids.data_ptr(),
                                    ladj.data_ptr(), cnt, len(counts), M, top, Q.data_ptr(), Q.shape[0],
                                    Q.stride(0), L, topk, ids.data_ptr(), dist.data_ptr(), _stream()))
    return ids, dist


def min_beam_width(k: int, min_local: int, h: int) -> int:
    return int(lib().fgim_min_beam_width(k, min_local, h))


def as_uint32(t: torch.Tensor):
    """int32 id tensor -> numpy uint32 (FGIM_NONE = 0xFFFFFFFF)."""
    return t.cpu().numpy().view("uint32")
