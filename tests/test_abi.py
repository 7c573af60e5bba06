"""Host-side checks of the C ABI: the library loads without a GPU, exports
every entry point of include/fgim.h, and rejects bad arguments before it
touches the device."""
import ctypes
import os
import re

import pytest

import paper_2603_21710_amd as fg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fgim.h")).read()
    return sorted(set(re.findall(r"^\S.*?\b(fgim_[a-z0-9_]+)\(", src, re.M)))


def test_header_and_binding_agree():
    assert sorted(fg.EXPORTS) == _declared()


def _struct_fields(name):
    src = open(os.path.join(ROOT, "include", "fgim.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct \{([^{}]*)\} " + name + ";", src).group(1)
    return [re.sub(r"\[.*\]", "", d.split()[-1]).lstrip("*") for d in body.split(";") if d.strip()]


@pytest.mark.parametrize("name,cls", [("fgim_params", "Params"), ("fgim_dataset", "Dataset"),
                                      ("fgim_stats", "Stats"), ("fgim_subindex", "Subindex")])
def test_binding_structs_follow_the_header(name, cls):
    assert [f for f, _ in getattr(fg, cls)._fields_] == _struct_fields(name)


def test_library_exports_every_declared_symbol():
    L = fg.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_min_beam_width():
    assert fg.min_beam_width(16, 0, 2) == 16
    assert fg.min_beam_width(24, 3, 8) == 3
    assert fg.min_beam_width(32, 40, 4) == 1
    assert fg.min_beam_width(32, 0, 1) == 0


def _dataset(n=100, dim=32, ld=None, subs=None, metric=0, base=0x10000):
    subs = subs if subs is not None else [(0, 60, 8, 0x20000, 0), (60, 40, 8, 0x30000, 3)]
    arr = (fg.Subindex * len(subs))(*[fg.Subindex(*s) for s in subs])
    d = fg.Dataset(base, n, dim, ld or dim, metric, ctypes.addressof(arr), len(subs), None, None, None)
    return d, arr


@pytest.mark.parametrize("kw,pk", [
    (dict(dim=30), {}),
    (dict(dim=8192), {}),
    (dict(ld=20), {}),
    (dict(base=0), {}),
    (dict(base=0x10004), {}),
    (dict(metric=7), {}),
    (dict(subs=[(0, 60, 8, 0x20000, 0), (61, 39, 8, 0x30000, 0)]), {}),
    (dict(subs=[(0, 60, 8, 0x20000, 60), (60, 40, 8, 0x30000, 0)]), {}),
    (dict(subs=[(0, 60, 0, 0x20000, 0), (60, 40, 8, 0x30000, 0)]), {}),
    (dict(subs=[(0, 60, 8, 0, 0), (60, 40, 8, 0x30000, 0)]), {}),
    (dict(subs=[(0, 60, 8, 0x20000, 0)]), {}),
    ({}, dict(k=0)),
    ({}, dict(L=0)),
    ({}, dict(k=200)),
    ({}, dict(L=300)),
    ({}, dict(lanes_per_dist=3)),
    ({}, dict(lanes_per_dist=16)),
    ({}, dict(visited_slots=1000)),
])
def test_bad_arguments_rejected_on_host(kw, pk):
    d, keep = _dataset(**kw)
    p = fg.params(**{**dict(k=8, L=16), **pk})
    rc = fg.lib().fgim_cross_query(ctypes.byref(d), ctypes.byref(p), 0x40000, 0x50000, None, None)
    assert rc in (1, 5), fg.lib().fgim_last_error()
    assert fg.lib().fgim_last_error()


def test_null_outputs_rejected():
    d, keep = _dataset()
    p = fg.params(k=8, L=16)
    assert fg.lib().fgim_cross_query(ctypes.byref(d), ctypes.byref(p), None, 0x50000, None, None) == 1
    assert fg.lib().fgim_cross_query(None, ctypes.byref(p), 0x40000, 0x50000, None, None) == 1


@pytest.mark.parametrize("ids,dist,n,k", [
    (None, 0x50000, 100, 8),
    (0x40000, None, 100, 8),
    (0x40000, 0x50000, 0, 8),
    (0x40000, 0x50000, 100, 0),
    (0x40000, 0x50000, 100, 200),
])
def test_repair_bad_arguments_rejected_on_host(ids, dist, n, k):
    assert fg.lib().fgim_repair(ids, dist, n, k, None, None, None) == 1
    assert fg.lib().fgim_last_error()


@pytest.mark.parametrize("pk,lowp", [(dict(autotune=True), None), (dict(precision="bf16"), None),
                                     (dict(precision="fp8"), 0x60000)])
def test_noalloc_limits_rejected_on_host(pk, lowp):
    # autotune needs trial-launch memory; the low-precision forms need the
    # caller's copy (and FP8 its scales): rejected before any device call
    d, keep = _dataset()
    d.base_lp = lowp
    p = fg.params(**{**dict(k=8, L=16), **pk})
    rc = fg.lib().fgim_cross_query_noalloc(ctypes.byref(d), ctypes.byref(p), 0x40000, 0x50000, None)
    assert rc == 1, fg.lib().fgim_last_error()
    assert b"noalloc" in fg.lib().fgim_last_error()


@pytest.mark.parametrize("metric,rule,param", [(1, "alpha", 1.2), (1, "tau", 0.1), (0, "alpha", 0.9),
                                               (0, "tau", -1.0), (2, "alpha", float("nan"))])
def test_selection_rule_arguments_rejected_on_host(metric, rule, param):
    d, keep = _dataset(metric=metric)
    p = fg.params(k=8, L=16, R=8, select_rule=rule, select_param=param)
    rc = fg.lib().fgim_prune(ctypes.byref(d), ctypes.byref(p), 0x40000, 0x50000, 0x60000, 0x70000, 0x80000, None)
    assert rc == 1, fg.lib().fgim_last_error()


@pytest.mark.parametrize("args", [
    (0x10000, 100, 32, 32, 0x20000, 35, 0x30000),   # ld_out < dim + 4
    (0x10000, 100, 32, 32, 0x20004, 36, 0x30000),   # misaligned output
    (0x10000, 100, 32, 32, None, 36, 0x30000),      # no output
    (0x10000, 100, 32, 32, 0x10000, 36, 0x30000),   # output overlaps the input
    (0x10000, 100, 30, 32, 0x20000, 36, 0x30000),   # dim not a multiple of 4
])
def test_mips_to_l2_bad_arguments_rejected_on_host(args):
    rc = fg.lib().fgim_mips_to_l2(*args, None)
    assert rc in (1, 5), fg.lib().fgim_last_error()


def test_stream_batches_limit_rejected_on_host():
    d, keep = _dataset()
    p = fg.params(k=8, L=16, rounds=1, stream_batches=5000)
    rc = fg.lib().fgim_refine(ctypes.byref(d), ctypes.byref(p), 0x40000, 0x50000, None, None, None)
    assert rc == 1 and b"stream_batches" in fg.lib().fgim_last_error()


@pytest.mark.parametrize("data,nbytes,out", [(0, 64, 0x50000), (0x40000, 64, 0), (0x40004, 64, 0x50000),
                                             (0x40000, 60, 0x50000), (0, 0, 0)])
def test_read_stream_bad_arguments_rejected_on_host(data, nbytes, out):
    assert fg.lib().fgim_read_stream(data, nbytes, out, None) == 1
    assert fg.lib().fgim_last_error()


def test_update_chunks_limit_rejected_on_host():
    d, keep = _dataset()
    p = fg.params(k=8, L=16, rounds=1, update_chunks=5000)
    rc = fg.lib().fgim_refine(ctypes.byref(d), ctypes.byref(p), 0x40000, 0x50000, None, None, None)
    assert rc == 1 and b"update_chunks" in fg.lib().fgim_last_error()
