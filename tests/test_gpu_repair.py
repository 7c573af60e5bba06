"""GPU parity of indegree repair alone (Algorithm 4, fgim_repair) against
the oracle on lists built to stress the batched pass: many zero-indegree
vertices whose closest neighbours are a few shared hubs (so steps of one
batch collide on lists and evicted entries, and hub lists run out of
replaceable entries, forcing further attempts), rows with free slots, and
both register widths (k <= 64 and k > 64)."""
import numpy as np
import pytest
import torch

import oracle
from helpers import NONE

pytestmark = pytest.mark.gpu

fg = pytest.importorskip("paper_2603_21710_amd")


def hub_lists(N, k, hubs, seed, fill=1.0, skew=1.0):
    """Row u: up to k distinct ids drawn from the first `hubs` vertices
    (hubs = 0: from all vertices with probability ~ (id + 10)^-skew), never
    u, sorted by random distinct distances; a share 1 - fill of the rows is
    cut short (free slots)."""
    rng = np.random.default_rng(seed)
    ids = np.full((N, k), NONE, np.uint32)
    dist = np.full((N, k), np.inf, np.float32)
    if not hubs:
        w = (np.arange(N) + 10.0) ** -skew
        draws = rng.choice(N, size=(N, 8 * k), p=w / w.sum())
    for u in range(N):
        if hubs:
            cand = rng.choice(hubs, size=min(hubs, k + 1), replace=False)
        else:
            _, first = np.unique(draws[u], return_index=True)
            cand = draws[u][np.sort(first)]
        cand = cand[cand != u][:k]
        m = k if rng.random() < fill else int(rng.integers(1, k))
        cand = cand[:m]
        d = np.sort(rng.random(m).astype(np.float32))
        ids[u, :m] = cand
        dist[u, :m] = d
    return ids, dist


CASES = [
    ("hubs", 4000, 8, 50, 1.0, 1.0),
    ("hubs_free_slots", 4000, 8, 40, 0.7, 1.0),
    ("few_hubs", 3000, 16, 20, 1.0, 1.0),
    ("wide", 1500, 100, 300, 0.9, 1.0),
    ("skewed", 20000, 16, 0, 1.0, 1.0),
    ("skewed_wide", 6000, 72, 0, 0.95, 1.5),
]


@pytest.mark.parametrize("name,N,k,hubs,fill,skew", CASES, ids=[c[0] for c in CASES])
def test_repair_matches_oracle(name, N, k, hubs, fill, skew):
    ids, dist = hub_lists(N, k, hubs, seed=N + k + hubs, fill=fill, skew=skew)
    oi, od, _, oT, on = oracle.repair(ids, dist)
    print(f"case {name}: N={N} k={k} zero-indegree before={int((oT == 0).sum()) + on} repaired={on}",
          flush=True)
    gi = torch.from_numpy(ids.view(np.int32)).cuda()
    gd = torch.from_numpy(dist).cuda()
    T, n = fg.repair(gi, gd)
    assert n == on
    got = gi.cpu().numpy().view(np.uint32)
    bad = np.argwhere(got != oi)
    assert bad.size == 0, f"{len(bad)} id mismatches, first {bad[:3].tolist()}"
    assert (gd.cpu().numpy().view(np.uint32) == od.view(np.uint32)).all()
    assert (T.cpu().numpy().view(np.uint32) == oT).all()


def test_repair_rejects_out_of_range_ids():
    ids, dist = hub_lists(500, 8, 50, seed=3)
    ids[7, 2] = 500
    gi = torch.from_numpy(ids.view(np.int32)).cuda()
    gd = torch.from_numpy(dist).cuda()
    before = gi.clone()
    with pytest.raises(fg.FgimError) as ei:
        fg.repair(gi, gd)
    assert ei.value.name == "FGIM_ERR_GRAPH"
    assert torch.equal(gi, before)
