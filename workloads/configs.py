"""Workload configurations for the merge of h proximity graphs.

Each configuration names the sub-index sizes, the vector distribution, the
distance, the input-graph degree R_in and the merge parameters: k (degree of
the k-NNG built by stages 1-2), L (beam width of the cross-queries), rounds
(I_max, refinement iterations) and R (degree of the pruned output graph).

The shapes stand in for the paper's evaluation datasets (Sift, Deep, Gist,
GloVe, MSong, Crawl and an industrial 768-d embedding set, Section 5.1,
Table "The properties of the datasets"), none of which is available here.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class WorkloadConfig:
    name: str
    sizes: Tuple[int, ...]          # n_i of each sub-index, in global-id order
    dim: int
    metric: str                     # "l2" | "ip" | "cos"
    dist: str                       # generator kind, see synth.make_vectors
    dist_params: Tuple[Tuple[str, float], ...]
    r_in: int                       # degree bound of each input PG
    k: int                          # k-NNG degree (stages 1-2)
    L: int                          # cross-query beam width
    rounds: int                     # refinement iterations I_max
    R: int                          # output PG degree (stage 3)
    n_queries: int
    precision: str = "fp32"         # "fp32" | "bf16" | "fp8"
    seed: int = 0                   # data seed; queries use seed + 1000

    @property
    def n_total(self) -> int:
        return int(sum(self.sizes))

    @property
    def h(self) -> int:
        return len(self.sizes)

    def params(self) -> Dict[str, float]:
        return dict(self.dist_params)

    def offsets(self) -> List[int]:
        off, acc = [], 0
        for n in self.sizes:
            off.append(acc)
            acc += n
        return off

    def scaled(self, sizes: Tuple[int, ...], name: Optional[str] = None,
               n_queries: Optional[int] = None) -> "WorkloadConfig":
        """Same distribution and merge parameters at other sub-index sizes."""
        return dataclasses.replace(
            self, sizes=tuple(int(s) for s in sizes),
            name=name or f"{self.name}@{'+'.join(str(s) for s in sizes)}",
            n_queries=self.n_queries if n_queries is None else n_queries)


def _fresh_sizes(count: int, lo: int, hi: int, seed: int) -> Tuple[int, ...]:
    """Log-uniform sub-index sizes in [lo, hi], rounded to multiples of 1000."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    return tuple(int(round(math.exp(x) / 1000.0)) * 1000 for x in u)


CONFIGS: Dict[str, WorkloadConfig] = {
    # Plain FP32 merge of 2 PGs x 5,000 vectors, d=32, 16-cluster Gaussian
    # mixture with centres ~ N(0, 4I) and unit within-cluster spread, L2.
    "cfg1": WorkloadConfig(
        name="cfg1", sizes=(5000, 5000), dim=32, metric="l2", dist="gmm",
        dist_params=(("clusters", 16), ("centre_std", 2.0), ("sigma", 1.0)),
        r_in=32, k=16, L=32, rounds=2, R=32, n_queries=200, seed=1001),
    # Same sizes with centres ~ N(0, I): overlapping clusters, so that the
    # input graphs are navigable from their medoid (quality supplement).
    "cfg1ov": WorkloadConfig(
        name="cfg1ov", sizes=(5000, 5000), dim=32, metric="l2", dist="gmm",
        dist_params=(("clusters", 16), ("centre_std", 1.0), ("sigma", 1.0)),
        r_in=32, k=16, L=32, rounds=2, R=32, n_queries=200, seed=1011),
    # SIFT-shaped: 2 x 500,000, d=128, 64 clusters, integer values in 0..255.
    "cfg2": WorkloadConfig(
        name="cfg2", sizes=(500_000, 500_000), dim=128, metric="l2",
        dist="sift", dist_params=(("clusters", 64), ("centre_base", 10.0),
                                  ("centre_scale", 20.0), ("sigma", 20.0)),
        r_in=32, k=32, L=64, rounds=4, R=32, n_queries=10_000, seed=1002),
    # Batching form: 8 uneven sub-indexes (2M), d=96, unit-normalised
    # 256-cluster mixture, inner product.
    "cfg3": WorkloadConfig(
        name="cfg3",
        sizes=(50_000, 100_000, 150_000, 200_000, 250_000, 300_000,
               450_000, 500_000),
        dim=96, metric="ip", dist="gmm_unit",
        dist_params=(("clusters", 256), ("centre_std", 1.0), ("sigma", 1.0)),
        r_in=24, k=24, L=48, rounds=3, R=32, n_queries=10_000, seed=1003),
    # Same with centres ~ N(0, 0.25 I): overlapping directions, so that the
    # input graphs are navigable from their medoid (quality supplement; the
    # literal recipe reaches under 1 % of each graph).
    "cfg3ov": WorkloadConfig(
        name="cfg3ov",
        sizes=(50_000, 100_000, 150_000, 200_000, 250_000, 300_000,
               450_000, 500_000),
        dim=96, metric="ip", dist="gmm_unit",
        dist_params=(("clusters", 256), ("centre_std", 0.5), ("sigma", 1.0)),
        r_in=24, k=24, L=48, rounds=3, R=32, n_queries=10_000, seed=1013),
    # Precision form: 2 x 500,000, d=768, von Mises-Fisher mixture
    # (1,024 directions, kappa=50), cosine on unit vectors.
    "cfg4": WorkloadConfig(
        name="cfg4", sizes=(500_000, 500_000), dim=768, metric="cos",
        dist="vmf", dist_params=(("clusters", 1024), ("kappa", 50.0)),
        r_in=48, k=32, L=64, rounds=4, R=48, n_queries=10_000,
        precision="bf16", seed=1004),
    # Batching + precision at scale: 4 x 2.5M plus 16 fresh sub-indexes of
    # 10k..200k vectors, d=128, 1,024-cluster Gaussian mixture, L2.
    "cfg5": WorkloadConfig(
        name="cfg5",
        sizes=(2_500_000,) * 4 + _fresh_sizes(16, 10_000, 200_000, 3005),
        dim=128, metric="l2", dist="gmm",
        dist_params=(("clusters", 1024), ("centre_std", 1.0), ("sigma", 1.0)),
        r_in=48, k=32, L=96, rounds=4, R=48, n_queries=10_000,
        precision="bf16", seed=1005),
    # Same sizes with centres ~ N(0, 0.25 I): overlapping clusters, so that
    # the input graphs are navigable from their medoid (quality supplement;
    # the literal recipe's graphs are islands of one cluster each).
    "cfg5ov": WorkloadConfig(
        name="cfg5ov",
        sizes=(2_500_000,) * 4 + _fresh_sizes(16, 10_000, 200_000, 3005),
        dim=128, metric="l2", dist="gmm",
        dist_params=(("clusters", 1024), ("centre_std", 0.5), ("sigma", 1.0)),
        r_in=48, k=32, L=96, rounds=4, R=48, n_queries=10_000,
        precision="bf16", seed=1015),
}


def get_config(name: str) -> WorkloadConfig:
    try:
        return CONFIGS[name]
    except KeyError:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(CONFIGS)}")
