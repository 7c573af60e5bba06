"""Shared test helpers: golden loading and 1-D point embeddings."""
import json
import os

import numpy as np

NONE = 0xFFFFFFFF
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def line_points(xs, dim=4):
    """1-D coordinates embedded as (x, 0, 0, 0): squared L2 = (x - y)^2 exactly."""
    X = np.zeros((len(xs), dim), np.float32)
    X[:, 0] = np.asarray(xs, np.float32)
    return X


def pad_ids(rows, k):
    out = np.full((len(rows), k), NONE, np.uint32)
    for i, r in enumerate(rows):
        for j, v in enumerate(r):
            if v is not None:
                out[i, j] = v
    return out


def pad_dists(rows, k):
    out = np.full((len(rows), k), np.inf, np.float32)
    for i, r in enumerate(rows):
        for j, v in enumerate(r):
            if v is not None:
                out[i, j] = v
    return out


def pad_adj(rows, stride=None):
    stride = stride or max(1, max(len(r) for r in rows))
    return pad_ids(rows, stride)
