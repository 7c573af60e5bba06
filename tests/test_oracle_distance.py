"""Pins of the oracle's canonical FP32 distance (Section 2.1 delta; the
fixed FP32 summation order is the reading used for bit-exact parity)."""
import numpy as np
import pytest

import oracle

U = 2.0 ** -24


def gamma(n):
    return n * U / (1 - n * U)


@pytest.mark.parametrize("d", [1, 3, 4, 32, 96, 100, 128, 768])
def test_l2_within_higham_bound_of_fp64(d):
    # Each coordinate difference is rounded once and the sum of squares is
    # formed with at most 4 + log2(d/4) + 1 roundings along any path, so the
    # error is below gamma_{d+2} * sum (a-b)^2 (Higham, Thm 3.1 / Sec 4.2).
    rng = np.random.default_rng(d)
    for _ in range(20):
        a = rng.normal(size=d).astype(np.float32)
        b = rng.normal(size=d).astype(np.float32)
        ref = float(np.sum((a.astype(np.float64) - b.astype(np.float64)) ** 2))
        got = oracle.distance(a, b, "l2")
        assert abs(got - ref) <= gamma(d + 2) * ref + 1e-30


@pytest.mark.parametrize("d", [4, 32, 128])
def test_ip_within_bound(d):
    rng = np.random.default_rng(100 + d)
    for _ in range(20):
        a = rng.normal(size=d).astype(np.float32)
        b = rng.normal(size=d).astype(np.float32)
        exact = float(np.dot(a.astype(np.float64), b.astype(np.float64)))
        bound = gamma(d) * float(np.sum(np.abs(a.astype(np.float64) * b)))
        assert abs(oracle.distance(a, b, "ip") - (-exact)) <= bound
        assert abs(oracle.distance(a, b, "cos") - (1.0 - exact)) <= bound + U


def test_exact_on_integer_data():
    # SIFT-shaped rows: integers 0..255, d=128.  Every partial sum is an
    # integer below 2^24 (255^2 * 128 = 8,323,200), so any summation order
    # gives the exact value.
    rng = np.random.default_rng(7)
    for _ in range(50):
        a = rng.integers(0, 256, 128)
        b = rng.integers(0, 256, 128)
        exact = int(((a - b) ** 2).sum())
        assert oracle.distance(a.astype(np.float32), b.astype(np.float32), "l2") == exact
        ip = int((a * b).sum())
        if ip < 2 ** 24:
            assert oracle.distance(a.astype(np.float32), b.astype(np.float32), "ip") == -ip


def test_symmetry_bitwise():
    rng = np.random.default_rng(3)
    for d in (5, 32, 96, 768):
        for _ in range(20):
            a = rng.normal(size=d).astype(np.float32)
            b = rng.normal(size=d).astype(np.float32)
            for m in ("l2", "ip", "cos"):
                x = np.float32(oracle.distance(a, b, m))
                y = np.float32(oracle.distance(b, a, m))
                assert x.tobytes() == y.tobytes()


def test_stride_tree_order():
    # d=16: four chunks whose sums are 2^24, 1, -2^24, 1 (inner product with
    # b = ones).  The stride tree adds (s0 + s2) + (s1 + s3) = 0 + 2 = 2, so
    # delta = -2.  Left-to-right summation would give ((2^24+1)-2^24)+1 = 1
    # (2^24+1 rounds to 2^24), and so would neighbour pairing.
    a = np.zeros(16, np.float32)
    a[0] = 2.0 ** 24
    a[4] = 1.0
    a[8] = -(2.0 ** 24)
    a[12] = 1.0
    assert oracle.distance(a, np.ones(16, np.float32), "ip") == -2.0


def test_chunk_is_fma_chain():
    # Within a chunk each product is added with one rounding (fused
    # multiply-add).  With e = 1 + 2^-12: e*e = 1 + 2^-11 + 2^-24 rounds to
    # 1 + 2^-11 in the first fma; the second fma adds -e*e exactly and
    # leaves -2^-24, so delta_ip = 2^-24.  Separate rounding of the product
    # would cancel to 0.
    e = 1.0 + 2.0 ** -12
    a = np.array([e, -e, 0.0, 0.0], np.float32)
    b = np.array([e, e, 0.0, 0.0], np.float32)
    assert oracle.distance(a, b, "ip") == np.float32(2.0 ** -24)


def test_zero_padding_invariance():
    rng = np.random.default_rng(11)
    a = rng.normal(size=5).astype(np.float32)
    b = rng.normal(size=5).astype(np.float32)
    a8 = np.concatenate([a, np.zeros(3, np.float32)])
    b8 = np.concatenate([b, np.zeros(3, np.float32)])
    for m in ("l2", "ip", "cos"):
        assert oracle.distance(a, b, m) == oracle.distance(a8, b8, m)


def test_small_values_and_negative_zero():
    a = np.array([1, 2, 3, 4], np.float32)
    assert oracle.distance(a, np.zeros(4, np.float32), "l2") == 30.0
    assert oracle.distance(a, a, "ip") == -30.0
    e0 = np.array([1, 0, 0, 0], np.float32)
    e1 = np.array([0, 1, 0, 0], np.float32)
    v = np.float32(oracle.distance(e0, e1, "ip"))
    assert v == 0.0 and not np.signbit(v)
    assert oracle.distance(e0, e0, "cos") == 0.0
