"""Pins of the oracle's BF16 and FP8-E4M3 encodings against torch's
conversions (round to nearest even) and the format definitions."""
import numpy as np
import torch

import oracle


def test_bf16_roundtrip_all_patterns():
    for b in range(0, 1 << 16, 1):
        f = np.array([b << 16], np.uint32).view(np.float32)[0]
        e = (b >> 7) & 0xFF
        m = b & 0x7F
        if e == 0xFF and m:
            continue
        assert oracle.bf16_from_f32(f) == b
        assert oracle.bf16_to_f32(b) == f or np.isnan(f)


def test_bf16_matches_torch_rne():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-30, 30, 4000),
                        (np.arange(1 << 12) * 2.0 ** -10 + 1.0)]).astype(np.float32)
    t = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    got = np.array([oracle.bf16_from_f32(v) for v in x], np.uint16)
    assert (got == t).all()


def test_fp8_decode_matches_torch():
    codes = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    ref = codes.view(torch.float8_e4m3fn).to(torch.float32).numpy()
    for c in range(256):
        v = oracle.fp8_to_f32(c)
        assert (np.isnan(v) and np.isnan(ref[c])) or v == ref[c]
    assert oracle.fp8_to_f32(0x7E) == 448.0
    assert oracle.fp8_to_f32(0x01) == 2.0 ** -9


def test_fp8_encode_matches_torch_in_range():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-448, 448, 20000),
                        rng.normal(size=5000) * 2.0 ** -7,
                        [0.0, 448.0, -448.0, 2.0 ** -10, 3 * 2.0 ** -10]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = np.array([oracle.fp8_from_f32(v) for v in x], np.uint8)
    assert (got == ref).all()


def test_fp8_saturates():
    assert oracle.fp8_from_f32(1e6) == 0x7E
    assert oracle.fp8_from_f32(-500.0) == 0xFE


def test_quantize_fp8_error_bound():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(64, 96)).astype(np.float32)
    X[3] = 0.0
    codes, sc, deq = oracle.quantize_fp8(X)
    assert sc[3] == 1.0 and (deq[3] == 0).all()
    amax = np.abs(X).max(1)
    # 3 mantissa bits: relative error <= 2^-4 in the normal range, absolute
    # <= s * 2^-10 below it.
    err = np.abs(deq - X)
    bound = np.maximum(np.abs(X) * 2.0 ** -4, (amax / 448.0)[:, None] * 2.0 ** -10) * 1.0001
    assert (err <= bound + 1e-30).all()
    assert (np.abs(codes.view(np.int8).astype(np.int32)) <= 0x7E).all()


def test_quantize_bf16_matches_torch():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(32, 64)).astype(np.float32)
    codes, deq = oracle.quantize_bf16(X)
    ref = torch.from_numpy(X).to(torch.bfloat16)
    assert (codes == ref.view(torch.int16).numpy().view(np.uint16)).all()
    assert (deq == ref.to(torch.float32).numpy()).all()
