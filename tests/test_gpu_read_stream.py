"""The read-stream measurement kernel reads every word once: its checksum is
the XOR of all 32-bit words, on sizes that do not fill its unrolled loop."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

fg = pytest.importorskip("paper_2603_21710_amd")


@pytest.mark.parametrize("words", [0, 4, 1028, 4 * 1000003, 1 << 26])
def test_read_stream_checksum(words):
    rng = np.random.default_rng(words)
    a = rng.integers(-2**31, 2**31 - 1, words, dtype=np.int64).astype(np.int32)
    print(f"case words={words}", flush=True)
    got = int(fg.read_stream(torch.from_numpy(a).cuda()).cpu()[0])
    want = int(np.bitwise_xor.reduce(a.view(np.uint32))) if words else 0
    assert (got & 0xFFFFFFFF) == want
