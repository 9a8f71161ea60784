"""GPU check of the read-bandwidth probe: it must read every word (its sum is exact mod 2^64)."""
import numpy as np
import pytest
import torch

from paper_1910_10063_amd import skew

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_words", [0, 4, 68, 4096 * 257 + 4, 10_000_000, (1 << 26) + 12])
def test_stream_probe_sum(n_words):
    print(f"[case] stream_probe n_words={n_words}", flush=True)
    rng = np.random.default_rng(n_words)
    h = rng.integers(0, 2**32, n_words, dtype=np.uint64).astype(np.uint32)
    d = torch.from_numpy(h.view(np.int32)).to("cuda")
    got = int(skew.stream_probe(d).cpu().numpy().view(np.uint64)[0])
    want = int(h.astype(np.uint64).sum(dtype=np.uint64)) if n_words else 0
    assert got == want
