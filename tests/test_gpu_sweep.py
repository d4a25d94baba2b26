"""A seeded sweep of shapes through every precision, against the oracle (needs the GPU).

The shapes are drawn once from a fixed generator: rows around multiples of 16 and 128
(tile edges), widths around multiples of 16, 32 and 128 (k-step edges of the FP32,
BF16 and e4m3 kernels), table counts that select each tile width, and chunk sizes that
leave ragged last chunks.  Each case must pass the full parity bar of `full_parity`."""
import numpy as np
import pytest

from ace_inputs import gaussian_clusters, projection_matrix
from tests.parity import full_parity

pytestmark = pytest.mark.gpu


def _cases():
    rng = np.random.default_rng(20260601)
    out = []
    for i in range(24):
        base_n = int(rng.choice([16, 128, 256, 1024]))
        n = max(1, base_n * int(rng.integers(1, 4)) + int(rng.integers(-2, 3)))
        base_d = int(rng.choice([16, 32, 128]))
        d = max(1, base_d * int(rng.integers(1, 5)) + int(rng.integers(-3, 4)))
        K = int(rng.integers(1, 17))
        L = int(rng.choice([1, 2, 3, 5, 7, 8, 13, 20, 33, 50, 64, 100]))
        precision = ["fp32", "bf16", "fp8"][i % 3]
        chunk = int(rng.choice([0, 0, 17, 100, 1000]))
        out.append((i, n, d, K, L, precision, chunk))
    return out


@pytest.mark.parametrize("i,n,d,K,L,precision,chunk", _cases())
def test_sweep(i, n, d, K, L, precision, chunk):
    X, _ = gaussian_clusters(n, d, 3, 0.05, seed=1000 + i)
    W = projection_matrix(d, K, L, 2000 + i)
    r = full_parity(X, W, K, L, precision=precision, max_batch_rows=chunk)
    print((i, n, d, K, L, precision, chunk, r), flush=True)
