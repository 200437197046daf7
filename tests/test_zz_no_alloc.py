"""The allocation-free entry point (t2s_unet_mfma_probe_static) against the entry point
it is a variant of (t2s_unet_mfma_probe, which stages through memory it allocates):
the same products, bit for bit, on two calls in a row (the second with fewer tiles,
so stale tiles of the first call in the static buffer must not leak), and the size
limit rejected with an error."""

import numpy as np
import pytest

import paper_1809_04195_amd as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _needs_gpu(gpu):
    return gpu


def _tiles(rng, n):
    A = rng.integers(-64, 65, (n, 16, 16)).astype(np.float32) / 16
    B = rng.standard_normal((n, 16, 16)).astype(np.float32)
    return A, B


def test_static_probe_matches_allocating_probe_twice():
    rng = np.random.default_rng(7)
    for n in (8, 3):
        A, B = _tiles(rng, n)
        D = T.t2s_unet_mfma_probe_static(A, B)
        for i in range(n):
            ref = T.t2s_unet_mfma_probe(A[i], B[i])
            assert np.array_equal(D[i], ref), (n, i)
        # bf16-rounded operands, fp32 accumulation: close to the exact product
        exact = np.einsum("nij,njk->nik", A.astype(np.float64), B.astype(np.float64))
        assert np.abs(D - exact).max() < 0.05 * np.abs(exact).max()


def test_static_probe_rejects_counts_beyond_its_buffer():
    A = np.zeros((9, 16, 16), dtype=np.float32)
    with pytest.raises(T.T2SError):
        T.t2s_unet_mfma_probe_static(A, A)
    A1 = np.ones((1, 16, 16), dtype=np.float32)
    assert np.array_equal(T.t2s_unet_mfma_probe_static(A1, A1)[0], np.full((16, 16), 16.0, dtype=np.float32))
