"""The fused binning's bin rule, emulated on the CPU: an FP32 estimate
nbins sqrt(q / qmax) (the hardware square root may be off by an ulp or two)
corrected by one comparison each way against the estimated bin's edges must
give the exact integer bin max{b : b^2 qmax <= nbins^2 q} (clamped to
nbins - 1) for every q the supported lattices produce (q, qmax < 2^32,
nbins <= 4096).  Checked at every bin edge and its neighbours, and on random
q, with the square root perturbed by up to 2 ulp either way."""
import numpy as np
import pytest


def exact_bin(q, nb, qm):
    b = np.floor(np.sqrt(q.astype(np.float64) * nb * nb / qm)).astype(np.int64)
    b = np.where((b + 1) ** 2 * qm <= nb * nb * q, b + 1, b)
    b = np.where(b * b * qm > nb * nb * q, b - 1, b)
    return np.minimum(b, nb - 1)


def edge_bin(q, nb, qm, ulps):
    cq = np.float32(nb * nb / qm)
    est = np.sqrt(q.astype(np.float32) * cq)
    step = np.float32(np.inf) if ulps > 0 else np.float32(0)
    for _ in range(abs(ulps)):
        est = np.nextafter(est, step)
    b = est.astype(np.int64)
    assert b.min() >= 0 and b.max() <= nb
    bs = np.arange(nb + 2, dtype=np.int64)
    th = -(-(bs * bs * qm) // (nb * nb))       # smallest q of bin b
    lo = th[:nb + 1]
    hi = np.concatenate([th[1:nb + 1], [2 ** 32 - 1]])
    b = b + (q >= hi[b]) - (q < lo[b])
    return np.minimum(b, nb - 1)


@pytest.mark.parametrize("qm", [3 * 16 ** 2, 3 * 256 ** 2, 3 * 1024 ** 2, 3 * 15360 ** 2, 4_000_000_000])
@pytest.mark.parametrize("nb", [1, 7, 128, 1000, 4096])
def test_edge_correction_is_exact(qm, nb):
    rng = np.random.default_rng(nb * 7 + qm % 1000)
    bs = np.arange(nb + 1, dtype=np.int64)
    th = -(-(bs * bs * qm) // (nb * nb))
    q = np.concatenate([th - 1, th, th + 1, rng.integers(1, qm + 1, 50000)])
    q = q[(q >= 1) & (q <= qm)]
    want = exact_bin(q, nb, qm)
    for ulps in (-2, -1, 0, 1, 2):
        assert np.array_equal(edge_bin(q, nb, qm, ulps), want)
