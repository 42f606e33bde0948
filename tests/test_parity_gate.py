"""The GPU parity gate itself (CPU only): a localized fault must fail it.

One mode of a 256^3 half spectrum off by half its size moves rel-L2 by about
0.5 / sqrt(N) = 1.2e-4, under the 2.4e-4 gate; the max-error gate catches it.
"""
import numpy as np
import pytest

from gpu_helpers import assert_close, rel_l2, tol


def _spectrum(shape, seed):
    rng = np.random.default_rng(seed)
    n0, n1, n2 = shape
    k = (n2, n1, n0 // 2 + 1)
    return (rng.standard_normal(k) + 1j * rng.standard_normal(k)).astype(np.complex128)


def test_gate_passes_rounding_noise():
    shape = (256, 256, 256)
    ref = _spectrum(shape, 1)
    got = (ref * (1 + 2e-7)).astype(np.complex64)
    assert_close(got, ref, shape)


def test_gate_fails_one_shifted_mode():
    shape = (256, 256, 256)
    ref = _spectrum(shape, 2)
    got = ref.copy()
    k = (17, 200, 33)
    got[k] += 0.5 * np.sqrt(2.0) * np.exp(0.3j)  # half the rms modulus, one mode
    assert rel_l2(got, ref) <= tol(shape), "the L2 gate alone would let this through"
    with pytest.raises(AssertionError, match="max error"):
        assert_close(got, ref, shape)


def test_gate_fails_spread_error():
    shape = (32, 32, 32)
    ref = _spectrum(shape, 3)
    got = ref * (1 + 1e-3)
    with pytest.raises(AssertionError, match="rel-L2"):
        assert_close(got, ref, shape)
