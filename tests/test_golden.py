"""The oracle against the hand-derived fixtures of tests/golden/: the forward
DFT of two small lattices (section 3.6 transforms) and the closed-form
solution of the Poisson problem for one Fourier mode, with continuous and
discrete k^2 at two lattice spacings."""
import numpy as np
import pytest

import oracle
from golden_fixtures import line_4x2x2, poisson_cos_8x4x4, ramp_2x2x2


@pytest.mark.parametrize("case", [ramp_2x2x2, line_4x2x2])
def test_oracle_dft_fixtures(case):
    f, F = case()
    n0 = f.shape[2]
    assert np.abs(oracle.c2c(f.astype(np.complex128)) - F).max() <= 1e-12
    assert np.abs(oracle.r2c(f) - F[..., : n0 // 2 + 1]).max() <= 1e-12
    # and back: the unnormalised inverse is N times the input
    assert np.abs(oracle.c2r(F[..., : n0 // 2 + 1], n0) - f.size * f).max() <= 1e-11


def test_oracle_poisson_fixture():
    rho, cases = poisson_cos_8x4x4()
    for dx, k2mode, a in cases:
        phi = oracle.poisson(rho, dx=dx, k2mode=k2mode)
        assert np.abs(phi - a * rho).max() <= 1e-12 * abs(a), (dx, k2mode)


def test_fixtures_catch_planted_mistakes():
    """Plausible mistakes, planted in copies of the oracle's results, fail the
    fixtures: the opposite sign convention, transposed axes, a dropped dx^2
    and the continuous k^2 in place of the discrete one."""
    f, F = line_4x2x2()
    assert np.abs(np.conj(oracle.c2c(f.astype(np.complex128))) - F).max() > 1.0
    f, F = ramp_2x2x2()
    assert np.abs(oracle.c2c(np.ascontiguousarray(f.transpose(2, 1, 0)).astype(np.complex128)) - F).max() > 1.0
    rho, cases = poisson_cos_8x4x4()
    for dx, k2mode, a in cases:
        if dx != 1.0:
            assert np.abs(oracle.poisson(rho, dx=1.0, k2mode=k2mode) - a * rho).max() > 0.1 * abs(a)
        assert np.abs(oracle.poisson(rho, dx=dx, k2mode=1 - k2mode) - a * rho).max() > 0.01 * abs(a)
