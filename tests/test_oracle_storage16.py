"""Pins of the oracle's 16-bit storage format (binary16 spinors with a
per-site FP32 scale, binary16 links), the reduced-precision storage of the
mixed solver's inner iterations.

* binary16 rounding is round-to-nearest-even (literal ties and neighbours);
* the largest component of every non-zero site is stored as exactly +-1 and
  no code exceeds 1 in magnitude; zero sites store zeros;
* round trip: every component within s (2^-12 + 2^-21) of the input, the
  binary16 half-spacing in [1/2, 1] plus the FP32 steps;
* scaling the field by 2^k leaves the codes unchanged and scales s by 2^k;
* links: every entry within 2^-12 + 2^-24 of the input.
"""
import numpy as np
import pytest

from paper_2411_18511_amd import inputs


def test_binary16_rounding_mode():
    one = np.float32(1.0)
    eps = np.float32(2.0 ** -11)  # half the binary16 spacing above 1
    assert np.float16(one + eps) == np.float16(1.0)  # tie -> even
    assert np.float16(one + 3 * eps) == np.float16(1.0 + 2.0 ** -9)  # tie -> even (upwards)
    assert np.float16(np.float32(1.0 + 2.0 ** -11 + 2.0 ** -20)) == np.float16(1.0 + 2.0 ** -10)


@pytest.mark.parametrize("n", [2, 3])
def test_spinor16_format(oracle, n):
    dims = (4, 2, 4, 6)
    psi = inputs.gaussian_spinor(dims, n, 3)
    psi[0, 0, 0, 0] = 0  # one zero site
    codes, s = oracle.quantize_spinor16(psi)
    assert codes.dtype == np.float16 and s.dtype == np.float32
    assert codes.shape == psi.shape + (2,) and s.shape == dims
    a = np.abs(codes.astype(np.float64)).reshape(dims + (-1,))
    assert s[0, 0, 0, 0] == 0 and np.all(a[0, 0, 0, 0] == 0)
    nz = s > 0
    assert np.all(a[nz].max(axis=-1) == 1.0)
    assert a.max() <= 1.0
    back = oracle.dequantize_spinor16(codes, s)
    err = np.maximum(np.abs(back.real - psi.real), np.abs(back.imag - psi.imag))
    bound = s.astype(np.float64)[..., None, None] * (2.0 ** -12 + 2.0 ** -21)
    assert np.all(err <= bound)
    # typical error is far below the bound, and not zero
    assert 0 < np.linalg.norm((back - psi).ravel()) / np.linalg.norm(psi.ravel()) < 3e-4
    for k in (-7, 5):
        c2, s2 = oracle.quantize_spinor16(psi * 2.0 ** k)
        assert np.array_equal(c2, codes)
        assert np.array_equal(s2, s * np.float32(2.0 ** k))


def test_links16(oracle):
    U = inputs.gauge_field((4, 2, 2, 2), 5)
    R = oracle.round_links16(U)
    err = np.maximum(np.abs(R.real - U.real), np.abs(R.imag - U.imag))
    assert err.max() <= 2.0 ** -12 + 2.0 ** -24
    assert err.max() > 0
    Ra = oracle.round_links16(oracle.represent_adjoint(U))
    assert Ra.dtype == np.float64
    assert np.abs(Ra - oracle.represent_adjoint(U)).max() <= 2.0 ** -12 + 2.0 ** -24
