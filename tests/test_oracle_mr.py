"""Pins of the oracle's multiresolution transform (Sec. 3.1 details iterated
from the finest level down; Sec. 3.2 lifted coarse values for CDF 4/4).

Closed forms: for a separable trigonometric field f = prod_a cos(w_a p_a +
phi_a) on the periodic lattice, the DD4 prediction (weights -1/16, 9/16,
9/16, -1/16 at odd offsets -3s, -s, s, 3s) multiplies the axis factor by
A(w s) = 9/8 cos(w s) - 1/8 cos(3 w s) along each axis where the point is
odd and by 1 along the others, so the level-m detail is c_m(p) (1 - prod A).
The CDF 4/4 update (-1, 9, 9, -1)/32 on the neighbouring details adds
A (1 - A) / 2 times the value along each axis, so every lifted level
multiplies the coarse field by prod_a H(w_a s), H = 1 + A (1 - A) / 2; with
CDF 4/0 (decimation) the factor is 1.  These formulas are derived from the
filters alone, not from the oracle's code, and they pin the forward
transform point by point and (applied to the formula's own coefficients) the
inverse."""
import numpy as np
import pytest

from oracle import oracle as orc


def A(t):
    return 9.0 / 8.0 * np.cos(t) - 1.0 / 8.0 * np.cos(3.0 * t)


def H(t):
    a = A(t)
    return 1.0 + 0.5 * a * (1.0 - a)


def trig_field(n, k, phi):
    idx = np.arange(n)
    Z, Y, X = np.meshgrid(idx, idx, idx, indexing="ij")
    P = (X, Y, Z)
    om = [2.0 * np.pi * kk / n for kk in k]
    f = np.ones((n, n, n))
    for a in range(3):
        f = f * np.cos(om[a] * P[a] + phi[a])
    return f, P, om


def closed_form(n, nlev, k, phi, wavelet):
    f, P, om = trig_field(n, k, phi)
    out = np.empty_like(f)
    level = np.zeros((n, n, n), dtype=np.int64)
    for m in range(1, nlev + 1):
        s = 2 ** m
        level[(P[0] % s == 0) & (P[1] % s == 0) & (P[2] % s == 0)] = m
    gain = 1.0  # coarse-field factor before level m
    for m in range(nlev + 1):
        sel = level == m
        if m == nlev:
            out[sel] = gain * f[sel]
            break
        s = 2 ** m
        prod = np.ones((n, n, n))
        for a in range(3):
            odd = (P[a] // s) % 2 == 1
            prod = np.where(odd, prod * A(om[a] * s), prod)
        out[sel] = gain * f[sel] * (1.0 - prod[sel])
        if wavelet == 1:
            gain *= np.prod([H(om[a] * s) for a in range(3)])
    return f, out


CASES = [(32, 3, (1, 2, 3)), (24, 2, (2, 1, 1)), (48, 3, (3, 0, 2))]


@pytest.mark.parametrize("wavelet", [0, 1])
@pytest.mark.parametrize("n,nlev,k", CASES)
def test_forward_matches_closed_form(wavelet, n, nlev, k):
    f, expect = closed_form(n, nlev, k, (0.3, -1.1, 0.7), wavelet)
    got = orc.mr_forward(f, nlev, wavelet)
    assert np.max(np.abs(got - expect)) < 1e-13


@pytest.mark.parametrize("wavelet", [0, 1])
@pytest.mark.parametrize("n,nlev,k", CASES)
def test_inverse_of_closed_form(wavelet, n, nlev, k):
    f, coeffs = closed_form(n, nlev, k, (0.3, -1.1, 0.7), wavelet)
    back = orc.mr_inverse(coeffs, nlev, wavelet)
    assert np.max(np.abs(back - f)) < 1e-13


def test_details_vanish_and_coarse_is_kept_for_constants():
    u = np.full((2, 16, 16, 16), 2.5)
    u[1] = -1.0
    idx = np.arange(16)
    Z, Y, X = np.meshgrid(idx, idx, idx, indexing="ij")
    coarse = (X % 4 == 0) & (Y % 4 == 0) & (Z % 4 == 0)
    for wavelet in (0, 1):
        w = orc.mr_forward(u, 2, wavelet)
        assert np.array_equal(w[:, coarse], u[:, coarse])
        assert np.array_equal(w[:, ~coarse], np.zeros_like(u[:, ~coarse]))


@pytest.mark.parametrize("wavelet", [0, 1])
def test_perfect_reconstruction_random(wavelet):
    rng = np.random.default_rng(7)
    u = rng.standard_normal((3, 32, 32, 32))
    w = orc.mr_forward(u, 3, wavelet)
    assert np.max(np.abs(w - u)) > 0.1
    back = orc.mr_inverse(w, 3, wavelet)
    assert np.max(np.abs(back - u)) < 1e-13


def test_cdf40_single_level_is_the_block_detail():
    """One CDF 4/0 level: the odd points hold u - P R u, the quantity whose
    maximum the block thresholding reports; filtering a block zeroes exactly
    these details, so forward, zeroing the level-0 details and the inverse
    equals the prediction of the odd points from the even lattice."""
    rng = np.random.default_rng(3)
    u = rng.standard_normal((16, 16, 16))
    w = orc.mr_forward(u, 1, 0)
    idx = np.arange(16)
    Z, Y, X = np.meshgrid(idx, idx, idx, indexing="ij")
    even = (X % 2 == 0) & (Y % 2 == 0) & (Z % 2 == 0)
    assert np.array_equal(w[even], u[even])
    w2 = np.where(even, w, 0.0)
    filt = orc.mr_inverse(w2, 1, 0)
    # 1D check of one x-odd, y-even, z-even point against the DD4 weights
    z, y, x = 4, 6, 5
    p = (-u[z, y, x - 3] + 9 * u[z, y, x - 1] + 9 * u[z, y, x + 1] - u[z, y, x + 3]) / 16.0
    assert abs(filt[z, y, x] - p) < 1e-14
    assert abs(w[z, y, x] - (u[z, y, x] - p)) < 1e-14


def test_nlev_zero_is_identity_and_bad_sizes_raise():
    u = np.random.default_rng(1).standard_normal((8, 8, 8))
    assert np.array_equal(orc.mr_forward(u, 0, 1), u)
    with pytest.raises(ValueError):
        orc.mr_forward(np.zeros((24, 24, 24)), 3, 0)  # 24 / 8 = 3 < 4
    with pytest.raises(ValueError):
        orc.mr_forward(np.zeros((20, 20, 20)), 3, 0)  # not a multiple of 8
    with pytest.raises(ValueError):
        orc.mr_forward(np.zeros((16, 16, 16)), 1, 2)  # no such wavelet
