"""Pins of the oracle's Teter-Payne-Allan preconditioner, the one the CG
figure of Sec. III.B cites: K(x) = (27+18x+12x^2+8x^3)/(27+18x+12x^2+8x^3+16x^4)
with x = |k+G|^2 / max(E_kin, 1e-3).

The checks do not evaluate the polynomial in floating point a second time:
exact rational values at small integer and half-integer x (Python fractions),
the Taylor structure at x = 0 (K = 1 - (16/27) x^4 + O(x^5): the first three
derivatives vanish, so low-kinetic components pass unchanged), the large-x
asymptote x K(x) -> 1/2 (high components damped like the inverse kinetic
energy), monotone decrease, and the scaling of x by each band's kinetic energy
with its 1e-3 Ry floor. A dropped term or a wrong coefficient moves at least
one exact value; a swapped kin/ekin ratio breaks the scaling checks.
"""
from fractions import Fraction

import numpy as np

import oracle


def _k_exact(x: Fraction) -> Fraction:
    num = 27 + 18 * x + 12 * x ** 2 + 8 * x ** 3
    return num / (num + 16 * x ** 4)


# hand-reduced exact values: K(1) = 65/81, K(2) = 175/431, K(1/2) = 40/41, K(3) = 405/1701 = 5/21
EXACT = {Fraction(1): Fraction(65, 81), Fraction(2): Fraction(175, 431), Fraction(1, 2): Fraction(40, 41),
         Fraction(3): Fraction(5, 21)}


def test_tpa_exact_rational_values():
    xs = sorted(EXACT)
    # ekin = 1 makes x = kin exactly
    k = oracle.tpa_preconditioner(np.array([float(x) for x in xs]), np.array([1.0]))[0]
    for x, kv in zip(xs, k):
        assert _k_exact(x) == EXACT[x]          # the reduced fractions above are the polynomial's
        assert abs(kv - float(EXACT[x])) < 4e-16


def test_tpa_flat_at_zero_and_inverse_tail():
    k0 = oracle.tpa_preconditioner(np.array([0.0]), np.array([1.0]))[0, 0]
    assert k0 == 1.0
    # 1 - K(x) = 16 x^4 / (27 + ...): (1 - K) / x^4 -> 16/27
    x = np.array([1e-2, 3e-3])
    k = oracle.tpa_preconditioner(x, np.array([1.0]))[0]
    ratio = (1.0 - k) / x ** 4
    assert np.all(np.abs(ratio - 16.0 / 27.0) < 0.02 * 16.0 / 27.0)
    # x K(x) -> 8/16 = 1/2, the gap closing like 1/x
    big = np.array([1e4, 1e6])
    kb = oracle.tpa_preconditioner(big, np.array([1.0]))[0]
    assert np.all(np.abs(big * kb - 0.5) < 1e-3)
    assert abs(1e6 * kb[1] - 0.5) < abs(1e4 * kb[0] - 0.5)


def test_tpa_monotone_and_bounded():
    x = np.linspace(0.0, 50.0, 2001)
    k = oracle.tpa_preconditioner(x, np.array([1.0]))[0]
    assert np.all(np.diff(k) < 0.0)
    assert np.all((k > 0.0) & (k <= 1.0))


def test_tpa_scaling_by_band_kinetic_energy():
    kin = np.array([0.0, 0.5, 1.0, 4.0])
    ek = np.array([2.0, 0.5, 1e-6])            # the last band sits below the 1e-3 Ry floor
    k = oracle.tpa_preconditioner(kin, ek)
    assert k.shape == (3, 4)
    # x = kin / ekin: the band with ekin = 2 at kin = 4 sees x = 2; ekin = 0.5 at kin = 1 sees x = 2
    assert abs(k[0, 3] - float(EXACT[Fraction(2)])) < 4e-16
    assert abs(k[1, 2] - float(EXACT[Fraction(2)])) < 4e-16
    # ekin = 0.5 at kin = 0.5 sees x = 1
    assert abs(k[1, 1] - float(EXACT[Fraction(1)])) < 4e-16
    # floor: ekin -> 1e-3, so kin = 1e-3 * 3 would give x = 3; kin = 0.5 gives x = 500
    kf = oracle.tpa_preconditioner(np.array([3e-3]), np.array([1e-6]))[0, 0]
    assert abs(kf - float(EXACT[Fraction(3)])) < 1e-15
    assert abs(500.0 * k[2, 1] - 0.5) < 2e-3
