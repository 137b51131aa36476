"""Pins for the oracle's Boys function F_m(x) = int_0^1 y^{2m} exp(-x y^2) dy
(Eq. (28) of the paper), against facts that do not come from the oracle."""
import math

import mpmath
import numpy as np
import pytest
import scipy.special as sp

from oracle import oracle as O

mpmath.mp.dps = 40

X_GRID = [0.0, 1e-15, 1e-8, 1e-3, 0.1, 0.5, 1.0, 2.0, 5.0, 10.0, 17.3, 29.9, 35.9, 36.0, 36.1,
          45.0, 49.99, 50.0, 50.01, 60.0, 117.9, 118.0, 118.1, 250.0, 1e3, 1e4, 1e5, 1e7]


def boys_mp(m, x):
    """Eq. (28) by mpmath: lower incomplete gamma form, 40 digits."""
    x = mpmath.mpf(x)
    if x == 0:
        return mpmath.mpf(1) / (2 * m + 1)
    a = mpmath.mpf(m) + mpmath.mpf(1) / 2
    return mpmath.gammainc(a, 0, x) / (2 * x ** a)


def test_boys_matches_definition_by_quadrature():
    # direct numerical integration of the defining integral, Eq. (28)
    for m in (0, 1, 4, 9):
        for x in (0.0, 0.7, 3.0, 12.0, 40.0):
            ref = mpmath.quad(lambda y: y ** (2 * m) * mpmath.exp(-x * y * y), [0, 1])
            got = O.boys([x], m)[m, 0]
            assert abs(got - float(ref)) <= 1e-15 * float(ref) + 1e-300


@pytest.mark.parametrize("quad", [False, True])
def test_boys_vs_mpmath(quad):
    mmax = 25
    F = O.boys(X_GRID, mmax, quad=quad)
    worst = 0.0
    for i, x in enumerate(X_GRID):
        for m in range(mmax + 1):
            ref = float(boys_mp(m, x))
            if ref == 0.0 or ref < 1e-300:
                continue
            worst = max(worst, abs(F[m, i] - ref) / ref)
    assert worst < 5e-15, worst


def test_boys_at_zero():
    F = O.boys([0.0], 30)
    for m in range(31):
        assert F[m, 0] == pytest.approx(1.0 / (2 * m + 1), rel=1e-16)


def test_boys_f0_closed_form():
    # F_0(x) = sqrt(pi/(4x)) erf(sqrt(x)); the printed Sec. 3.2.1 formula lacks the 1/2
    for x in [1e-6, 0.3, 2.0, 7.5, 33.0, 51.0, 400.0]:
        ref = mpmath.sqrt(mpmath.pi / (4 * x)) * mpmath.erf(mpmath.sqrt(x))
        assert O.boys([x], 0)[0, 0] == pytest.approx(float(ref), rel=2e-16)
    # the printed form without the 1/2 would be twice as large
    x = 2.0
    assert O.boys([x], 0)[0, 0] == pytest.approx(0.5 * math.sqrt(math.pi / x) * math.erf(math.sqrt(x)), rel=1e-15)


def test_boys_scipy_identities():
    xs = np.array([1e-4, 0.25, 1.0, 3.3, 8.0, 20.0, 35.0, 47.0, 55.0, 90.0])
    F = O.boys(xs, 12)
    for m in range(13):
        a = m + 0.5
        g = sp.gamma(a) * sp.gammainc(a, xs) / (2 * xs ** a)
        assert np.allclose(F[m], g, rtol=2e-14, atol=0)
        small = xs < 30
        h = sp.hyp1f1(a, a + 1, -xs[small]) / (2 * m + 1)
        assert np.allclose(F[m][small], h, rtol=1e-12, atol=0)


def test_boys_downward_recursion_consistency():
    # F_m = (2x F_{m+1} + exp(-x)) / (2m+1): Eq. (42) rearranged; checked
    # in both evaluation branches of the oracle
    xs = np.array([0.0, 0.01, 1.5, 9.0, 30.0, 49.0, 51.0, 80.0, 500.0])
    F = O.boys(xs, 20)
    for m in range(20):
        rhs = (2 * xs * F[m + 1] + np.exp(-xs)) / (2 * m + 1)
        assert np.allclose(F[m], rhs, rtol=1e-14, atol=0)


def test_boys_derivative():
    # dF_m/dx = -F_{m+1}
    for x in [0.4, 3.0, 25.0, 70.0]:
        h = 1e-4 * x
        F = O.boys([x - h, x, x + h], 6)
        for m in range(6):
            d = (F[m, 2] - F[m, 0]) / (2 * h)
            assert d == pytest.approx(-F[m + 1, 1], rel=1e-7)


def test_boys_large_x_asymptote():
    # F_m(x) -> Gamma(m+1/2)/(2 x^{m+1/2}); relative deviation = Q(m+1/2, x)
    for x in [40.0, 118.0, 1e3, 1e7]:
        F = O.boys([x], 25)
        for m in range(26):
            asym = float(mpmath.gamma(m + 0.5) / (2 * mpmath.mpf(x) ** (m + 0.5)))
            Q = sp.gammaincc(m + 0.5, x)
            assert abs(F[m, 0] / asym - 1.0) <= Q + 2e-15


def test_boys_quad_vs_f64():
    xs = np.concatenate([np.linspace(0, 60, 97), [118.5, 1e4]])
    Fd = O.boys(xs, 30)
    Fq = O.boys(xs, 30, quad=True)
    # the fp64 series sums up to ~100 positive terms: a few ulp of rounding
    assert np.all(np.abs(Fd - Fq) <= 2e-15 * np.abs(Fq) + 1e-300)
