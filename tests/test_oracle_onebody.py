"""Pins of the oracle's overlap and kinetic-energy integrals (the 1-particle
set of Sec. 2.1 with Eq. (8)), each against something the oracle does not
compute the same way: Gauss-Hermite quadrature of the gradient form
T = 1/2 <grad a . grad b> (integration by parts of -1/2 <a|nabla^2|b>, the
oracle differentiates the ket twice), the textbook s-type closed form, and
the a <-> b symmetry the one-sided formula does not build in."""
import math

import numpy as np
import pytest

from oracle import oracle as O


def _cart(l):
    return [(l - s, s - v, v) for s in range(l + 1) for v in range(s + 1)]


def _quad_1d(i, j, za, zb, A, B, n=40):
    """(overlap, gradient product) of one axis by Gauss-Hermite quadrature"""
    y, w = np.polynomial.hermite.hermgauss(n)
    p = za + zb
    P = (za * A + zb * B) / p
    x = P + y / math.sqrt(p)
    pref = math.exp(-za * zb / p * (A - B) ** 2) / math.sqrt(p)
    xa, xb = x - A, x - B
    s = pref * np.sum(w * xa ** i * xb ** j)
    da = (i * xa ** (i - 1) if i > 0 else 0.0) - 2 * za * xa ** (i + 1)
    db = (j * xb ** (j - 1) if j > 0 else 0.0) - 2 * zb * xb ** (j + 1)
    g = pref * np.sum(w * da * db)
    return s, g


@pytest.mark.parametrize("la,lb", [(0, 0), (1, 0), (0, 2), (1, 1), (2, 1), (2, 2), (3, 2), (4, 4), (5, 2), (6, 4),
                                   (6, 6)])
def test_kinetic_vs_gradient_form_quadrature(la, lb):
    rng = np.random.default_rng(10 * la + lb)
    for _ in range(4):
        za, zb = np.exp(rng.uniform(-1.5, 2.0, 2))
        A, B = rng.uniform(-1.0, 1.0, 3), rng.uniform(-1.0, 1.0, 3)
        T = O.kinetic(la, lb, A, B, [za], [1.0], [zb], [1.0], cartesian=True)
        for a_, (ax, ay, az) in enumerate(_cart(la)):
            for b_, (bx, by, bz) in enumerate(_cart(lb)):
                sx, gx = _quad_1d(ax, bx, za, zb, A[0], B[0])
                sy, gy = _quad_1d(ay, by, za, zb, A[1], B[1])
                sz, gz = _quad_1d(az, bz, za, zb, A[2], B[2])
                ref = 0.5 * (gx * sy * sz + sx * gy * sz + sx * sy * gz)
                assert T[a_, b_] == pytest.approx(ref, rel=1e-11, abs=1e-14 * max(1.0, abs(ref)))


def test_kinetic_s_closed_form():
    # T_ss = mu (3 - 2 mu |A-B|^2) S_ss with mu = za zb / (za + zb)
    rng = np.random.default_rng(3)
    for _ in range(10):
        za, zb = np.exp(rng.uniform(-2, 3, 2))
        A, B = rng.uniform(-2, 2, 3), rng.uniform(-2, 2, 3)
        mu = za * zb / (za + zb)
        S = O.overlap(0, 0, A, B, [za], [1.0], [zb], [1.0])[0, 0]
        T = O.kinetic(0, 0, A, B, [za], [1.0], [zb], [1.0])[0, 0]
        assert T == pytest.approx(mu * (3 - 2 * mu * np.sum((A - B) ** 2)) * S, rel=1e-13)


@pytest.mark.parametrize("cartesian", [True, False])
def test_kinetic_hermitian(cartesian):
    # the oracle applies the Laplacian to the ket only; T must still be symmetric
    rng = np.random.default_rng(4)
    for la, lb in [(1, 0), (2, 1), (2, 2), (3, 1), (4, 2), (5, 3), (6, 6)]:
        za, zb = np.exp(rng.uniform(-1, 2, 3)), np.exp(rng.uniform(-1, 2, 2))
        ca, cb = rng.uniform(0.1, 1, 3), rng.uniform(0.1, 1, 2)
        A, B = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
        T1 = O.kinetic(la, lb, A, B, za, ca, zb, cb, cartesian=cartesian)
        T2 = O.kinetic(lb, la, B, A, zb, cb, za, ca, cartesian=cartesian)
        assert np.allclose(T1, T2.T, rtol=1e-12, atol=1e-14 * np.abs(T1).max())


def test_one_body_layout_matches_per_pair_calls():
    from paper_2506_12501_amd import workloads as W
    b = W.make_class_batch("(dp|ss)", 3, 1, 2, 4.0, 0.1, 10.0, 0.1, 1.0, seed=9)
    S, T = O.one_body(b.basis, b.bra)
    S = S.reshape(15, 3)
    for ij, (a, c) in enumerate(b.bra):
        sa = slice(b.basis.poff[a], b.basis.poff[a] + b.basis.nprim[a])
        sc = slice(b.basis.poff[c], b.basis.poff[c] + b.basis.nprim[c])
        ref = O.overlap(2, 1, b.basis.xyz[a], b.basis.xyz[c], b.basis.exps[sa], b.basis.coefs[sa],
                        b.basis.exps[sc], b.basis.coefs[sc], cartesian=False)
        assert np.allclose(S[:, ij], ref.reshape(-1))


@pytest.mark.parametrize("la,lb", [(4, 0), (5, 4), (6, 6)])
def test_overlap_vs_gauss_hermite_high_l(la, lb):
    """overlaps of l = 4..6 shells (Eq. (8)) against Gauss-Hermite quadrature
    of the monomial products, Cartesian; and the solid form equals the solid
    coefficients applied to the Cartesian one"""
    rng = np.random.default_rng(20 + la + lb)
    za, zb = np.exp(rng.uniform(-1.0, 1.5, 2))
    A, B = rng.uniform(-1.0, 1.0, 3), rng.uniform(-1.0, 1.0, 3)
    S = O.overlap(la, lb, A, B, [za], [1.0], [zb], [1.0], cartesian=True)
    for a_, (ax, ay, az) in enumerate(_cart(la)):
        for b_, (bx, by, bz) in enumerate(_cart(lb)):
            ref = _quad_1d(ax, bx, za, zb, A[0], B[0])[0] * _quad_1d(ay, by, za, zb, A[1], B[1])[0] * \
                _quad_1d(az, bz, za, zb, A[2], B[2])[0]
            assert S[a_, b_] == pytest.approx(ref, rel=1e-11, abs=1e-14 * np.abs(S).max())
    Ss = O.overlap(la, lb, A, B, [za], [1.0], [zb], [1.0], cartesian=False, quad=True)
    ref = O.solid_coefs(la, quad=True) @ O.overlap(la, lb, A, B, [za], [1.0], [zb], [1.0], cartesian=True,
                                                    quad=True) @ O.solid_coefs(lb, quad=True).T
    assert np.allclose(Ss, ref, rtol=1e-12, atol=1e-14 * np.abs(ref).max())
