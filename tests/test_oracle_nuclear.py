"""Pins of the oracle's 1-particle Coulomb (nuclear attraction) integrals,
Eqs. (24), (26), (30), (34), each against something the oracle does not
compute the same way: Gaussian-transform quadrature of 1/r (no Boys function,
no recursion), the (s|s) closed form with the error function, linearity in
the charges, a <-> b symmetry, and the far-field limit."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests import quadrature as Q


@pytest.mark.parametrize("la,lb", [(0, 0), (1, 0), (0, 1), (1, 1), (2, 0), (2, 1), (1, 2), (2, 2), (3, 1),
                                   (4, 0), (2, 4), (5, 1), (4, 3), (6, 0), (6, 2)])
def test_primitive_vs_gaussian_transform_quadrature(la, lb):
    rng = np.random.default_rng(40 + 5 * la + lb)
    for _ in range(3):
        za, zb = np.exp(rng.uniform(-1.0, 1.5, 2))
        A, B, C = (rng.uniform(-1.0, 1.0, 3) for _ in range(3))
        q = rng.uniform(0.5, 3.0)
        V = O.nuclear(la, lb, A, B, [za], [1.0], [zb], [1.0], [[*C, q]], cartesian=True)
        ref = -q * Q.nuclear_prim_cart(la, lb, za, zb, A, B, C)
        assert np.allclose(V, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max()), (la, lb, V, ref)


def test_ss_closed_form():
    """(s|s) = -q c_a c_b (2 pi/p) exp(-za zb/p |AB|^2) F0(p |PC|^2),
    F0(x) = sqrt(pi/(4x)) erf(sqrt x) (from Eq. (28) directly)"""
    rng = np.random.default_rng(3)
    for _ in range(10):
        za, zb = np.exp(rng.uniform(-2, 3, 2))
        A, B, C = (rng.uniform(-2, 2, 3) for _ in range(3))
        p = za + zb
        P = (za * A + zb * B) / p
        x = p * np.sum((P - C) ** 2)
        F0 = math.sqrt(math.pi / (4 * x)) * math.erf(math.sqrt(x))
        ref = -1.7 * 0.3 * 0.9 * 2 * math.pi / p * math.exp(-za * zb / p * np.sum((A - B) ** 2)) * F0
        V = O.nuclear(0, 0, A, B, [za], [0.3], [zb], [0.9], [[*C, 1.7]])
        assert abs(V[0, 0] - ref) <= 1e-14 * abs(ref)


def test_charge_on_the_product_centre():
    """charge at P: F0(0) = 1, (s|s) = -q c_a c_b (2 pi/p) K_AB"""
    za, zb = 0.7, 1.9
    A, B = np.array([0.1, -0.3, 0.4]), np.array([-0.5, 0.2, 0.0])
    p = za + zb
    P = (za * A + zb * B) / p
    V = O.nuclear(0, 0, A, B, [za], [1.0], [zb], [1.0], [[*P, 2.0]])
    ref = -2.0 * 2 * math.pi / p * math.exp(-za * zb / p * np.sum((A - B) ** 2))
    assert abs(V[0, 0] - ref) <= 1e-14 * abs(ref)


@pytest.mark.parametrize("cart", [True, False])
def test_linear_in_the_charges(cart):
    rng = np.random.default_rng(8)
    A, B = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
    za, zb = [0.4, 2.0, 9.0], [0.8, 3.0]
    ca, cb = [0.2, 0.5, 0.3], [0.6, 0.4]
    ch = np.c_[rng.uniform(-3, 3, (7, 3)), rng.uniform(0.5, 8, 7)]
    whole = O.nuclear(2, 1, A, B, za, ca, zb, cb, ch, cartesian=cart)
    parts = sum(O.nuclear(2, 1, A, B, za, ca, zb, cb, ch[i:i + 1], cartesian=cart) for i in range(7))
    assert np.allclose(whole, parts, rtol=1e-13, atol=1e-15)
    doubled = O.nuclear(2, 1, A, B, za, ca, zb, cb, np.c_[ch[:, :3], 2 * ch[:, 3]], cartesian=cart)
    assert np.allclose(doubled, 2 * whole, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("la,lb", [(1, 0), (2, 1), (2, 2), (4, 2), (5, 3), (6, 6)])
def test_bra_ket_symmetry(la, lb):
    """V_ab = V_ba: the operator is a multiplication, the E recursion of
    Eqs. (10)-(11) is not symmetric in its two indices"""
    rng = np.random.default_rng(la + 7 * lb)
    A, B = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
    za, zb = [0.5, 3.0], [1.2]
    ca, cb = [0.7, 0.3], [1.0]
    ch = np.c_[rng.uniform(-2, 2, (5, 3)), rng.uniform(1, 6, 5)]
    for cart in (True, False):
        ab = O.nuclear(la, lb, A, B, za, ca, zb, cb, ch, cartesian=cart)
        ba = O.nuclear(lb, la, B, A, zb, cb, za, ca, ch, cartesian=cart)
        assert np.allclose(ab, ba.T, rtol=1e-12, atol=1e-14)


def test_far_charge_is_a_point_monopole():
    """a charge far from a compact pair sees -q S_ab / |P - C| to O(1/R^2)"""
    A, B = np.array([0.1, 0.0, -0.2]), np.array([-0.2, 0.3, 0.1])
    za, zb = [1.5], [2.5]
    C = np.array([0.0, 0.0, 2000.0])
    V = O.nuclear(1, 1, A, B, za, [1.0], zb, [1.0], [[*C, 1.0]])
    S = O.overlap(1, 1, A, B, za, [1.0], zb, [1.0])
    P = (1.5 * A + 2.5 * B) / 4.0
    ref = -S / np.linalg.norm(P - C)
    # the dipole of a p-p product about P (extent ~1 bohr) enters at 1/R^2
    assert np.allclose(V, ref, rtol=0, atol=4.0 * np.abs(S).max() / 2000.0 ** 2)
    assert np.abs(ref).max() > 100 * 4.0 * np.abs(S).max() / 2000.0 ** 2


def test_quad_build_agrees():
    rng = np.random.default_rng(12)
    A, B = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
    ch = np.c_[rng.uniform(-2, 2, (4, 3)), rng.uniform(1, 6, 4)]
    a = O.nuclear(2, 2, A, B, [0.3, 4.0], [0.5, 0.5], [1.1], [1.0], ch, cartesian=False)
    b = O.nuclear(2, 2, A, B, [0.3, 4.0], [0.5, 0.5], [1.1], [1.0], ch, cartesian=False, quad=True)
    assert np.allclose(a, b, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("la,lb", [(4, 1), (5, 3), (6, 6)])
def test_quad_build_agrees_high_l(la, lb):
    """fp64 against __float128 (whose solid coefficients are formed in
    __float128 too): Cartesian within 1e-13 of the block maximum, solid within
    1e-11 (the Cartesian-to-solid sums of an l = 6 shell cancel)"""
    rng = np.random.default_rng(13 + la + lb)
    A, B = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
    ch = np.c_[rng.uniform(-3, 3, (6, 3)), rng.uniform(1, 6, 6)]
    for cart, tol in ((True, 1e-13), (False, 1e-11)):
        a = O.nuclear(la, lb, A, B, [0.3, 4.0], [0.5, 0.5], [1.1], [1.0], ch, cartesian=cart)
        b = O.nuclear(la, lb, A, B, [0.3, 4.0], [0.5, 0.5], [1.1], [1.0], ch, cartesian=cart, quad=True)
        assert np.max(np.abs(a - b)) <= tol * np.max(np.abs(b)), (la, lb, cart, np.max(np.abs(a - b)) / np.max(np.abs(b)))
