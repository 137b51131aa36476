"""Pins of the oracle's density contraction (digestion) of integral batches:
unit densities pick single integrals out of the oracle's own batch in the
documented index placement, the two contractions share one bilinear form,
a batch with bra = ket and a symmetric density gives Jbra = Jket, and the
contraction is linear in the density."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import workloads as W


def batch(name, nb, nk, seed):
    return W.make_class_batch(name, nb, nk, 2, 4.0, 0.1, 10.0, 0.1, 1.0, seed=seed)


def sizes(b, cart=False):
    la, lb, lc, ld = W.parse_class(b.name)
    nab = O.nfunc(la, cart) * (O.nfunc(lb, cart) if lb >= 0 else 1)
    ncd = O.nfunc(lc, cart) * (O.nfunc(ld, cart) if ld >= 0 else 1)
    return nab, ncd


@pytest.mark.parametrize("name", ["(pp|ps)", "(dp|ss)", "(p|dd)"])
def test_unit_densities_pick_integrals(name):
    b = batch(name, 3, 4, seed=5)
    nab, ncd = sizes(b)
    I = O.eri(b.basis, b.ncentre, b.bra, b.ket)
    rng = np.random.default_rng(0)
    for _ in range(4):
        kl, cd = rng.integers(4), rng.integers(ncd)
        ij, ab = rng.integers(3), rng.integers(nab)
        Dk = np.zeros((4, ncd)); Dk[kl, cd] = 1.0
        Db = np.zeros((3, nab)); Db[ij, ab] = 1.0
        Jb, Jk = O.digest(b.basis, b.ncentre, b.bra, b.ket, Db, Dk)
        assert np.array_equal(Jb, I[:, :, cd, kl])
        assert np.array_equal(Jk, I[ij, ab, :, :].T)


def test_bilinear_form():
    """sum Dbra Jbra = sum Dket Jket = Dbra . (ab|cd) . Dket"""
    b = batch("(dd|pp)", 5, 6, seed=9)
    nab, ncd = sizes(b)
    rng = np.random.default_rng(1)
    Db, Dk = rng.standard_normal((5, nab)), rng.standard_normal((6, ncd))
    Jb, Jk = O.digest(b.basis, 4, b.bra, b.ket, Db, Dk)
    e1, e2 = np.sum(Db * Jb), np.sum(Dk * Jk)
    assert abs(e1 - e2) <= 1e-12 * max(abs(e1), 1.0)


def test_same_pairs_symmetric_density():
    """bra = ket pairs: (ab|cd)_{ij,kl} = (cd|ab)_{kl,ij}, so one density on
    both sides gives Jbra = Jket"""
    b = batch("(pp|ss)", 6, 1, seed=3)
    nab, _ = sizes(b)
    D = np.random.default_rng(2).standard_normal((6, nab))
    Jb, Jk = O.digest(b.basis, 4, b.bra, b.bra, D, D)
    assert np.allclose(Jb, Jk, rtol=1e-13, atol=1e-15)


def test_linear_in_the_density():
    b = batch("(ds|ps)", 4, 5, seed=4)
    nab, ncd = sizes(b)
    rng = np.random.default_rng(3)
    D1, D2 = rng.standard_normal((5, ncd)), rng.standard_normal((5, ncd))
    Db = rng.standard_normal((4, nab))
    a1, _ = O.digest(b.basis, 4, b.bra, b.ket, Db, D1)
    a2, _ = O.digest(b.basis, 4, b.bra, b.ket, Db, D2)
    a3, _ = O.digest(b.basis, 4, b.bra, b.ket, Db, 2.0 * D1 - D2)
    assert np.allclose(a3, 2.0 * a1 - a2, rtol=1e-12, atol=1e-14)
