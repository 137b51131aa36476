"""Integral parity, GPU vs CPU oracle: small classes (register kernel)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import workloads as W
from tests.gpu_util import assert_close

pytestmark = pytest.mark.gpu


def run(batch, cartesian=False):
    from paper_2506_12501_amd import native
    sh = native.DeviceShells(batch.basis)
    got = native.eri(sh, batch.ncentre, batch.bra, batch.ket, cartesian=cartesian).cpu().numpy()
    ref = O.eri(batch.basis, batch.ncentre, batch.bra, batch.ket, cartesian=cartesian)
    return got, ref


@pytest.mark.parametrize("name", W.C1_CLASSES + ["(sp|ss)", "(ss|sp)", "(ss|pp)", "(sp|ps)", "(ps|pp)"])
def test_config1_classes(name):
    got, ref = run(W.config1(name, npair=16, seed=3))
    assert_close(got, ref, name)


@pytest.mark.parametrize("name", ["(ds|ss)", "(ds|ps)", "(pd|ss)", "(dp|ps)", "(dd|ss)", "(ds|ds)", "(pp|ds)",
                                  "(dd|ps)", "(sd|dp)"])
@pytest.mark.parametrize("cart", [False, True])
def test_d_classes_contracted(name, cart):
    b = W.make_class_batch(name, 70, 5, 2, 6.0, 0.05, 50.0, 0.1, 1.0, seed=11)
    got, ref = run(b, cart)
    assert_close(got, ref, name)


@pytest.mark.parametrize("name", ["(s|ss)", "(p|ps)", "(d|pp)", "(s|dd)", "(p|dd)", "(d|ds)"])
def test_three_centre_small(name):
    b = W.make_class_batch(name, 67, 4, 3, 4.0, 0.1, 20.0, 0.1, 1.0, seed=5)
    got, ref = run(b)
    assert_close(got, ref, name)


@pytest.mark.parametrize("name", ["(s|s)", "(p|p)", "(d|d)", "(d|s)", "(f|f)", "(g|g)", "(f|d)"])
def test_two_centre(name):
    b = W.make_class_batch(name, 65, 6, 3, 4.0, 0.1, 20.0, 0.1, 1.0, seed=6)
    got, ref = run(b)
    assert_close(got, ref, name)


def test_cartesian_three_and_two_centre():
    for name in ["(p|dd)", "(d|ds)", "(p|p)"]:
        b = W.make_class_batch(name, 30, 3, 2, 4.0, 0.1, 20.0, 0.1, 1.0, seed=9)
        got, ref = run(b, cartesian=True)
        assert_close(got, ref, name)


def test_ragged_tail_and_single_pair():
    for nb, nk in [(1, 1), (63, 1), (65, 2), (129, 3)]:
        b = W.make_class_batch("(pp|ps)", nb, nk, 2, 5.0, 0.1, 30.0, 0.2, 1.0, seed=nb)
        got, ref = run(b)
        assert_close(got, ref, f"(pp|ps) {nb}x{nk}")
