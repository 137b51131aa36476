"""1-particle integrals of shells with l = 4..6 (the classes of the paper's
Table 2 beyond f), GPU vs the __float128 oracle (the fp64 oracle's solid
transform of an l = 6 shell loses up to ~1e-11 of the block maximum), through
the C-ABI entry points: overlap and kinetic energy on the one-pair-per-wave
kernel; nuclear attraction on the lane kernel for l_a + l_b <= 6 and, beyond,
on the one-pair-per-wave kernel (lanes over Hermite columns)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import workloads as W
from tests.gpu_util import assert_close

pytestmark = pytest.mark.gpu

LET = "spdfghi"
HIGH = [(la, lb) for la in range(7) for lb in range(7) if max(la, lb) >= 4]


def pair_batch(la, lb, npair, K, seed):
    b = W.make_class_batch(f"({LET[la]}{LET[lb]}|ss)", npair, 1, K, 6.0, 0.05, 50.0, 0.1, 1.0, seed=seed)
    return b.basis, b.bra


def as_blocks(x, na, nb, n):   # [ij + n*ab] -> [n, na, nb]
    return np.asarray(x).reshape(na, nb, n).transpose(2, 0, 1)


@pytest.mark.parametrize("la,lb", HIGH)
@pytest.mark.parametrize("cart", [False, True])
def test_overlap_kinetic(la, lb, cart):
    from paper_2506_12501_amd import native
    basis, pairs = pair_batch(la, lb, 19, 3, seed=50 + 7 * la + lb)
    sh = native.DeviceShells(basis)
    S, T = native.one_body(sh, pairs, cartesian=cart)
    rs, rt = O.one_body(basis, pairs, cartesian=cart, quad=True)
    na, nb = O.nfunc(la, cart), O.nfunc(lb, cart)
    assert_close(S.cpu().numpy(), as_blocks(rs, na, nb, len(pairs)), f"S ({la}|{lb}) cart={cart}")
    assert_close(T.cpu().numpy(), as_blocks(rt, na, nb, len(pairs)), f"T ({la}|{lb}) cart={cart}")


def test_overlap_only_and_kinetic_only():
    from paper_2506_12501_amd import native
    basis, pairs = pair_batch(5, 3, 7, 2, seed=3)
    sh = native.DeviceShells(basis)
    rs, rt = O.one_body(basis, pairs, quad=True)
    S, _ = native.one_body(sh, pairs, kinetic=False)
    _, T = native.one_body(sh, pairs, overlap=False)
    assert_close(S.cpu().numpy(), as_blocks(rs, 11, 7, 7), "S alone")
    assert_close(T.cpu().numpy(), as_blocks(rt, 11, 7, 7), "T alone")


def _nuclear(basis, pairs, charges, cart):
    import torch
    from paper_2506_12501_amd import native
    sh = native.DeviceShells(basis)
    V = native.nuclear(sh, pairs, torch.as_tensor(charges, device="cuda"), cartesian=cart).cpu().numpy()
    la, lb = int(basis.l[pairs[0, 0]]), int(basis.l[pairs[0, 1]])
    ref = O.nuclear_batch(basis, pairs, charges, cartesian=cart, quad=True)
    return V, as_blocks(ref, O.nfunc(la, cart), O.nfunc(lb, cart), len(pairs))


def _charges(basis, pairs, n, seed):
    """random charges plus one on a shell centre, one on a product centre
    (Boys argument 0) and a far one (the asymptotic Boys branch)"""
    ch = W.point_charges(n, 6.0, seed=seed)
    a, b = pairs[0]
    za, zb = basis.exps[basis.poff[a]], basis.exps[basis.poff[b]]
    P = (za * basis.xyz[a] + zb * basis.xyz[b]) / (za + zb)
    extra = [[*basis.xyz[a], 3.0], [*P, 2.0], [*(basis.xyz[b] + 40.0), 5.0]]
    return np.ascontiguousarray(np.r_[ch, extra])


@pytest.mark.parametrize("la,lb", HIGH)
def test_nuclear_spherical(la, lb):
    basis, pairs = pair_batch(la, lb, 5, 2, seed=70 + 7 * la + lb)
    got, ref = _nuclear(basis, pairs, _charges(basis, pairs, 9, seed=la + 3 * lb), False)
    assert_close(got, ref, f"V ({la}|{lb})")


@pytest.mark.parametrize("la,lb", [(4, 0), (4, 4), (5, 1), (5, 3), (6, 2), (2, 6)])
def test_nuclear_cartesian(la, lb):
    basis, pairs = pair_batch(la, lb, 4, 2, seed=90 + 7 * la + lb)
    got, ref = _nuclear(basis, pairs, _charges(basis, pairs, 6, seed=la + 5 * lb), True)
    assert_close(got, ref, f"V ({la}|{lb}) Cartesian")


def test_nuclear_many_charges_in_slices():
    """150 charges on the one-pair-per-wave kernel (l_a + l_b >= 7)"""
    basis, pairs = pair_batch(4, 3, 3, 1, seed=5)
    got, ref = _nuclear(basis, pairs, _charges(basis, pairs, 147, seed=6), False)
    assert_close(got, ref, "V (g|f) 150 charges")


def test_nuclear_no_charges_gives_zero():
    import torch
    from paper_2506_12501_amd import native
    basis, pairs = pair_batch(5, 0, 70, 1, seed=2)
    sh = native.DeviceShells(basis)
    V = native.nuclear(sh, pairs, torch.zeros((0, 4), dtype=torch.float64, device="cuda"))
    assert bool(torch.all(V == 0.0))


@pytest.mark.parametrize("la,lb", [(6, 5), (6, 6)])
def test_nuclear_cartesian_largest(la, lb):
    """the largest Cartesian classes (588 and 784 functions per pair)"""
    basis, pairs = pair_batch(la, lb, 3, 2, seed=95 + la + lb)
    got, ref = _nuclear(basis, pairs, _charges(basis, pairs, 5, seed=la * lb), True)
    assert_close(got, ref, f"V ({la}|{lb}) Cartesian")


def test_l7_is_refused():
    import torch
    from paper_2506_12501_amd import native
    basis, pairs = pair_batch(2, 2, 1, 1, seed=1)
    basis.l[pairs[0, 0]] = 7
    sh = native.DeviceShells(basis)
    with pytest.raises(native.MdxError) as e:
        native.one_body(sh, pairs)
    assert e.value.status == native.MDX_EUNSUPPORTED
