"""Overlap and kinetic-energy integrals (Sec. 2.1, Eq. (8)), GPU vs CPU oracle,
through the C-ABI entry point mdx_one_body_batch."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import workloads as W
from tests.cluster_util import assert_close_cs
from tests.gpu_util import assert_close

pytestmark = pytest.mark.gpu

LET = "spdf"


def run(basis, pairs, cart, quad=False, **kw):
    from paper_2506_12501_amd import native
    sh = native.DeviceShells(basis)
    S, T = native.one_body(sh, pairs, cartesian=cart, **kw)
    pairs = np.asarray(pairs)
    la, lb = int(basis.l[pairs[0, 0]]), int(basis.l[pairs[0, 1]])
    na, nb = O.nfunc(la, cart), O.nfunc(lb, cart)
    rs, rt = O.one_body(basis, pairs, cartesian=cart, quad=quad)

    def ref(x):   # [ij + npair*ab] -> [npair, na, nb]
        return x.reshape(na, nb, len(pairs)).transpose(2, 0, 1)
    return S, T, ref(rs), ref(rt)


def cs_scales(basis, pairs, cart):
    """sqrt(X_aa X_bb) per element, X = S and T: both operators are positive
    definite, so |X_ab| <= sqrt(X_aa X_bb) (Cauchy-Schwarz)"""
    la, lb = int(basis.l[pairs[0, 0]]), int(basis.l[pairs[0, 1]])
    na, nb = O.nfunc(la, cart), O.nfunc(lb, cart)
    out = []
    for k in range(2):
        da = O.one_body(basis, np.stack([pairs[:, 0]] * 2, 1), cartesian=cart)[k].reshape(na, na, -1)
        db = O.one_body(basis, np.stack([pairs[:, 1]] * 2, 1), cartesian=cart)[k].reshape(nb, nb, -1)
        ga = np.abs(np.einsum("iin->ni", da))
        gb = np.abs(np.einsum("jjn->nj", db))
        out.append(np.sqrt(ga[:, :, None] * gb[:, None, :]))
    return out


def check_cs(basis, pairs, cart, what):
    """Elements of tight contracted shells on one centre are sums of large
    primitive terms that cancel (exactly, when the integral vanishes by
    symmetry); the bar is the Cauchy-Schwarz-scaled one used for the cluster
    integrals, against the __float128 oracle."""
    S, T, rs, rt = run(basis, pairs, cart, quad=True)
    cs, ct = cs_scales(basis, pairs, cart)
    assert_close_cs(S.cpu().numpy().reshape(-1), rs.reshape(-1), cs.reshape(-1), "S " + what)
    assert_close_cs(T.cpu().numpy().reshape(-1), rt.reshape(-1), ct.reshape(-1), "T " + what)


def pair_batch(la, lb, npair, K, seed):
    b = W.make_class_batch(f"({LET[la]}{LET[lb]}|ss)", npair, 1, K, 6.0, 0.05, 50.0, 0.1, 1.0, seed=seed)
    return b.basis, b.bra


@pytest.mark.parametrize("la", [0, 1, 2, 3])
@pytest.mark.parametrize("lb", [0, 1, 2, 3])
@pytest.mark.parametrize("cart", [False, True])
def test_classes_contracted(la, lb, cart):
    basis, pairs = pair_batch(la, lb, 133, 3, seed=7 + 3 * la + lb)
    S, T, rs, rt = run(basis, pairs, cart)
    assert_close(S.cpu().numpy(), rs, f"S {la}{lb}")
    assert_close(T.cpu().numpy(), rt, f"T {la}{lb}")


@pytest.mark.parametrize("npair", [1, 63, 64, 65, 257])
def test_ragged_counts(npair):
    basis, pairs = pair_batch(2, 1, npair, 2, seed=npair)
    S, T, rs, rt = run(basis, pairs, False)
    assert_close(S.cpu().numpy(), rs, "S")
    assert_close(T.cpu().numpy(), rt, "T")


def test_same_shell_and_same_centre_pairs():
    """a = b (R = 0, the diagonal blocks) and distinct shells on one centre"""
    basis, atom = W.water_cluster(seed=2, nx=1, ny=2, nz=2)
    for la in range(3):
        for lb in range(3):
            pairs = np.array([(a, b) for a in range(len(basis.l)) for b in range(len(basis.l))
                              if basis.l[a] == la and basis.l[b] == lb and atom[a] == atom[b]], np.int32)
            if len(pairs) == 0:
                continue
            check_cs(basis, pairs, False, f"{la}{lb}")


def test_water_cluster_all_classes():
    """every shell pair of a 12-atom cut of the cluster workload (K up to 8,
    exponents up to 5000), grouped by class"""
    basis, _ = W.water_cluster(seed=0, nx=2, ny=2, nz=3)
    ns = len(basis.l)
    for la in range(3):
        for lb in range(3):
            pairs = np.array([(a, b) for a in range(ns) for b in range(ns)
                              if basis.l[a] == la and basis.l[b] == lb], np.int32)
            check_cs(basis, pairs, True, f"{la}{lb}")


def test_overlap_or_kinetic_alone():
    basis, pairs = pair_batch(1, 2, 70, 3, seed=4)
    S, T, rs, rt = run(basis, pairs, False, kinetic=False)
    assert T is None
    assert_close(S.cpu().numpy(), rs, "S alone")
    S, T, rs, rt = run(basis, pairs, False, overlap=False)
    assert S is None
    assert_close(T.cpu().numpy(), rt, "T alone")


def test_empty_batch():
    from paper_2506_12501_amd import native
    basis, pairs = pair_batch(1, 1, 4, 1, seed=1)
    S, T = native.one_body(native.DeviceShells(basis), pairs[:0])
    assert S.numel() == 0 and T.numel() == 0


def test_errors():
    from paper_2506_12501_amd import native
    b = W.make_class_batch("(gd|ss)", 3, 1, 1, 4.0, 0.1, 10.0, 0.1, 1.0, seed=1)
    b.basis.l[b.bra[:, 0]] = 7          # beyond the compiled l <= 6
    sh = native.DeviceShells(b.basis)
    with pytest.raises(native.MdxError) as e:
        native.one_body(sh, b.bra)
    assert e.value.status == native.MDX_EUNSUPPORTED
    mixed = np.array([[b.bra[0, 1], b.bra[1, 1]], [b.bra[0, 0], b.bra[1, 1]]], np.int32)
    with pytest.raises(native.MdxError) as e:
        native.one_body(sh, mixed)
    assert e.value.status == native.MDX_EINVAL
    bad = np.array([[0, len(b.basis.l)]], np.int32)
    with pytest.raises(native.MdxError) as e:
        native.one_body(sh, bad)
    assert e.value.status == native.MDX_EINVAL
