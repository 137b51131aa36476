"""1-particle Coulomb (nuclear attraction) integrals with early summation over
charges (Eqs. (24), (26), (30), (34), (37)), GPU vs CPU oracle (which sums
charge by charge), through the C-ABI entry point mdx_nuclear_batch."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import workloads as W
from tests.cluster_util import assert_close_cs
from tests.gpu_util import assert_close

pytestmark = pytest.mark.gpu

LET = "spdfghi"


def run(basis, pairs, charges, cart, quad=False):
    import torch
    from paper_2506_12501_amd import native
    sh = native.DeviceShells(basis)
    ch = torch.as_tensor(charges, device="cuda")
    V = native.nuclear(sh, pairs, ch, cartesian=cart)
    pairs = np.asarray(pairs)
    la, lb = int(basis.l[pairs[0, 0]]), int(basis.l[pairs[0, 1]])
    na, nb = O.nfunc(la, cart), O.nfunc(lb, cart)
    ref = O.nuclear_batch(basis, pairs, charges, cartesian=cart, quad=quad)
    return V.cpu().numpy(), ref.reshape(na, nb, len(pairs)).transpose(2, 0, 1)


def pair_batch(la, lb, npair, K, seed):
    b = W.make_class_batch(f"({LET[la]}{LET[lb]}|ss)", npair, 1, K, 6.0, 0.05, 50.0, 0.1, 1.0, seed=seed)
    return b.basis, b.bra


def charges_with_edges(basis, pairs, n, seed):
    """random charges in the box plus charges on a shell centre, on the
    product centre of a pair's first primitives (Boys argument 0) and far
    away (the asymptotic Boys branch)"""
    ch = W.point_charges(n, 6.0, seed=seed)
    a, b = pairs[0]
    za, zb = basis.exps[basis.poff[a]], basis.exps[basis.poff[b]]
    P = (za * basis.xyz[a] + zb * basis.xyz[b]) / (za + zb)
    extra = [[*basis.xyz[a], 3.0], [*P, 2.0], [*(basis.xyz[b] + 40.0), 5.0]]
    return np.ascontiguousarray(np.r_[ch, extra])


@pytest.mark.parametrize("la", [0, 1, 2, 3])
@pytest.mark.parametrize("lb", [0, 1, 2, 3])
@pytest.mark.parametrize("cart", [False, True])
def test_classes_contracted(la, lb, cart):
    basis, pairs = pair_batch(la, lb, 67, 3, seed=21 + 3 * la + lb)
    ch = charges_with_edges(basis, pairs, 100, seed=la + 5 * lb)
    got, ref = run(basis, pairs, ch, cart)
    assert_close(got, ref, f"V {la}{lb}")


# shells of l = 4..6 in classes with l_a + l_b <= 6 run on the lane kernel too
LANE_HIGH = [(la, lb) for la in range(7) for lb in range(7) if max(la, lb) >= 4 and la + lb <= 6]


@pytest.mark.parametrize("la,lb", LANE_HIGH)
def test_lane_classes_with_a_high_shell(la, lb):
    """65 pairs (a full wave and a ragged one), K = 2, 40 charges plus the edge
    charges, against the __float128 oracle (the fp64 oracle's solid transform
    of an l >= 5 shell is not accurate to the bar)"""
    basis, pairs = pair_batch(la, lb, 65, 2, seed=41 + 7 * la + lb)
    ch = charges_with_edges(basis, pairs, 40, seed=la + 7 * lb)
    got, ref = run(basis, pairs, ch, False, quad=True)
    assert_close(got, ref, f"V {la}{lb}")


@pytest.mark.parametrize("la,lb", [(4, 2), (0, 6)])
def test_lane_classes_with_a_high_shell_cartesian(la, lb):
    basis, pairs = pair_batch(la, lb, 65, 2, seed=43 + 7 * la + lb)
    ch = charges_with_edges(basis, pairs, 40, seed=la + 5 * lb)
    got, ref = run(basis, pairs, ch, True, quad=True)
    assert_close(got, ref, f"V {la}{lb} Cartesian")


@pytest.mark.parametrize("npair", [1, 64, 65, 130])
def test_ragged_counts(npair):
    basis, pairs = pair_batch(2, 1, npair, 2, seed=npair)
    got, ref = run(basis, pairs, W.point_charges(9, 6.0, seed=npair), False)
    assert_close(got, ref, "V")


def test_no_charges_gives_zero():
    basis, pairs = pair_batch(1, 1, 70, 1, seed=2)
    got, ref = run(basis, pairs, np.zeros((0, 4)), False)
    assert np.all(got == 0.0) and np.all(ref == 0.0)


def test_water_cluster_cut_with_nuclear_charges():
    """every l <= 2 shell pair of a 12-atom cut of the cluster workload (K up
    to 8, exponents to 5000) in the field of its nuclei (8 on heavy atoms, 1
    on light ones).  -V is positive definite for positive charges, so the
    Cauchy-Schwarz-scaled bar of the cluster integrals applies, with
    sqrt(V_aa V_bb), against the __float128 oracle."""
    basis, atom = W.water_cluster(seed=0, nx=2, ny=2, nz=3)
    ns = len(basis.l)
    first = [int(np.flatnonzero(atom == k)[0]) for k in range(atom.max() + 1)]
    ch = np.array([[*basis.xyz[s], 8.0 if k % 3 == 0 else 1.0] for k, s in enumerate(first)])
    for la in range(3):
        for lb in range(la + 1):
            pairs = np.array([(a, b) for a in range(ns) for b in range(ns)
                              if basis.l[a] == la and basis.l[b] == lb], np.int32)
            got, ref = run(basis, pairs, ch, False, quad=True)
            na, nb = O.nfunc(la, False), O.nfunc(lb, False)
            da = O.nuclear_batch(basis, np.stack([pairs[:, 0]] * 2, 1), ch).reshape(na, na, -1)
            db = O.nuclear_batch(basis, np.stack([pairs[:, 1]] * 2, 1), ch).reshape(nb, nb, -1)
            ga = np.abs(np.einsum("iin->ni", da))
            gb = np.abs(np.einsum("jjn->nj", db))
            scale = np.sqrt(ga[:, :, None] * gb[:, None, :])
            assert_close_cs(got.reshape(-1), ref.reshape(-1), scale.reshape(-1), f"V {la}{lb}")


def test_errors():
    import torch
    from paper_2506_12501_amd import native
    b = W.make_class_batch("(gd|ss)", 3, 1, 1, 4.0, 0.1, 10.0, 0.1, 1.0, seed=1)
    b.basis.l[b.bra[:, 0]] = 7          # beyond the compiled l <= 6
    sh = native.DeviceShells(b.basis)
    ch = torch.as_tensor(W.point_charges(4, seed=1), device="cuda")
    with pytest.raises(native.MdxError) as e:
        native.nuclear(sh, b.bra, ch)
    assert e.value.status == native.MDX_EUNSUPPORTED
    L = native.lib()
    ctx = native.Context.get(0)
    pairs = native._pairs(b.bra[:, 1:].repeat(2, axis=1))   # (d|d) pairs
    ws = torch.empty(1024, dtype=torch.float64, device="cuda")
    V = torch.empty(3 * 25, dtype=torch.float64, device="cuda")
    wsp = ctypes.c_void_p((ws.data_ptr() + 255) // 256 * 256)
    args = (ctx.handle, ctypes.byref(sh.struct), 3, native._i32p(pairs))
    assert L.mdx_nuclear_batch(*args, -1, ch.data_ptr(), 0, V.data_ptr(), wsp, 4096, None) == native.MDX_EINVAL
    assert L.mdx_nuclear_batch(*args, 4, None, 0, V.data_ptr(), wsp, 4096, None) == native.MDX_EINVAL
    assert L.mdx_nuclear_batch(*args, 4, ch.data_ptr(), 0, None, wsp, 4096, None) == native.MDX_EINVAL
    assert L.mdx_nuclear_batch(*args, 4, ch.data_ptr(), 0, V.data_ptr(), wsp, 8, None) == native.MDX_EWORKSPACE
    assert L.mdx_nuclear_batch(*args, 4, ch.data_ptr(), 0, V.data_ptr(), wsp, 4096, None) == native.MDX_OK
    torch.cuda.synchronize()
