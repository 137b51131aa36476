"""Digestion (the "consume" use of a batch): integrals contracted with
pair-blocked densities inside the kernels, through the C-ABI entry point
mdx_eri_digest_batch, against the oracle's contraction of its own batch."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import workloads as W
from tests.gpu_util import ATOL, RTOL

pytestmark = pytest.mark.gpu


def check(got, ref, scale, what):
    """J sums up to nket*ncd products that cancel; as for the contracted
    gradients: pass iff |err| <= 1e-12, or <= 1e-10 |ref|, or <= 1e-14 of
    the sum of the magnitudes of its terms"""
    err = np.abs(got - ref)
    ok = (err <= ATOL) | (err <= RTOL * np.abs(ref)) | (err <= 1e-14 * scale)
    assert ok.all(), f"{what}: {np.count_nonzero(~ok)} of {ok.size} off; worst {err.max():.3e}"


def run(b, cart=False, seed=0, sides=(True, True)):
    import torch
    from paper_2506_12501_amd import native
    la, lb, lc, ld = W.parse_class(b.name)
    nab = O.nfunc(la, cart) * (O.nfunc(lb, cart) if lb >= 0 else 1)
    ncd = O.nfunc(lc, cart) * (O.nfunc(ld, cart) if ld >= 0 else 1)
    rng = np.random.default_rng(seed)
    Db = rng.standard_normal((len(b.bra), nab))
    Dk = rng.standard_normal((len(b.ket), ncd))
    sh = native.DeviceShells(b.basis)
    Jb, Jk = native.eri_digest(sh, b.ncentre, b.bra, b.ket,
                               torch.as_tensor(Db, device="cuda") if sides[1] else None,
                               torch.as_tensor(Dk, device="cuda") if sides[0] else None, cartesian=cart)
    I = O.eri(b.basis, b.ncentre, b.bra, b.ket, cartesian=cart)   # [nbra, nab, ncd, nket]
    rb, rk = O.digest(b.basis, b.ncentre, b.bra, b.ket, Db, Dk, cartesian=cart)
    sb = np.einsum("iack,kc->ia", np.abs(I), np.abs(Dk))
    sk = np.einsum("iack,ia->kc", np.abs(I), np.abs(Db))
    if sides[0]:
        check(Jb.cpu().numpy(), rb, sb, b.name + " Jbra")
    else:
        assert Jb is None
    if sides[1]:
        check(Jk.cpu().numpy(), rk, sk, b.name + " Jket")
    else:
        assert Jk is None


@pytest.mark.parametrize("name", ["(ss|ss)", "(ps|ps)", "(pp|pp)", "(ds|ps)", "(pp|ds)", "(dd|ss)"])
def test_register_kernel_classes(name):
    """one lane per shellset; 70 bra pairs leave a ragged second wave"""
    run(W.make_class_batch(name, 70, 9, 2, 4.0, 0.1, 20.0, 0.1, 1.0, seed=3))


def test_swapped_orientation():
    """(ss|pp) runs with the ket pairs as the kernel's bra pairs"""
    run(W.make_class_batch("(ss|pp)", 33, 70, 2, 4.0, 0.1, 20.0, 0.1, 1.0, seed=4))
    run(W.make_class_batch("(ps|dd)", 9, 21, 2, 4.0, 0.1, 20.0, 0.1, 1.0, seed=5))


@pytest.mark.parametrize("name", ["(dd|dd)", "(pd|dd)", "(dd|pp)", "(dp|ds)"])
def test_matrix_core_classes(name):
    run(W.make_class_batch(name, 37, 19, 2, 4.0, 0.1, 20.0, 0.1, 1.0, seed=6))


@pytest.mark.parametrize("name", ["(ff|ff)", "(f|dd)"])
def test_single_primitive_classes_on_the_general_kernel(name):
    run(W.make_class_batch(name, 11, 7, 1, 4.0, 0.1, 20.0, 0.1, 1.0, seed=7))


@pytest.mark.parametrize("name", ["(p|p)", "(d|d)", "(f|d)", "(d|ds)"])
def test_two_and_three_centre(name):
    run(W.make_class_batch(name, 66, 5, 2, 4.0, 0.1, 20.0, 0.1, 1.0, seed=10))


def test_matrix_core_cartesian():
    run(W.make_class_batch("(dd|dd)", 9, 7, 1, 4.0, 0.1, 20.0, 0.1, 1.0, seed=11), cart=True)


def test_empty_batch_is_a_no_op():
    import torch
    from paper_2506_12501_amd import native
    b = W.make_class_batch("(pp|pp)", 3, 2, 1, 4.0, 0.1, 20.0, 0.1, 1.0, seed=12)
    Jb, Jk = native.eri_digest(native.DeviceShells(b.basis), 4, b.bra[:0], b.ket,
                               torch.zeros((0, 9), dtype=torch.float64, device="cuda"),
                               torch.ones((2, 9), dtype=torch.float64, device="cuda"))
    assert Jb.numel() == 0 and np.all(Jk.cpu().numpy() == 0.0)


def test_cartesian_and_one_side_only():
    b = W.make_class_batch("(dp|ps)", 40, 13, 2, 4.0, 0.1, 20.0, 0.1, 1.0, seed=8)
    run(b, cart=True)
    run(b, sides=(True, False))
    run(b, sides=(False, True))


def test_accumulates_and_checks_arguments():
    import torch
    from paper_2506_12501_amd import native
    b = W.make_class_batch("(pp|ps)", 20, 6, 1, 4.0, 0.1, 20.0, 0.1, 1.0, seed=9)
    sh = native.DeviceShells(b.basis)
    ctx = native.Context.get(0)
    L = native.lib()
    bra, ket = native._pairs(b.bra), native._pairs(b.ket)
    wsz = L.mdx_eri_workspace_size(ctx.handle, ctypes.byref(sh.struct), 4, 20, native._i32p(bra), 6,
                                   native._i32p(ket), 0)
    ws = torch.empty(wsz // 8 + 64, dtype=torch.float64, device="cuda")
    wsp = ctypes.c_void_p((ws.data_ptr() + 255) // 256 * 256)
    Db = torch.randn(9 * 20, dtype=torch.float64, device="cuda")
    Dk = torch.randn(3 * 6, dtype=torch.float64, device="cuda")
    Jb = torch.zeros(9 * 20, dtype=torch.float64, device="cuda")
    Jk = torch.zeros(3 * 6, dtype=torch.float64, device="cuda")
    args = (ctx.handle, ctypes.byref(sh.struct), 4, 20, native._i32p(bra), 6, native._i32p(ket), 0)
    for _ in range(2):
        assert L.mdx_eri_digest_batch(*args, Db.data_ptr(), Dk.data_ptr(), Jb.data_ptr(), Jk.data_ptr(), wsp, wsz,
                                      None) == native.MDX_OK
    torch.cuda.synchronize()
    once_b, once_k = native.eri_digest(sh, 4, b.bra, b.ket, Db.view(9, 20).t(), Dk.view(3, 6).t())
    assert np.allclose(Jb.view(9, 20).t().cpu().numpy(), 2 * once_b.cpu().numpy(), rtol=1e-12, atol=1e-13)
    assert np.allclose(Jk.view(3, 6).t().cpu().numpy(), 2 * once_k.cpu().numpy(), rtol=1e-12, atol=1e-13)
    assert L.mdx_eri_digest_batch(*args, Db.data_ptr(), None, Jb.data_ptr(), None, wsp, wsz,
                                  None) == native.MDX_EINVAL
    assert L.mdx_eri_digest_batch(*args, None, Dk.data_ptr(), None, Jk.data_ptr(), wsp, wsz,
                                  None) == native.MDX_EINVAL
