"""Paired batches (MDX_PAIRED): quartet q = (bra q, ket q), out[q + n*(ab +
nab*cd)], GPU vs CPU oracle through the C-ABI entry point mdx_eri_batch."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import workloads as W
from tests.gpu_util import assert_close

pytestmark = pytest.mark.gpu


def run(b, cart=False):
    from paper_2506_12501_amd import native
    sh = native.DeviceShells(b.basis)
    got = native.eri(sh, b.ncentre, b.bra, b.ket, cartesian=cart, paired=True).cpu().numpy()
    q = np.stack([np.arange(len(b.bra))] * 2, axis=1)
    ref = O.eri(b.basis, b.ncentre, b.bra, b.ket, cartesian=cart, quartets=q)   # [q, nab, ncd]
    assert_close(got, ref, b.name + " paired")


@pytest.mark.parametrize("name", ["(ss|ss)", "(pp|ps)", "(dd|ss)", "(ss|pp)"])
def test_register_kernel_one_quartet_per_lane(name):
    """130 quartets: two full waves and a ragged third; (ss|pp) runs swapped"""
    run(W.make_class_batch(name, 130, 130, 2, 4.0, 0.1, 20.0, 0.1, 1.0, seed=41))


@pytest.mark.parametrize("name", ["(dd|dd)", "(pd|dd)", "(dp|ps)"])
def test_matrix_core_one_quartet_per_workgroup(name):
    run(W.make_class_batch(name, 21, 21, 2, 4.0, 0.1, 20.0, 0.1, 1.0, seed=42))


@pytest.mark.parametrize("name", ["(ff|ff)", "(f|dd)", "(d|d)", "(p|dd)"])
def test_single_primitive_three_and_two_centre(name):
    run(W.make_class_batch(name, 9, 9, 1, 4.0, 0.1, 20.0, 0.1, 1.0, seed=43))


@pytest.mark.parametrize("name", ["(dd|dd)", "(pp|ps)"])
def test_cartesian(name):
    run(W.make_class_batch(name, 11, 11, 1, 4.0, 0.1, 20.0, 0.1, 1.0, seed=44), cart=True)


def test_errors():
    import torch
    from paper_2506_12501_amd import native
    b = W.make_class_batch("(pp|ps)", 5, 4, 1, 4.0, 0.1, 20.0, 0.1, 1.0, seed=45)
    sh = native.DeviceShells(b.basis)
    with pytest.raises(native.MdxError) as e:
        native.eri(sh, 4, b.bra, b.ket, paired=True)   # nbra != nket
    assert e.value.status == native.MDX_EINVAL
    L = native.lib()
    ctx = native.Context.get(0)
    bra, ket = native._pairs(b.bra[:4]), native._pairs(b.ket)
    ws = torch.empty(1 << 16, dtype=torch.float64, device="cuda")
    wsp = ctypes.c_void_p((ws.data_ptr() + 255) // 256 * 256)
    buf = torch.zeros(4096, dtype=torch.float64, device="cuda")
    args = (ctx.handle, ctypes.byref(sh.struct), 4, 4, native._i32p(bra), 4, native._i32p(ket), native.MDX_PAIRED)
    assert L.mdx_eri_digest_batch(*args, buf.data_ptr(), buf.data_ptr(), buf.data_ptr(), buf.data_ptr(), wsp,
                                  1 << 19, None) == native.MDX_EINVAL
    assert L.mdx_eri_grad_batch(*args, buf.data_ptr(), buf.data_ptr(), wsp, 1 << 19, None) == native.MDX_EINVAL
    torch.cuda.synchronize()
