"""mdx_eri_batch_noalloc: the allocation-free form of mdx_eri_batch (its
workspace is a static device buffer of the library) against mdx_eri_batch on
the same inputs, two calls in a row with the second one smaller, through the
C ABI."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import workloads as W
from tests.gpu_util import assert_close

pytestmark = pytest.mark.gpu


def _both(batch, out_noalloc, cartesian=False):
    from paper_2506_12501_amd import native
    sh = native.DeviceShells(batch.basis)
    ref = native.eri(sh, batch.ncentre, batch.bra, batch.ket, cartesian=cartesian)
    got = native.eri_noalloc(sh, batch.ncentre, batch.bra, batch.ket, out_noalloc, cartesian=cartesian)
    return got.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("name,big,small", [("(dd|dd)", (40, 33), (7, 5)), ("(pp|pp)", (130, 70), (9, 3)),
                                            ("(f|dd)", (37, 20), (4, 2))])
def test_two_calls_match_the_workspace_entry_point(name, big, small):
    import torch
    b1 = W.make_class_batch(name, big[0], big[1], 3 if name == "(dd|dd)" else 1, 8.0, 0.05, 50.0, 0.1, 1.0,
                            seed=41)
    b2 = W.make_class_batch(name, small[0], small[1], 2 if name == "(dd|dd)" else 1, 5.0, 0.1, 30.0, 0.1, 1.0,
                            seed=42)
    out = torch.full((b1.bra.shape[0] * b1.ket.shape[0] * 625,), np.nan, dtype=torch.float64, device="cuda")
    g1, r1 = _both(b1, out)
    assert np.array_equal(g1, r1), name            # the same kernels on the same inputs
    out.fill_(np.nan)
    g2, r2 = _both(b2, out)                         # second, smaller call: scratch holds the first call's data
    assert np.array_equal(g2, r2), name
    assert_close(g2, O.eri(b2.basis, b2.ncentre, b2.bra, b2.ket), name)


def test_paired_and_cartesian_forms():
    import torch
    from paper_2506_12501_amd import native
    b = W.make_class_batch("(dp|dd)", 6, 6, 2, 6.0, 0.1, 30.0, 0.1, 1.0, seed=43)
    sh = native.DeviceShells(b.basis)
    out = torch.empty(6 * 18 * 36, dtype=torch.float64, device="cuda")
    got = native.eri_noalloc(sh, 4, b.bra, b.ket, out, cartesian=True, paired=True).cpu().numpy()
    ref = native.eri(sh, 4, b.bra, b.ket, cartesian=True, paired=True).cpu().numpy()
    assert np.array_equal(got, ref)


def test_batch_beyond_the_static_buffer_is_refused():
    """a workspace need above MDX_NOALLOC_SCRATCH_BYTES is refused before any
    launch, with the output untouched"""
    import torch
    from paper_2506_12501_amd import native
    b = W.make_class_batch("(dd|dd)", 1000, 1, 3, 8.0, 0.05, 50.0, 0.1, 1.0, seed=44)
    sh = native.DeviceShells(b.basis)
    L = native.lib()
    ctx = native.Context.get(0)
    bra, ket = native._pairs(b.bra), native._pairs(b.ket)
    wsz = L.mdx_eri_workspace_size(ctx.handle, ctypes.byref(sh.struct), 4, bra.shape[0], native._i32p(bra),
                                   ket.shape[0], native._i32p(ket), 0)
    assert wsz > native.MDX_NOALLOC_SCRATCH_BYTES, wsz
    out = torch.full((1000 * 625,), 7.0, dtype=torch.float64, device="cuda")
    st = L.mdx_eri_batch_noalloc(ctx.handle, ctypes.byref(sh.struct), 4, bra.shape[0], native._i32p(bra),
                                 ket.shape[0], native._i32p(ket), 0, native._ptr(out), native._stream(torch))
    assert st == native.MDX_EWORKSPACE
    assert "static buffer" in L.mdx_last_error().decode()
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))
