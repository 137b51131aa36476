"""Every compiled kernel variant of a class must match the oracle (the
autotuner may pick any of them)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import workloads as W
from tests.gpu_util import assert_close

pytestmark = pytest.mark.gpu

# contraction degrees K give 9 (odd) or 4 ket primitives per pair, so the
# two-primitive sweep rounds meet a partial last round and full ones
CASES = [("(dd|dd)", 3), ("(pd|dd)", 3), ("(ff|ff)", 1), ("(gg|gg)", 1), ("(pp|pp)", 2), ("(dd|ps)", 2),
         ("(dd|pp)", 3), ("(dp|dp)", 2), ("(dp|ds)", 3), ("(f|dd)", 2), ("(f|dd)", 1), ("(i|dd)", 1),
         ("(pp|ps)", 3), ("(ds|pp)", 2), ("(ds|ds)", 3), ("(ds|ps)", 2), ("(dp|pp)", 3), ("(dp|ps)", 1),
         ("(dd|ds)", 3), ("(dd|dd)", 1)]


@pytest.mark.parametrize("name,K", CASES)
def test_all_variants_match_oracle(name, K):
    from paper_2506_12501_amd import autotune, native
    b = W.make_class_batch(name, 5, 3, K, 6.0, 0.05, 30.0, 0.1, 1.0, seed=31)
    ref = O.eri(b.basis, b.ncentre, b.bra, b.ket)
    ctx = native.Context.get(0)
    la, lb, lc, ld = W.parse_class(name)
    vs = autotune.variants(ctx, b.ncentre, la, lb, lc, ld, False)
    assert vs, name
    sh = native.DeviceShells(b.basis)
    L = native.lib()
    try:
        ran = 0
        for v in vs:
            native.check(L.mdx_set_variant(ctx.handle, b.ncentre, la, max(lb, 0), lc, max(ld, 0), 0, v), "variant")
            try:
                got = native.eri(sh, b.ncentre, b.bra, b.ket).cpu().numpy()
            except native.MdxError as e:   # 3-centre several-per-workgroup variants refuse contracted kets
                assert e.status == native.MDX_EUNSUPPORTED and K > 1 and name.startswith("(f|"), (name, v, e)
                continue
            assert_close(got, ref, f"{name} variant {v}")
            ran += 1
        assert ran > 0
    finally:
        L.mdx_set_variant(ctx.handle, b.ncentre, la, max(lb, 0), lc, max(ld, 0), 0, -1)


def test_unknown_variant_rejected():
    from paper_2506_12501_amd import native
    ctx = native.Context.get(0)
    st = native.lib().mdx_set_variant(ctx.handle, 4, 0, 0, 0, 0, 0, 17)
    assert st == native.MDX_EINVAL


def test_single_primitive_variants_take_contracted_pairs_by_expansion():
    """a contracted dense batch under a single-primitive variant runs once per
    primitive combination, accumulated; in a plan (ragged batch) it is refused"""
    from paper_2506_12501_amd import autotune, native
    b = W.make_class_batch("(ff|ff)", 3, 2, 2, 6.0, 0.05, 30.0, 0.1, 1.0, seed=32)
    ref = O.eri(b.basis, 4, b.bra, b.ket)
    ctx = native.Context.get(0)
    vs = autotune.variants(ctx, 4, 3, 3, 3, 3, False)
    sh = native.DeviceShells(b.basis)
    L = native.lib()
    try:
        native.check(L.mdx_set_variant(ctx.handle, 4, 3, 3, 3, 3, 0, vs[-1]), "variant")
        got = native.eri(sh, 4, b.bra, b.ket).cpu().numpy()
        assert_close(got, ref, "(ff|ff) K=2 single-primitive variant, expanded")
        with pytest.raises(native.MdxError) as e:
            native.Plan(sh, [native.Batch(4, b.bra, b.ket, np.array([3, 2], np.int32), 0)])
        assert e.value.status == native.MDX_EUNSUPPORTED
    finally:
        L.mdx_set_variant(ctx.handle, 4, 3, 3, 3, 3, 0, -1)


@pytest.mark.parametrize("name", ["(f|dd)", "(i|dd)"])
def test_three_centre_units_with_ragged_tails(name):
    """the several-functions-per-workgroup 3-centre kernels: 37 bra functions
    (units of 8 or 16 end in a partial unit) against 5 ket pairs, every variant"""
    from paper_2506_12501_amd import autotune, native
    b = W.make_class_batch(name, 37, 5, 1, 5.0, 0.1, 20.0, None, None, seed=33)
    ref = O.eri(b.basis, b.ncentre, b.bra, b.ket)
    ctx = native.Context.get(0)
    la, lb, lc, ld = W.parse_class(name)
    vs = autotune.variants(ctx, 3, la, 0, lc, ld, False)
    sh = native.DeviceShells(b.basis)
    L = native.lib()
    try:
        for v in vs:
            native.check(L.mdx_set_variant(ctx.handle, 3, la, 0, lc, ld, 0, v), "variant")
            assert_close(native.eri(sh, 3, b.bra, b.ket).cpu().numpy(), ref, f"{name} variant {v}")
    finally:
        L.mdx_set_variant(ctx.handle, 3, la, 0, lc, ld, 0, -1)
