"""Register kernel of the classes whose shellsets do not fit a lane's
registers: the kernel takes their ket functions in parts (the primitive loops
run once per part).  Forced onto the register kernel (variant 0) and compared
with the CPU oracle, element by element, on ragged batches of contracted
shells."""
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import workloads as W
from tests.gpu_util import assert_close

pytestmark = pytest.mark.gpu

# (class, Cartesian): 4-centre (dp|pp), (dd|ds) spherical and Cartesian,
# (dp|ds) and (dd|ps) Cartesian; 3-centre (d|dd) and Cartesian (p|dd);
# 2-centre (g|g)
CASES = [("(dp|pp)", False), ("(dd|ds)", False), ("(dp|pp)", True), ("(dd|ds)", True), ("(dp|ds)", True),
         ("(dd|ps)", True), ("(d|dd)", False), ("(p|dd)", True), ("(g|g)", False)]


@pytest.mark.parametrize("name,cart", CASES)
def test_register_kernel_in_parts(name, cart):
    from paper_2506_12501_amd import native
    ctx = native.Context.get(0)
    la, lb, lc, ld = W.parse_class(name)
    b = W.make_class_batch(name, 67, 5, 2, 5.0, 0.05, 50.0, 0.1, 1.0, seed=17)
    ctx.set_variant(b.ncentre, la, max(lb, 0), lc, max(ld, 0), cart, 0)
    try:
        sh = native.DeviceShells(b.basis)
        got = native.eri(sh, b.ncentre, b.bra, b.ket, cartesian=cart).cpu().numpy()
    finally:
        ctx.set_variant(b.ncentre, la, max(lb, 0), lc, max(ld, 0), cart, -1)
    ref = O.eri(b.basis, b.ncentre, b.bra, b.ket, cartesian=cart)
    assert_close(got, ref, f"{name} {'Cartesian' if cart else 'spherical'}, register kernel")
