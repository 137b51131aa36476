"""Backward kernel parity (mdx_eri_grad_batch): twelve centre derivatives per
shellset contracted with an adjoint W, against
  - the oracle's analytic derivative integrals contracted with the same W,
  - central finite differences of the GPU forward integrals,
  - translational invariance (the four centres' derivatives sum to zero),
and the torch.autograd wrapper against the oracle.

Tolerance for a contracted sum g = sum_n W_n dI_n: pass iff |err| <= ATOL, or
<= RTOL |g|, or <= CTOL * sum_n |W_n dI_n|.  The last bound is the rounding
budget of a sum whose terms each carry a relative error of a few tens of
ulps (CTOL = 1e-14, about 90 ulps): cancellation in the sum can leave g far
below the size of its terms, where a bound relative to g alone is not
meaningful.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import workloads as W
from tests.gpu_util import ATOL, RTOL

pytestmark = pytest.mark.gpu

CTOL = 1e-14
ANG = W.ANGSTROM


def nfuncs(batch, cart):
    la, lb, lc, ld = W.parse_class(batch.name)
    f = lambda l: O.nfunc(l, cart) if l >= 0 else 1
    return f(la) * f(lb), f(lc) * f(ld)


def oracle_grad(batch, w, cart, quad=False):
    """reference g[ij, slot, kl] and its term scale sum |W dI|"""
    D = O.eri(batch.basis, batch.ncentre, batch.bra, batch.ket, cartesian=cart, deriv=True, quad=quad)
    nket, _, nbra, nab, ncd = D.shape
    Wf = w.reshape(nket, ncd, nab, nbra)
    g = np.einsum("kcai,kdiac->idk", Wf, D)
    s = np.einsum("kcai,kdiac->idk", np.abs(Wf), np.abs(D))
    return g, s


def gpu_grad(batch, w, cart, sh=None):
    import torch
    from paper_2506_12501_amd import native
    sh = sh or native.DeviceShells(batch.basis)
    wt = torch.as_tensor(w, device="cuda")
    return native.eri_grad(sh, batch.ncentre, batch.bra, batch.ket, wt, cartesian=cart).cpu().numpy()


def assert_grad_close(got, ref, scale, what):
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite values"
    err = np.abs(got - ref)
    ok = (err <= ATOL) | (err <= RTOL * np.abs(ref)) | (err <= CTOL * scale)
    if not ok.all():
        idx = np.unravel_index(np.argmax(np.where(ok, 0, err / np.maximum(scale, 1e-300))), err.shape)
        raise AssertionError(f"{what}: {np.count_nonzero(~ok)} of {ok.size} off; worst at {idx}: gpu {got[idx]!r} "
                             f"oracle {ref[idx]!r} scale {scale[idx]!r}")
    print(f"{what}: max err {err.max():.2e}, max err/scale {np.max(err / np.maximum(scale, 1e-300)):.2e}")


def check_class(batch, cart=False, seed=1, quad=False):
    nab, ncd = nfuncs(batch, cart)
    w = W.adjoint(batch, nab, ncd, seed=seed)
    ref, scale = oracle_grad(batch, w, cart, quad=quad)
    got = gpu_grad(batch, w, cart)
    assert_grad_close(got, ref, scale, f"{batch.name} {'cart' if cart else 'sph'}")
    return got, scale


@pytest.mark.parametrize("name,K", [("(ss|ss)", 2), ("(ps|ss)", 2), ("(ps|ps)", 1), ("(sp|ps)", 2), ("(pp|pp)", 2),
                                    ("(ds|sd)", 2), ("(dp|dp)", 2), ("(dd|pp)", 2), ("(pp|dd)", 1)])
def test_four_centre_small(name, K):
    b = W.make_class_batch(name, 5, 4, K, 6.0, 0.1, 30.0, 0.1, 1.0, seed=41)
    check_class(b)


@pytest.mark.parametrize("name", ["(dd|dd)", "(pd|dd)", "(dd|pd)"])
def test_config2_classes(name):
    # contracted K=3 shells with the distributions of the (dd|dd) benchmark
    b = W.make_class_batch(name, 4, 3, 3, 10.0, 0.05, 50.0, 0.1, 1.0, seed=42)
    check_class(b)


@pytest.mark.parametrize("name", ["(pp|pp)", "(dd|dd)", "(fs|pd)"])
def test_four_centre_cartesian(name):
    b = W.make_class_batch(name, 3, 3, 2, 6.0, 0.1, 30.0, 0.1, 1.0, seed=43)
    check_class(b, cart=True)


@pytest.mark.parametrize("name,K", [("(s|ss)", 2), ("(p|ps)", 2), ("(d|dd)", 1), ("(f|dd)", 3), ("(i|dd)", 1),
                                    ("(g|pp)", 2)])
def test_three_centre(name, K):
    b = W.make_class_batch(name, 5, 4, K, 5.0, 0.1, 20.0, 0.1, 1.0, seed=44)
    got, _ = check_class(b)
    assert np.all(got[:, 3:6, :] == 0.0)   # no second bra function


def test_three_centre_cartesian():
    b = W.make_class_batch("(f|dp)", 4, 3, 2, 5.0, 0.1, 20.0, 0.1, 1.0, seed=45)
    check_class(b, cart=True)


@pytest.mark.parametrize("name", ["(s|s)", "(p|d)", "(d|p)", "(g|d)", "(i|d)", "(f|f)"])
def test_two_centre(name):
    b = W.make_class_batch(name, 5, 4, 2, 5.0, 0.1, 20.0, 0.1, 1.0, seed=46)
    got, _ = check_class(b)
    assert np.all(got[:, 3:6, :] == 0.0) and np.all(got[:, 9:12, :] == 0.0)


def test_translational_invariance():
    # the two 4-centre passes are independent launches; their slots must cancel
    b = W.make_class_batch("(dp|pd)", 4, 4, 2, 6.0, 0.1, 30.0, 0.1, 1.0, seed=47)
    got, scale = check_class(b)
    tot = got[:, 0:3, :] + got[:, 3:6, :] + got[:, 6:9, :] + got[:, 9:12, :]
    s = scale[:, 0:3, :] + scale[:, 3:6, :] + scale[:, 6:9, :] + scale[:, 9:12, :]
    assert np.all(np.abs(tot) <= CTOL * s + ATOL)


def test_finite_difference():
    """central differences, h = 1e-4 A, of sum W (ab|cd) w.r.t. each shell centre
    coordinate, against the backward kernel summed over the shellsets that
    contain the shell"""
    import torch
    from paper_2506_12501_amd import native
    # compact geometry so that the derivatives are of order one
    b = W.make_class_batch("(dd|dd)", 2, 2, 3, 3.0, 0.1, 10.0, 0.1, 1.0, seed=48)
    nab, ncd = nfuncs(b, False)
    w = W.adjoint(b, nab, ncd, seed=1)
    sh = native.DeviceShells(b.basis)
    g = gpu_grad(b, w, False, sh)
    wt = torch.as_tensor(w, device="cuda")
    xyz0 = torch.as_tensor(np.asarray(b.basis.xyz, dtype=np.float64), device="cuda")

    def loss(xyz):
        out = native.eri(sh.with_center(xyz), 4, b.bra, b.ket)
        return float((out.permute(3, 2, 1, 0).reshape(-1) * wt).sum())

    h = 1e-4 * ANG
    nshell = xyz0.shape[0]
    fds, ans = [], []
    for s in range(nshell):
        for i in range(3):
            xp = xyz0.clone(); xp[s, i] += h
            xm = xyz0.clone(); xm[s, i] -= h
            fd = (loss(xp) - loss(xm)) / (2 * h)
            an = 0.0
            for X, (lst, col) in enumerate(((b.bra, 0), (b.bra, 1), (b.ket, 0), (b.ket, 1))):
                for p in range(lst.shape[0]):
                    if lst[p, col] == s:
                        an += g[p, 3 * X + i, :].sum() if X < 2 else g[:, 3 * X + i, p].sum()
            fds.append(fd)
            ans.append(an)
    fds, ans = np.array(fds), np.array(ans)
    # truncation error O(h^2 f3) at zeta <= 50: bound 1e-6 max|g| + 1e-9
    tol = 1e-6 * np.abs(ans).max() + 1e-9
    print(f"FD: max |g| {np.abs(ans).max():.3e}, max |fd - analytic| {np.abs(fds - ans).max():.2e}, tol {tol:.2e}")
    assert np.abs(ans).max() > 1e-3
    assert np.all(np.abs(fds - ans) <= tol), np.abs(fds - ans).max()


def test_autograd_function():
    import torch
    from paper_2506_12501_amd import native
    from paper_2506_12501_amd.autograd import ERIFunction
    b = W.make_class_batch("(pd|sp)", 3, 4, 2, 6.0, 0.1, 30.0, 0.1, 1.0, seed=49)
    nab, ncd = nfuncs(b, False)
    w = W.adjoint(b, nab, ncd, seed=3)
    ref, scale = oracle_grad(b, w, False)
    nshell = b.basis.xyz.shape[0]
    ref_c = np.zeros((nshell, 3))
    sc_c = np.zeros((nshell, 3))
    for X, (lst, col) in enumerate(((b.bra, 0), (b.bra, 1), (b.ket, 0), (b.ket, 1))):
        for p in range(lst.shape[0]):
            part = ref[p, 3 * X:3 * X + 3, :].sum(1) if X < 2 else ref[:, 3 * X:3 * X + 3, p].sum(0)
            spart = scale[p, 3 * X:3 * X + 3, :].sum(1) if X < 2 else scale[:, 3 * X:3 * X + 3, p].sum(0)
            ref_c[lst[p, col]] += part
            sc_c[lst[p, col]] += spart
    sh = native.DeviceShells(b.basis)
    center = torch.as_tensor(np.asarray(b.basis.xyz, dtype=np.float64), device="cuda").requires_grad_(True)
    out = ERIFunction.apply(center, sh, 4, b.bra, b.ket, False)
    wt = torch.as_tensor(w, device="cuda").reshape(b.ket.shape[0], ncd, nab, b.bra.shape[0]).permute(3, 2, 1, 0)
    (out * wt).sum().backward()
    assert_grad_close(center.grad.cpu().numpy(), ref_c, sc_c, "autograd (pd|sp)")


def test_full_size_sampled():
    """(dd|dd) 256 x 256 pairs, K=3, W ~ N(0,1) seed 1: every shellset computed
    on the GPU in one call; 48 sampled shellsets checked against the oracle"""
    b = W.config2("(dd|dd)")
    nab, ncd = nfuncs(b, False)
    w = W.adjoint(b, nab, ncd, seed=1)
    got = gpu_grad(b, w, False)
    nbra, nket = b.bra.shape[0], b.ket.shape[0]
    rng = np.random.default_rng(7)
    q = np.stack([rng.integers(0, nbra, 48), rng.integers(0, nket, 48)], axis=1)
    q[0] = (0, 0)
    q[1] = (nbra - 1, nket - 1)
    D = O.eri(b.basis, 4, b.bra, b.ket, quartets=q, deriv=True)   # [q, 12, ab, cd]
    Wf = w.reshape(nket, ncd, nab, nbra)
    for n, (i, k) in enumerate(q):
        wq = Wf[k, :, :, i]                                       # [cd, ab]
        ref = np.einsum("ca,dac->d", wq, D[n])
        sc = np.einsum("ca,dac->d", np.abs(wq), np.abs(D[n]))
        assert_grad_close(got[i, :, k], ref, sc, f"(dd|dd) shellset ({i},{k})")


def test_variants_agree():
    from paper_2506_12501_amd import autotune, native
    ctx = native.Context.get(0)
    b = W.make_class_batch("(dd|dd)", 3, 3, 3, 10.0, 0.05, 50.0, 0.1, 1.0, seed=50)
    nab, ncd = nfuncs(b, False)
    w = W.adjoint(b, nab, ncd, seed=1)
    ref, scale = oracle_grad(b, w, False)
    vs = autotune.variants(ctx, 4, 2, 2, 2, 2, False, gradient=True)
    assert len(vs) >= 2
    try:
        for v in vs:
            ctx.set_variant(4, 2, 2, 2, 2, native.MDX_GRADIENT, v)
            assert_grad_close(gpu_grad(b, w, False), ref, scale, f"(dd|dd) backward variant {v}")
    finally:
        ctx.set_variant(4, 2, 2, 2, 2, native.MDX_GRADIENT, -1)


# derivative sides of total order 5 and 6 (L' = l_d + l_w + 1 up to 13); the
# reference is the __float128 oracle, as for the forward integrals of l >= 4
HIGH = [("(ff|ff)", 1, 2, 2), ("(fd|dp)", 2, 3, 2), ("(gd|ps)", 1, 3, 2), ("(hp|ss)", 2, 2, 3), ("(is|pp)", 1, 2, 2),
        ("(gp|gp)", 1, 2, 2), ("(hs|dd)", 2, 2, 2)]


@pytest.mark.parametrize("name,K,nb,nk", HIGH, ids=[h[0] for h in HIGH])
def test_four_centre_high_order(name, K, nb, nk):
    b = W.make_class_batch(name, nb, nk, K, 5.0, 0.1, 20.0, 0.1, 1.0, seed=61)
    check_class(b, quad=True)


@pytest.mark.parametrize("name", ["(d|ff)", "(i|gd)", "(p|hp)"])
def test_three_centre_high_order(name):
    b = W.make_class_batch(name, 3, 2, 1, 5.0, 0.1, 20.0, 0.1, 1.0, seed=62)
    got, _ = check_class(b, quad=True)
    assert np.all(got[:, 3:6, :] == 0.0)


@pytest.mark.parametrize("name", ["(h|i)", "(i|i)", "(h|h)"])
def test_two_centre_high_order(name):
    b = W.make_class_batch(name, 3, 3, 2, 5.0, 0.1, 20.0, 0.1, 1.0, seed=63)
    got, _ = check_class(b, quad=True)
    assert np.all(got[:, 3:6, :] == 0.0) and np.all(got[:, 9:12, :] == 0.0)


@pytest.mark.parametrize("name", ["(fd|ss)", "(hp|ps)"])
def test_high_order_cartesian(name):
    # up to 64 Cartesian functions per pair: (fd) 60, (hp) 63
    b = W.make_class_batch(name, 2, 2, 1, 5.0, 0.1, 20.0, 0.1, 1.0, seed=64)
    check_class(b, cart=True, quad=True)


def test_unsupported_and_empty():
    from paper_2506_12501_amd import native
    # a Cartesian (ff) pair has 100 functions, beyond the 64 of the instances
    b = W.make_class_batch("(ff|ff)", 2, 2, 1, 5.0, 0.1, 20.0, None, None, seed=51)
    w = np.zeros(2 * 100 * 100 * 2)
    with pytest.raises(native.MdxError) as e:
        gpu_grad(b, w, True)
    assert e.value.status == native.MDX_EUNSUPPORTED
    e0 = W.make_class_batch("(dd|dd)", 0, 3, 1, 5.0, 0.1, 20.0, None, None, seed=52)
    assert gpu_grad(e0, np.zeros(0), False).size == 0
