"""Pins for the oracle's integrals against mathematics that it does not share:
closed forms, quadrature, symbolic differentiation, invariances and a
quad-precision build of itself."""
import itertools
import math

import mpmath
import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import workloads as W
from tests import quadrature as Q

mpmath.mp.dps = 30


def one_quartet(ls, zs, cs, centers, Ks=None):
    """Basis with one contracted shell per centre; returns (basis, bra, ket)."""
    sb = W.ShellBuilder()
    idx = []
    for l, z, c, A in zip(ls, zs, cs, centers):
        idx.append(sb.add(A, l, np.atleast_1d(z), np.atleast_1d(c)))
    b = sb.basis()
    bra = np.array([[idx[0], idx[1] if len(idx) > 1 else -1]], dtype=np.int32)
    ket = np.array([[idx[2] if len(idx) > 2 else idx[-1], idx[3] if len(idx) > 3 else -1]], dtype=np.int32)
    return b, bra, ket


def cart_eri(ls, zs, centers, quad=False):
    b, bra, ket = one_quartet(ls, zs, [1.0] * 4, centers)
    return O.eri(b, 4, bra, ket, cartesian=True, quad=quad)[0, :, :, 0]


def boys_mp(m, x):
    x = mpmath.mpf(x)
    if x == 0:
        return mpmath.mpf(1) / (2 * m + 1)
    a = mpmath.mpf(m) + mpmath.mpf(1) / 2
    return mpmath.gammainc(a, 0, x) / (2 * x ** a)


# ---------------------------------------------------------------------------
# Hermite coefficients and overlaps
# ---------------------------------------------------------------------------
def test_paper_counts():
    # Sec. 2.1: 2l+1 solids and (l+1)(l+2)(l+3)/6 Hermites per shell;
    # Sec. 2.2.2: 6 of the 10 Hermites of a d shell are terminal (order 2);
    # Sec. 4.3: (hh|hh) needs 286^2 [p|q] per lane (L_bra = 10).
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")))
    for l, (ns, nh) in enumerate(zip(g["n_solid"], g["n_hermite"])):
        assert O.solid_coefs(l).shape[0] == ns
        assert sum((k + 1) * (k + 2) // 2 for k in range(l + 1)) == nh
    assert (2 + 1) * (2 + 2) // 2 == g["terminal_hermites_d"]
    assert (10 + 1) * (10 + 2) * (10 + 3) // 6 == g["hermites_l10"]
    assert g["hermites_l10"] ** 2 == g["pq_hh_hh"]


def test_terminal_E_closed_forms():
    rng = np.random.default_rng(3)
    for _ in range(20):
        la, lb = rng.integers(0, 5, 2)
        za, zb = np.exp(rng.uniform(-2, 3, 2))
        A, B = rng.uniform(-2, 2, 2)
        E = O.ecoef_1d(int(la), int(lb), za, zb, A, B)
        p = za + zb
        E00 = math.exp(-za * zb / p * (A - B) ** 2)
        assert E[0, 0, 0] == pytest.approx(E00, rel=1e-15)
        for i in range(la + 1):
            for j in range(lb + 1):
                # Eq. (17): E^{a+b}_{ab} = E^0_00 / (2 zeta_p)^{a+b}
                assert E[i, j, i + j] == pytest.approx(E00 / (2 * p) ** (i + j), rel=1e-13)
    # Eq. (16): one-centre E^a_a = (2 zeta_a)^{-a}; Eq. (13) parity holds for P = A
    E = O.ecoef_1d(5, 0, 0.7, 0.0, 0.3, 0.3)
    for i in range(6):
        assert E[i, 0, i] == pytest.approx((2 * 0.7) ** -i, rel=1e-14)
        for t in range(i + 1):
            if (t + i) % 2:
                assert E[i, 0, t] == 0.0


def test_E_second_index_parity_clause_is_false():
    # Eq. (15)'s parity clause would make E^0_{10} vanish; it is X_PA E^0_00
    za, zb, A, B = 1.0, 2.0, 0.0, 1.0
    E = O.ecoef_1d(1, 0, za, zb, A, B)
    p = za + zb
    XPA = (za * A + zb * B) / p - A
    assert E[1, 0, 0] == pytest.approx(XPA * math.exp(-za * zb / p * (A - B) ** 2), rel=1e-15)
    assert E[1, 0, 0] != 0.0


def test_overlap_vs_gauss_hermite():
    # 1-D overlaps int x_A^i x_B^j exp(-za x_A^2 - zb x_B^2) dx = E^0_ij sqrt(pi/p), Eq. (8)
    y, w = np.polynomial.hermite.hermgauss(30)
    rng = np.random.default_rng(5)
    for _ in range(10):
        za, zb = np.exp(rng.uniform(-1.5, 2, 2))
        A, B = rng.uniform(-1.5, 1.5, 2)
        p = za + zb
        P = (za * A + zb * B) / p
        x = P + y / math.sqrt(p)
        pref = math.exp(-za * zb / p * (A - B) ** 2) / math.sqrt(p)
        E = O.ecoef_1d(4, 4, za, zb, A, B)
        for i in range(5):
            for j in range(5):
                ref = pref * np.sum(w * (x - A) ** i * (x - B) ** j)
                assert E[i, j, 0] * math.sqrt(math.pi / p) == pytest.approx(ref, rel=1e-12, abs=1e-15)


def test_solid_harmonics_orthonormal():
    # same-centre overlap of the real solid harmonic Gaussians is diagonal with
    # the norm of x^l: pins the Cartesian->solid coefficients (Eqs. (18)-(19))
    for l in range(0, 7):
        z = 0.9
        S = O.overlap(l, l, [0.1, -0.2, 0.3], [0.1, -0.2, 0.3], [z], [1.0], [z], [1.0], cartesian=False)
        Sx = O.overlap(l, l, [0.1, -0.2, 0.3], [0.1, -0.2, 0.3], [z], [1.0], [z], [1.0], cartesian=True)
        ref = Sx[0, 0]  # x^l with itself
        assert np.allclose(S, ref * np.eye(2 * l + 1), rtol=0, atol=1e-13 * ref)


def test_solid_harmonics_low_l_explicit():
    s3 = math.sqrt(3.0)
    C1 = O.solid_coefs(1)  # m = -1, 0, 1 -> y, z, x
    assert np.allclose(C1, [[0, 1, 0], [0, 0, 1], [1, 0, 0]])
    C2 = O.solid_coefs(2)  # xx, xy, xz, yy, yz, zz
    ref = [[0, s3, 0, 0, 0, 0], [0, 0, 0, 0, s3, 0], [-0.5, 0, 0, -0.5, 0, 1],
           [0, 0, s3, 0, 0, 0], [s3 / 2, 0, 0, -s3 / 2, 0, 0]]
    assert np.allclose(C2, ref, atol=1e-15)


# ---------------------------------------------------------------------------
# (ss|ss), limits
# ---------------------------------------------------------------------------
def test_ssss_closed_form():
    rng = np.random.default_rng(7)
    for _ in range(30):
        zs = np.exp(rng.uniform(math.log(0.05), math.log(500), 4))
        cen = rng.uniform(0, 8, (4, 3))
        got = cart_eri([0, 0, 0, 0], zs, cen)[0, 0]
        za, zb, zc, zd = [mpmath.mpf(z) for z in zs]
        A, B, C, D = [[mpmath.mpf(v) for v in c] for c in cen]
        p, q = za + zb, zc + zd
        P = [(za * A[i] + zb * B[i]) / p for i in range(3)]
        Qc = [(zc * C[i] + zd * D[i]) / q for i in range(3)]
        Kab = mpmath.exp(-za * zb / p * sum((A[i] - B[i]) ** 2 for i in range(3)))
        Kcd = mpmath.exp(-zc * zd / q * sum((C[i] - D[i]) ** 2 for i in range(3)))
        rho = p * q / (p + q)
        T = rho * sum((P[i] - Qc[i]) ** 2 for i in range(3))
        ref = 2 * mpmath.pi ** 2.5 / (p * q * mpmath.sqrt(p + q)) * Kab * Kcd * boys_mp(0, T)
        assert got == pytest.approx(float(ref), rel=1e-14)


def test_one_centre_and_far_field_limits():
    z = [0.8, 1.3, 0.6, 2.1]
    c0 = np.zeros(3)
    got = cart_eri([0, 0, 0, 0], z, [c0] * 4)[0, 0]
    p, q = z[0] + z[1], z[2] + z[3]
    assert got == pytest.approx(2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q)), rel=1e-15)
    # far field: (ab|cd) -> S_ab S_cd / R for separated charge distributions
    R = 400.0
    cen = [c0, c0, np.array([0, 0, R]), np.array([0, 0, R])]
    got = cart_eri([0, 0, 0, 0], z, cen)[0, 0]
    Sab = (math.pi / p) ** 1.5
    Scd = (math.pi / q) ** 1.5
    assert got == pytest.approx(Sab * Scd / R, rel=1e-14)


# ---------------------------------------------------------------------------
# Quadrature of the defining integral, Eq. (3), for l <= 2 on every centre
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ls", [(0, 0, 0, 0), (1, 0, 0, 0), (1, 1, 1, 1), (2, 0, 1, 0), (2, 1, 2, 0),
                                (0, 2, 1, 2), (2, 2, 2, 2)])
def test_cartesian_vs_quadrature(ls):
    rng = np.random.default_rng(sum(ls) * 17 + ls[0])
    for trial in range(2):
        zs = np.exp(rng.uniform(math.log(0.2), math.log(4.0), 4))
        cen = rng.uniform(0, 2.0, (4, 3))
        got = cart_eri(list(ls), zs, cen)
        ref = Q.eri_prim_cart(*ls, *zs, *cen).reshape(got.shape)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(got - ref)) <= 1e-12 * scale, (ls, np.max(np.abs(got - ref)) / scale)


def test_three_and_two_centre_vs_quadrature():
    # unit partner shell: zeta = 0, monomial of degree 0
    rng = np.random.default_rng(11)
    for la, lc, ld in [(0, 0, 0), (2, 1, 1), (3, 2, 1), (1, 2, 2)]:
        zs = np.exp(rng.uniform(math.log(0.3), math.log(3.0), 3))
        cen = rng.uniform(0, 2.0, (3, 3))
        sb = W.ShellBuilder()
        a = sb.add(cen[0], la, [zs[0]], [1.0])
        c = sb.add(cen[1], lc, [zs[1]], [1.0])
        d = sb.add(cen[2], ld, [zs[2]], [1.0])
        b = sb.basis()
        got = O.eri(b, 3, [[a, -1]], [[c, d]], cartesian=True)[0, :, :, 0]
        ref = Q.eri_prim_cart(la, 0, lc, ld, zs[0], 0.0, zs[1], zs[2], cen[0], cen[0], cen[1], cen[2])
        ref = ref.reshape(got.shape)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
        got2 = O.eri(b, 2, [[a, -1]], [[c, -1]], cartesian=True)[0, :, :, 0]
        ref2 = Q.eri_prim_cart(la, 0, lc, 0, zs[0], 0.0, zs[1], 0.0, cen[0], cen[0], cen[1], cen[1])
        ref2 = ref2.reshape(got2.shape)
        assert np.max(np.abs(got2 - ref2)) <= 1e-12 * np.max(np.abs(ref2))


# ---------------------------------------------------------------------------
# Symbolic differentiation of the (ss|ss) closed form, low L
# ---------------------------------------------------------------------------
def _sympy_low_l(ls, zs, cen, comps):
    import sympy as sy

    class Fb(sy.Function):
        nargs = 2

        def fdiff(self, argindex=2):
            m, T = self.args
            return -Fb(m + 1, T)

    X = sy.symbols("Ax Ay Az Bx By Bz Cx Cy Cz Dx Dy Dz")
    Av, Bv, Cv, Dv = X[0:3], X[3:6], X[6:9], X[9:12]
    za, zb, zc, zd = [sy.Rational(str(z)) if False else sy.Float(z, 30) for z in zs]
    p, q = za + zb, zc + zd
    P = [(za * Av[i] + zb * Bv[i]) / p for i in range(3)]
    Qv = [(zc * Cv[i] + zd * Dv[i]) / q for i in range(3)]
    rho = p * q / (p + q)
    T = rho * sum((P[i] - Qv[i]) ** 2 for i in range(3))
    Kab = sy.exp(-za * zb / p * sum((Av[i] - Bv[i]) ** 2 for i in range(3)))
    Kcd = sy.exp(-zc * zd / q * sum((Cv[i] - Dv[i]) ** 2 for i in range(3)))
    G = 2 * sy.pi ** sy.Rational(5, 2) / (p * q * sy.sqrt(p + q)) * Kab * Kcd * Fb(0, T)
    subs = {X[i]: sy.Float(float(cen[i // 3][i % 3]), 30) for i in range(12)}
    zeta = [za, zb, zc, zd]
    out = []
    for comp in comps:
        # comp: for each centre, Cartesian powers (nx, ny, nz).
        # x_A^n e^{-z x_A^2} = sum_j n!/(2^n j!(n-2j)!) z^{-(n-j)} d^{n-2j}/dA^{n-2j} e^{...}
        terms = [(sy.Integer(1), [])]
        for ci in range(4):
            for ax in range(3):
                n = comp[ci][ax]
                if n == 0:
                    continue
                new = []
                for coef, ders in terms:
                    for j in range(n // 2 + 1):
                        c = sy.factorial(n) / (2 ** n * sy.factorial(j) * sy.factorial(n - 2 * j)) \
                            * zeta[ci] ** (-(n - j))
                        new.append((coef * c, ders + [X[3 * ci + ax]] * (n - 2 * j)))
                terms = new
        val = 0
        for coef, ders in terms:
            e = G
            for d in ders:
                e = sy.diff(e, d)
            val += coef * e
        val = val.subs(subs)
        val = val.replace(Fb, lambda m, t: sy.Float(str(boys_mp(int(m), float(t))), 30))
        out.append(float(sy.N(val, 25)))
    return out


@pytest.mark.parametrize("ls", [(1, 0, 0, 0), (1, 0, 1, 0), (1, 1, 0, 0), (1, 1, 1, 0), (1, 1, 1, 1),
                                (2, 0, 0, 0), (0, 0, 2, 1)])
def test_low_l_vs_symbolic_derivatives(ls):
    rng = np.random.default_rng(100 + sum(ls))
    zs = np.exp(rng.uniform(math.log(0.2), math.log(20), 4))
    cen = rng.uniform(0, 3.0, (4, 3))
    got = cart_eri(list(ls), zs, cen)
    cl = [Q.cart_list(l) for l in ls]
    nb, nc, nd = len(cl[1]), len(cl[2]), len(cl[3])
    allc = list(itertools.product(range(len(cl[0])), range(nb), range(nc), range(nd)))
    pick = allc if len(allc) <= 12 else [allc[i] for i in rng.choice(len(allc), 12, replace=False)]
    comps = [[cl[0][a], cl[1][b], cl[2][c], cl[3][d]] for a, b, c, d in pick]
    ref = _sympy_low_l(ls, zs, cen, comps)
    for (a, b, c, d), r in zip(pick, ref):
        g = got[a * nb + b, c * nd + d]
        assert abs(g - r) <= 1e-13 * max(1.0, abs(r)), (ls, a, b, c, d, g, r)


# ---------------------------------------------------------------------------
# Invariances
# ---------------------------------------------------------------------------
def _random_quartet_basis(rng, ls, K=2):
    sb = W.ShellBuilder()
    ids = []
    for l in ls:
        z = np.exp(rng.uniform(math.log(0.1), math.log(10), K))
        c = rng.uniform(0.2, 1.0, K) * W.prim_norm(z, l)
        ids.append(sb.add(rng.uniform(0, 4, 3), l, z, c))
    return sb.basis(), ids


def test_eightfold_symmetry():
    rng = np.random.default_rng(21)
    ls = (2, 1, 3, 0)
    b, (a, bb, c, d) = _random_quartet_basis(rng, ls)
    ref = O.eri(b, 4, [[a, bb]], [[c, d]])[0, :, :, 0]
    na, nb, nc, nd = [2 * l + 1 for l in ls]
    T = ref.reshape(na, nb, nc, nd)
    perms = {
        (bb, a, c, d): T.transpose(1, 0, 2, 3),
        (a, bb, d, c): T.transpose(0, 1, 3, 2),
        (c, d, a, bb): T.transpose(2, 3, 0, 1),
        (d, c, bb, a): T.transpose(3, 2, 1, 0),
    }
    for (s0, s1, s2, s3), exp in perms.items():
        got = O.eri(b, 4, [[s0, s1]], [[s2, s3]])[0, :, :, 0]
        assert np.allclose(got.reshape(exp.shape), exp, rtol=1e-13, atol=1e-15)


def test_schwarz_and_positive_semidefinite():
    rng = np.random.default_rng(22)
    sb = W.ShellBuilder()
    ids = []
    for l in [0, 1, 2, 1, 0, 2]:
        z = np.exp(rng.uniform(math.log(0.2), math.log(8), 2))
        ids.append(sb.add(rng.uniform(0, 3, 3), l, z, rng.uniform(0.3, 1, 2) * W.prim_norm(z, l)))
    b = sb.basis()
    # pair-indexed ERI matrix over all (ab) functions of a few pairs of mixed class
    pairs = [(ids[0], ids[1]), (ids[2], ids[3]), (ids[4], ids[5]), (ids[1], ids[2])]
    blocks = {}
    for i, pi in enumerate(pairs):
        for j, pj in enumerate(pairs):
            blocks[i, j] = O.eri(b, 4, [pi], [pj])[0, :, :, 0]
    sizes = [blocks[i, i].shape[0] for i in range(len(pairs))]
    M = np.block([[blocks[i, j] for j in range(len(pairs))] for i in range(len(pairs))])
    assert np.allclose(M, M.T, rtol=1e-12, atol=1e-14)
    assert np.linalg.eigvalsh(M).min() > -1e-12 * np.abs(M).max()
    for i in range(len(pairs)):
        for j in range(len(pairs)):
            Bij = blocks[i, j]
            di = np.sqrt(np.abs(np.diag(blocks[i, i])))
            dj = np.sqrt(np.abs(np.diag(blocks[j, j])))
            assert np.all(np.abs(Bij) <= np.outer(di, dj) * (1 + 1e-12) + 1e-15)


def test_scaling_homogeneity():
    # coordinates x lam, exponents x lam^-2 -> integrals x lam^(la+lb+lc+ld+5)
    rng = np.random.default_rng(23)
    ls = [2, 1, 1, 2]
    zs = np.exp(rng.uniform(-1, 1.5, 4))
    cen = rng.uniform(0, 2, (4, 3))
    lam = 1.7
    a = cart_eri(ls, zs, cen)
    bb = cart_eri(ls, zs / lam ** 2, cen * lam)
    assert np.allclose(bb, a * lam ** (sum(ls) + 5), rtol=1e-12, atol=1e-14 * np.abs(bb).max())


def _rotation(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def test_rotation_invariance_of_solid_shellsets():
    rng = np.random.default_rng(24)
    for ls in [(2, 1, 2, 2), (3, 0, 1, 2), (4, 2, 0, 1)]:
        b, ids = _random_quartet_basis(rng, ls)
        ref = O.eri(b, 4, [[ids[0], ids[1]]], [[ids[2], ids[3]]])[0, :, :, 0]
        Rm = _rotation(rng)
        b2 = W.Basis(b.xyz @ Rm.T, b.l, b.nprim, b.poff, b.exps, b.coefs)
        got = O.eri(b2, 4, [[ids[0], ids[1]]], [[ids[2], ids[3]]])[0, :, :, 0]
        assert np.linalg.norm(got) == pytest.approx(np.linalg.norm(ref), rel=1e-12)
        # per-shell norms too: the rotation acts orthogonally on each shell index
        assert np.allclose(np.sort(np.linalg.svd(got, compute_uv=False)),
                           np.sort(np.linalg.svd(ref, compute_uv=False)), rtol=1e-11, atol=1e-14)


def test_fp64_vs_quad_oracle():
    rng = np.random.default_rng(25)
    for name in ["(dd|dd)", "(pd|dd)", "(pp|pp)", "(ff|ps)"]:
        batch = W.make_class_batch(name, 3, 3, 2, 6.0, 0.05, 50.0, 0.1, 1.0, seed=int(rng.integers(1000)))
        d = O.eri(batch.basis, 4, batch.bra, batch.ket)
        q = O.eri(batch.basis, 4, batch.bra, batch.ket, quad=True)
        big = np.max(np.abs(q))
        for i in range(3):
            for k in range(3):
                # relative accuracy per shellset, except for shellsets whose
                # Gaussian-product prefactor exp(-mu R^2) underflows towards
                # 1e-200: exp(-x) in fp64 carries a relative error ~ x * eps
                blk = q[i, :, :, k]
                assert np.max(np.abs(d[i, :, :, k] - blk)) <= 5e-14 * np.max(np.abs(blk)) + 1e-16 * big


def test_contraction_is_linear_in_primitives():
    rng = np.random.default_rng(26)
    ls = (1, 2, 2, 0)
    b, ids = _random_quartet_basis(rng, ls, K=3)
    full = O.eri(b, 4, [[ids[0], ids[1]]], [[ids[2], ids[3]]])[0, :, :, 0]
    # split shell 1 into its primitives and sum
    total = np.zeros_like(full)
    for k in range(3):
        sb = W.ShellBuilder()
        new = []
        for s in range(4):
            o, K = b.poff[s], b.nprim[s]
            if s == ids[1]:
                new.append(sb.add(b.xyz[s], b.l[s], [b.exps[o + k]], [b.coefs[o + k]]))
            else:
                new.append(sb.add(b.xyz[s], b.l[s], b.exps[o:o + K], b.coefs[o:o + K]))
        bb = sb.basis()
        total += O.eri(bb, 4, [[new[0], new[1]]], [[new[2], new[3]]])[0, :, :, 0]
    assert np.allclose(total, full, rtol=1e-13, atol=1e-15)


def test_cluster_fp64_within_schwarz_scaled_bar():
    """The fp64 oracle against its __float128 build on the screened s/p batches
    of a small water-like cluster (exponents to 5000, K = 8 contractions, many
    one-centre quartets that vanish by symmetry): every element within 1e-12
    abs, 1e-10 rel, or 1e-12 Q_ab Q_cd -- the bar the GPU plans are held to,
    which therefore is one that fp64 evaluation can meet."""
    from paper_2506_12501_amd import screening as S
    import tests.cluster_util as T
    b, _ = W.water_cluster(seed=5, nx=2, ny=2, nz=2)
    P = S.canonical_pairs(b.l, 1)
    Q = {pc: T.oracle_Q(b, p) for pc, p in P.items()}
    bts = S.class_batches(P, Q, 1e-12)
    S.with_offsets(bts, b.l)
    assert [bt["name"] for bt in bts] == ["(ss|ss)", "(ps|ss)", "(ps|ps)", "(pp|ss)", "(pp|ps)", "(pp|pp)"]
    for bt in bts:
        ref, scale = T.oracle_batch(b, bt, quad=True)
        f64, _ = T.oracle_batch(b, bt, quad=False)
        T.assert_close_cs(f64, ref, scale, bt["name"])


def _abs_row_sums(l):
    """sum_k |C[m, k]| of each real solid harmonic's Cartesian expansion"""
    return np.abs(O.solid_coefs(l, quad=True)).sum(axis=1)


@pytest.mark.parametrize("name,nbra,nket", [("(gg|gg)", 3, 2), ("(hh|hh)", 2, 1), ("(ii|ii)", 1, 1),
                                            ("(g|dd)", 6, 5), ("(h|dd)", 6, 5), ("(i|dd)", 6, 5)])
def test_fp64_vs_quad_oracle_high_l(name, nbra, nket):
    """The fp64 oracle against its __float128 build (whose Cartesian-to-solid
    coefficients are formed in __float128 as well, Eqs. (18)-(19)) on high-L
    classes, primitive shells of the high-L workload (exponents 0.1..20, 4 A box).

    Cartesian: within 1e-13 of each shellset's largest element.  Solid: the
    transform sums Cartesian values of up to ~1e3 times the size of the solid
    result (the spherical part of an l = 6 shell far from the ket is a high
    multipole), so its fp64 rounding is bounded by the transform of the
    Cartesian magnitudes: per element |err| <= 4e-15 * prod_s (sum_k |C_s[m,k]|)
    * max|cart|.  The shellset-relative error is also held below 1e-10."""
    b = W.config4(name, nbra=nbra, nket=nket, seed=24)
    la, lb, lc, ld = W.parse_class(name)
    lb = max(lb, 0)
    cq = O.eri(b.basis, b.ncentre, b.bra, b.ket, cartesian=True, quad=True)
    c64 = O.eri(b.basis, b.ncentre, b.bra, b.ket, cartesian=True)
    cmax = np.abs(cq).max(axis=(1, 2))                               # [nbra, nket]
    assert np.all(np.abs(c64 - cq).max(axis=(1, 2)) <= 1e-13 * cmax), name
    sq = O.eri(b.basis, b.ncentre, b.bra, b.ket, quad=True)
    s64 = O.eri(b.basis, b.ncentre, b.bra, b.ket)
    rab = np.multiply.outer(_abs_row_sums(la), _abs_row_sums(lb)).reshape(-1)
    rcd = np.multiply.outer(_abs_row_sums(lc), _abs_row_sums(ld)).reshape(-1)
    bound = 4e-15 * rab[None, :, None, None] * rcd[None, None, :, None] * cmax[:, None, None, :]
    err = np.abs(s64 - sq)
    assert np.all(err <= bound), (name, float(np.max(err / bound)))
    smax = np.abs(sq).max(axis=(1, 2))
    rel = err.max(axis=(1, 2)) / smax
    assert rel.max() <= 1e-10, (name, float(rel.max()))
    print(name, "fp64 vs quad, solid: max err / shellset max %.2e" % rel.max())
