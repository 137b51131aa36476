"""Independent numerical integration of primitive Cartesian ERIs (test helper).

Uses 1/r12 = (2/sqrt(pi)) int_0^inf exp(-s^2 r12^2) ds.  For fixed s the 6-D
integrand factorises over x, y, z into 2-D integrals of a polynomial times a
Gaussian, evaluated exactly by tensor Gauss-Hermite quadrature after
completing the square.  The s-integral uses Gauss-Legendre in u with
s = sqrt(rho) u / sqrt(1-u^2).  No Boys function, no recursion: it shares
nothing with the McMurchie-Davidson machinery it checks.
"""
import itertools
import math

import numpy as np

_GH = np.polynomial.hermite.hermgauss(12)
_GL = np.polynomial.legendre.leggauss(96)


def _axis_table(lmax, za, zb, zc, zd, A, B, C, D, s):
    """I[a,b,c,d,k] for one axis, all powers <= lmax, at s-nodes s[k]."""
    y, w = _GH
    nk = s.size
    out = np.zeros((lmax + 1,) * 4 + (nk,))
    for k in range(nk):
        s2 = s[k] ** 2
        M = np.array([[za + zb + s2, -s2], [-s2, zc + zd + s2]])
        bvec = np.array([za * A + zb * B, zc * C + zd * D])
        mu = np.linalg.solve(M, bvec)
        gamma = za * A * A + zb * B * B + zc * C * C + zd * D * D
        const = math.exp(-(gamma - bvec @ mu)) / math.sqrt(np.linalg.det(M))
        Lc = np.linalg.cholesky(M)
        Linv_T = np.linalg.inv(Lc.T)
        Y1, Y2 = np.meshgrid(y, y, indexing="ij")
        W = np.outer(w, w)
        X1 = mu[0] + Linv_T[0, 0] * Y1 + Linv_T[0, 1] * Y2
        X2 = mu[1] + Linv_T[1, 0] * Y1 + Linv_T[1, 1] * Y2
        pa = [(X1 - A) ** n for n in range(lmax + 1)]
        pb = [(X1 - B) ** n for n in range(lmax + 1)]
        pc = [(X2 - C) ** n for n in range(lmax + 1)]
        pd = [(X2 - D) ** n for n in range(lmax + 1)]
        for a, b, c, d in itertools.product(range(lmax + 1), repeat=4):
            out[a, b, c, d, k] = const * np.sum(W * pa[a] * pb[b] * pc[c] * pd[d])
    return out


def cart_list(l):
    return [(ax, ay, l - ax - ay) for ax in range(l, -1, -1) for ay in range(l - ax, -1, -1)]


def eri_prim_cart(la, lb, lc, ld, za, zb, zc, zd, A, B, C, D):
    """Primitive Cartesian [ab|cd] (unnormalised monomials), array [na,nb,nc,nd]."""
    p, q = za + zb, zc + zd
    rho = p * q / (p + q)
    u, wu = _GL
    u = 0.5 * (u + 1.0)
    wu = 0.5 * wu
    s = math.sqrt(rho) * u / np.sqrt(1 - u * u)
    jac = math.sqrt(rho) * (1 - u * u) ** -1.5
    lmax = max(la, lb, lc, ld)
    tabs = [_axis_table(lmax, za, zb, zc, zd, A[i], B[i], C[i], D[i], s) for i in range(3)]
    ca, cb, cc, cd = cart_list(la), cart_list(lb), cart_list(lc), cart_list(ld)
    out = np.zeros((len(ca), len(cb), len(cc), len(cd)))
    for ia, a in enumerate(ca):
        for ib, b in enumerate(cb):
            for ic, c in enumerate(cc):
                for id_, d in enumerate(cd):
                    f = np.ones_like(u)
                    for i in range(3):
                        f = f * tabs[i][a[i], b[i], c[i], d[i]]
                    out[ia, ib, ic, id_] = 2.0 / math.sqrt(math.pi) * np.sum(wu * jac * f)
    return out


def nuclear_prim_cart(la, lb, za, zb, A, B, C, nu=96):
    """Primitive Cartesian <a| 1/|r - C| |b> (unnormalised monomials, no sign),
    array [na, nb].  1/r = (2/sqrt(pi)) int_0^inf exp(-s^2 r^2) ds; for fixed s
    each axis is a 1-D integral of a polynomial times exp(-za x_A^2 - zb x_B^2
    - s^2 x_C^2), exact by Gauss-Hermite after completing the square.  The
    s-integral uses Gauss-Legendre in u with s = sqrt(p) u / sqrt(1 - u^2)."""
    y, w = _GH
    p = za + zb
    u, wu = np.polynomial.legendre.leggauss(nu)
    u = 0.5 * (u + 1.0)
    wu = 0.5 * wu
    s2 = p * u * u / (1 - u * u)
    jac = math.sqrt(p) * (1 - u * u) ** -1.5
    tabs = []
    for i in range(3):
        t = np.zeros((la + 1, lb + 1, nu))
        for k in range(nu):
            e = p + s2[k]
            M = (za * A[i] + zb * B[i] + s2[k] * C[i]) / e
            const = math.exp(-(za * A[i] ** 2 + zb * B[i] ** 2 + s2[k] * C[i] ** 2 - e * M * M)) / math.sqrt(e)
            x = M + y / math.sqrt(e)
            for a in range(la + 1):
                for b in range(lb + 1):
                    t[a, b, k] = const * np.sum(w * (x - A[i]) ** a * (x - B[i]) ** b)
        tabs.append(t)
    ca, cb = cart_list(la), cart_list(lb)
    out = np.zeros((len(ca), len(cb)))
    for ia, a in enumerate(ca):
        for ib, b in enumerate(cb):
            f = tabs[0][a[0], b[0]] * tabs[1][a[1], b[1]] * tabs[2][a[2], b[2]]
            out[ia, ib] = 2.0 / math.sqrt(math.pi) * np.sum(wu * jac * f)
    return out
