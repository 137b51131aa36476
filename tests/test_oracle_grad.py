"""Pins for the oracle's centre derivatives (12 per shellset: A,B,C,D x x,y,z)."""
import math

import mpmath
import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import workloads as W

H_FD = 1e-4 * W.ANGSTROM   # 1e-4 Angstrom in bohr


def _batch(ls, K=2, seed=0, box=3.0):
    rng = np.random.default_rng(seed)
    sb = W.ShellBuilder()
    ids = []
    for l in ls:
        z = np.exp(rng.uniform(math.log(0.1), math.log(8), K))
        ids.append(sb.add(rng.uniform(0, box, 3), l, z, rng.uniform(0.2, 1, K) * W.prim_norm(z, l)))
    return sb.basis(), ids


@pytest.mark.parametrize("ls", [(0, 0, 0, 0), (1, 0, 1, 1), (2, 2, 2, 2), (3, 1, 2, 0)])
def test_grad_vs_central_differences(ls):
    b, ids = _batch(ls, seed=sum(ls))
    bra, ket = [[ids[0], ids[1]]], [[ids[2], ids[3]]]
    g = O.eri(b, 4, bra, ket, deriv=True)[0, :, 0]          # [12, nab, ncd]
    scale = np.max(np.abs(g))
    for X in range(4):
        for ax in range(3):
            fp = O.eri(b.moved(ids[X], ax, H_FD), 4, bra, ket)[0, :, :, 0]
            fm = O.eri(b.moved(ids[X], ax, -H_FD), 4, bra, ket)[0, :, :, 0]
            fd = (fp - fm) / (2 * H_FD)
            assert np.max(np.abs(fd - g[3 * X + ax])) <= 1e-6 * scale + 1e-9


def test_translational_invariance():
    for ls in [(2, 1, 2, 2), (4, 0, 1, 3)]:
        b, ids = _batch(ls, seed=7)
        g = O.eri(b, 4, [[ids[0], ids[1]]], [[ids[2], ids[3]]], deriv=True)[0, :, 0]
        for ax in range(3):
            s = g[ax] + g[3 + ax] + g[6 + ax] + g[9 + ax]
            assert np.max(np.abs(s)) <= 1e-12 * np.max(np.abs(g))


def test_ssss_gradient_closed_form():
    # d/dA_x of 2 pi^{5/2}/(pq sqrt(p+q)) K_AB K_CD F_0(T), symbolic in mpmath
    zs = [0.7, 1.9, 0.45, 3.3]
    rng = np.random.default_rng(3)
    cen = rng.uniform(0, 2.5, (4, 3))
    b, ids = W.ShellBuilder(), []
    for z, c in zip(zs, cen):
        ids.append(b.add(c, 0, [z], [1.0]))
    bas = b.basis()
    g = O.eri(bas, 4, [[ids[0], ids[1]]], [[ids[2], ids[3]]], deriv=True)[0, :, 0, 0, 0]
    mpmath.mp.dps = 30

    def value(*x):
        A, B, C, D = [x[3 * i:3 * i + 3] for i in range(4)]
        za, zb, zc, zd = [mpmath.mpf(z) for z in zs]
        p, q = za + zb, zc + zd
        P = [(za * A[i] + zb * B[i]) / p for i in range(3)]
        Q = [(zc * C[i] + zd * D[i]) / q for i in range(3)]
        Kab = mpmath.exp(-za * zb / p * sum((A[i] - B[i]) ** 2 for i in range(3)))
        Kcd = mpmath.exp(-zc * zd / q * sum((C[i] - D[i]) ** 2 for i in range(3)))
        T = p * q / (p + q) * sum((P[i] - Q[i]) ** 2 for i in range(3))
        F0 = mpmath.sqrt(mpmath.pi / (4 * T)) * mpmath.erf(mpmath.sqrt(T))
        return 2 * mpmath.pi ** 2.5 / (p * q * mpmath.sqrt(p + q)) * Kab * Kcd * F0

    x0 = [mpmath.mpf(float(v)) for v in cen.reshape(-1)]
    for k in range(12):
        d = mpmath.diff(lambda t: value(*(x0[:k] + [t] + x0[k + 1:])), x0[k])
        assert g[k] == pytest.approx(float(d), rel=1e-12, abs=1e-15)


def test_three_centre_gradient_fd():
    b, ids = _batch((3, 2, 1), seed=11)
    bra, ket = [[ids[0], -1]], [[ids[1], ids[2]]]
    g = O.eri(b, 3, bra, ket, deriv=True)[0, :, 0]
    assert np.all(g[3:6] == 0.0)           # B slot is the unit shell: no dependence
    scale = np.max(np.abs(g))
    for X, s in [(0, ids[0]), (2, ids[1]), (3, ids[2])]:
        for ax in range(3):
            fp = O.eri(b.moved(s, ax, H_FD), 3, bra, ket)[0, :, :, 0]
            fm = O.eri(b.moved(s, ax, -H_FD), 3, bra, ket)[0, :, :, 0]
            assert np.max(np.abs((fp - fm) / (2 * H_FD) - g[3 * X + ax])) <= 1e-6 * scale + 1e-9
