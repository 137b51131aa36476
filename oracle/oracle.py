"""ctypes front end of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module.  It loads ``liboracle_f64.so`` (fp64) or ``liboracle_q.so``
(``__float128`` internally, fp64 in/out), both built from ``mdx_oracle.c``
by ``oracle/build.py``.  Nothing here touches the GPU library.

Output layouts (see mdx_oracle.c):
  dense  : out[ij + nbra*(ab + nab*(cd + ncd*kl))]  (Fortran order
           [nbra, nab, ncd, nket] in numpy terms)
  list   : out[q, ab, cd]
  deriv  : dense -> [nket, 12, nbra]-major blocks of [nab, ncd] (see below),
           list  -> [q, 12, ab, cd]
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

_libs: dict = {}

_c_int = ctypes.c_int
_p_d = ctypes.POINTER(ctypes.c_double)
_p_i = ctypes.POINTER(ctypes.c_int)


def _load(quad: bool = False):
    key = "q" if quad else "f64"
    if key in _libs:
        return _libs[key]
    path = os.path.join(HERE, f"liboracle_{key}.so")
    if not os.path.exists(path):
        raise RuntimeError(f"oracle library {path} is not built; run oracle/build.py")
    lib = ctypes.CDLL(path)
    pre = "mdx_oracle_q_" if quad else "mdx_oracle_"
    fns = {}
    f = getattr(lib, pre + "boys")
    f.argtypes = [_c_int, _p_d, _c_int, _p_d]
    f.restype = None
    fns["boys"] = f
    f = getattr(lib, pre + "solid_coefs")
    f.argtypes = [_c_int, _p_d]
    f.restype = None
    fns["solid_coefs"] = f
    f = getattr(lib, pre + "ecoef_1d")
    f.argtypes = [_c_int, _c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                  ctypes.c_double, _p_d]
    f.restype = None
    fns["ecoef_1d"] = f
    f = getattr(lib, pre + "overlap")
    f.argtypes = [_c_int, _c_int, _p_d, _p_d, _c_int, _c_int, _p_d, _p_d, _p_d, _p_d, _c_int, _p_d]
    f.restype = None
    fns["overlap"] = f
    f = getattr(lib, pre + "kinetic")
    f.argtypes = [_c_int, _c_int, _p_d, _p_d, _c_int, _c_int, _p_d, _p_d, _p_d, _p_d, _c_int, _p_d]
    f.restype = None
    fns["kinetic"] = f
    f = getattr(lib, pre + "nuclear")
    f.argtypes = [_c_int, _c_int, _p_d, _p_d, _c_int, _c_int, _p_d, _p_d, _p_d, _p_d, _c_int, _p_d, _c_int,
                  _p_d]
    f.restype = None
    fns["nuclear"] = f
    f = getattr(lib, pre + "eri")
    f.argtypes = [_c_int, _c_int, _p_d, _p_i, _p_i, _p_i, _p_d, _p_d, _c_int, _p_i, _c_int, _p_i,
                  _c_int, _p_i, _c_int, _c_int, _p_d]
    f.restype = _c_int
    fns["eri"] = f
    _libs[key] = fns
    return fns


def _dp(a):
    return a.ctypes.data_as(_p_d)


def _ip(a):
    return a.ctypes.data_as(_p_i)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def boys(x, mmax: int, quad: bool = False) -> np.ndarray:
    """F[m, i] = F_m(x[i]) for m = 0..mmax."""
    x = _f64(np.atleast_1d(x))
    out = np.zeros((mmax + 1, x.size))
    _load(quad)["boys"](x.size, _dp(x), mmax, _dp(out))
    return out


def solid_coefs(l: int, quad: bool = False) -> np.ndarray:
    """C[m+l, cart]: coefficient of the Cartesian monomial in S_lm."""
    nc = (l + 1) * (l + 2) // 2
    out = np.zeros((2 * l + 1, nc))
    _load(quad)["solid_coefs"](l, _dp(out))
    return out


def ecoef_1d(la: int, lb: int, za: float, zb: float, A: float, B: float, quad: bool = False):
    """E[i, j, t] (1-D Hermite coefficients including exp(-mu X_AB^2))."""
    out = np.zeros((la + 1, lb + 1, la + lb + 1))
    _load(quad)["ecoef_1d"](la, lb, za, zb, A, B, _dp(out))
    return out


def overlap(la, lb, A, B, za, ca, zb, cb, cartesian=True, quad=False) -> np.ndarray:
    A = _f64(A); B = _f64(B)
    za = _f64(np.atleast_1d(za)); ca = _f64(np.atleast_1d(ca))
    zb = _f64(np.atleast_1d(zb)); cb = _f64(np.atleast_1d(cb))
    na = (la + 1) * (la + 2) // 2 if cartesian else 2 * la + 1
    nb = (lb + 1) * (lb + 2) // 2 if cartesian else 2 * lb + 1
    out = np.zeros((na, nb))
    _load(quad)["overlap"](la, lb, _dp(A), _dp(B), za.size, zb.size, _dp(za), _dp(ca), _dp(zb),
                           _dp(cb), int(cartesian), _dp(out))
    return out


def kinetic(la, lb, A, B, za, ca, zb, cb, cartesian=True, quad=False) -> np.ndarray:
    """-1/2 <a|nabla^2|b> of two contracted shells (Laplacian on the ket)."""
    A = _f64(A); B = _f64(B)
    za = _f64(np.atleast_1d(za)); ca = _f64(np.atleast_1d(ca))
    zb = _f64(np.atleast_1d(zb)); cb = _f64(np.atleast_1d(cb))
    na = (la + 1) * (la + 2) // 2 if cartesian else 2 * la + 1
    nb = (lb + 1) * (lb + 2) // 2 if cartesian else 2 * lb + 1
    out = np.zeros((na, nb))
    _load(quad)["kinetic"](la, lb, _dp(A), _dp(B), za.size, zb.size, _dp(za), _dp(ca), _dp(zb),
                           _dp(cb), int(cartesian), _dp(out))
    return out


def nuclear(la, lb, A, B, za, ca, zb, cb, charges, cartesian=True, quad=False) -> np.ndarray:
    """-sum_I q_I <a| 1/|r - I| |b> of two contracted shells; charges [n, 4]
    rows (x, y, z, q) -- Eqs. (24), (26), (30), (34), charge by charge."""
    A = _f64(A); B = _f64(B)
    za = _f64(np.atleast_1d(za)); ca = _f64(np.atleast_1d(ca))
    zb = _f64(np.atleast_1d(zb)); cb = _f64(np.atleast_1d(cb))
    ch = _f64(np.asarray(charges, dtype=np.float64).reshape(-1, 4))
    na = (la + 1) * (la + 2) // 2 if cartesian else 2 * la + 1
    nb = (lb + 1) * (lb + 2) // 2 if cartesian else 2 * lb + 1
    out = np.zeros((na, nb))
    _load(quad)["nuclear"](la, lb, _dp(A), _dp(B), za.size, zb.size, _dp(za), _dp(ca), _dp(zb), _dp(cb),
                           ch.shape[0], _dp(ch), int(cartesian), _dp(out))
    return out


def nuclear_batch(basis, pairs, charges, cartesian: bool = False, quad: bool = False):
    """1-particle Coulomb integrals of a batch of shell pairs (same class) in
    the field of the point charges, out[ij + npair*ab] (the library's layout)."""
    pairs = np.asarray(pairs)
    la, lb = int(basis.l[pairs[0, 0]]), int(basis.l[pairs[0, 1]])
    na, nb = nfunc(la, cartesian), nfunc(lb, cartesian)
    V = np.zeros((na * nb, len(pairs)))
    for ij, (a, b) in enumerate(pairs):
        sa = slice(basis.poff[a], basis.poff[a] + basis.nprim[a])
        sb = slice(basis.poff[b], basis.poff[b] + basis.nprim[b])
        V[:, ij] = nuclear(la, lb, basis.xyz[a], basis.xyz[b], basis.exps[sa], basis.coefs[sa], basis.exps[sb],
                           basis.coefs[sb], charges, cartesian=cartesian, quad=quad).reshape(-1)
    return V.reshape(-1)


def digest(basis, ncentre: int, bra, ket, Dbra, Dket, cartesian: bool = False, quad: bool = False):
    """Contraction of a dense batch with pair-blocked densities (the "consume"
    use of the integrals, Sec. 3.1):
        Jbra[ij, ab] = sum_{kl, cd} (ab|cd)_{ij,kl} Dket[kl, cd]
        Jket[kl, cd] = sum_{ij, ab} (ab|cd)_{ij,kl} Dbra[ij, ab]
    Dbra [nbra, nab], Dket [nket, ncd] (row = pair); returns (Jbra, Jket) in
    the same shapes.  The integrals are this module's eri(); the contraction
    is a plain tensor sum."""
    I = eri(basis, ncentre, bra, ket, cartesian=cartesian, quad=quad)   # [nbra, nab, ncd, nket]
    Jbra = np.einsum("iack,kc->ia", I, np.asarray(Dket, dtype=np.float64))
    Jket = np.einsum("iack,ia->kc", I, np.asarray(Dbra, dtype=np.float64))
    return Jbra, Jket


def one_body(basis, pairs, cartesian: bool = False, quad: bool = False):
    """Overlap and kinetic integrals of a batch of shell pairs (same class),
    out[ij + npair*ab] with ab = a*nfunc(lb) + b (the library's layout)."""
    pairs = np.asarray(pairs)
    la, lb = int(basis.l[pairs[0, 0]]), int(basis.l[pairs[0, 1]])
    na, nb = nfunc(la, cartesian), nfunc(lb, cartesian)
    S = np.zeros((na * nb, len(pairs)))
    T = np.zeros((na * nb, len(pairs)))
    for ij, (a, b) in enumerate(pairs):
        sa = slice(basis.poff[a], basis.poff[a] + basis.nprim[a])
        sb = slice(basis.poff[b], basis.poff[b] + basis.nprim[b])
        args = (la, lb, basis.xyz[a], basis.xyz[b], basis.exps[sa], basis.coefs[sa], basis.exps[sb],
                basis.coefs[sb])
        S[:, ij] = overlap(*args, cartesian=cartesian, quad=quad).reshape(-1)
        T[:, ij] = kinetic(*args, cartesian=cartesian, quad=quad).reshape(-1)
    return S.reshape(-1), T.reshape(-1)


def nfunc(l: int, cartesian: bool) -> int:
    return (l + 1) * (l + 2) // 2 if cartesian else 2 * l + 1


def eri(basis, ncentre: int, bra, ket, cartesian: bool = False, quartets=None,
        deriv: bool = False, quad: bool = False) -> np.ndarray:
    """Contracted shell-quartet integrals.

    basis: object with xyz [nshell,3], l, nprim, poff, exps, coefs.
    bra, ket: int arrays [n, 2] of shell indices (second column ignored for
    a 1-centre side).
    quartets: optional int array [nq, 2] of (bra index, ket index); if None
    the dense outer product is returned as an array of shape
    [nbra, nab, ncd, nket] (Fortran order, i.e. the library's layout).
    deriv: return the 12 centre derivatives (A,B,C,D) x (x,y,z).
    """
    xyz = _f64(basis.xyz).reshape(-1)
    l = _i32(basis.l); nprim = _i32(basis.nprim); poff = _i32(basis.poff)
    ex = _f64(basis.exps); co = _f64(basis.coefs)
    bra = _i32(np.asarray(bra).reshape(-1, 2)); ket = _i32(np.asarray(ket).reshape(-1, 2))
    nbra, nket = bra.shape[0], ket.shape[0]
    la = int(l[bra[0, 0]]); lb = int(l[bra[0, 1]]) if ncentre == 4 else 0
    lc = int(l[ket[0, 0]]); ld = int(l[ket[0, 1]]) if ncentre >= 3 else 0
    nab = nfunc(la, cartesian) * nfunc(lb, cartesian)
    ncd = nfunc(lc, cartesian) * nfunc(ld, cartesian)
    nd = 12 if deriv else 1
    if quartets is not None:
        q = _i32(np.asarray(quartets).reshape(-1, 2))
        nq = q.shape[0]
        out = np.zeros(nq * nd * nab * ncd)
        qp = _ip(q)
    else:
        nq = -1
        out = np.zeros(nbra * nket * nd * nab * ncd)
        q = np.zeros(2, dtype=np.int32)
        qp = _ip(q)
    rc = _load(quad)["eri"](ncentre, l.size, _dp(xyz), _ip(l), _ip(nprim), _ip(poff), _dp(ex),
                            _dp(co), nbra, _ip(bra), nket, _ip(ket), nq, qp, int(cartesian),
                            12 if deriv else -1, _dp(out))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    if quartets is not None:
        return out.reshape(nq, nd, nab, ncd) if deriv else out.reshape(nq, nab, ncd)
    if deriv:
        # out[((ij + nbra*(d + 12*kl))*nab + ab)*ncd + cd]
        return out.reshape(nket, 12, nbra, nab, ncd)
    return out.reshape(nket, ncd, nab, nbra).transpose(3, 2, 1, 0)
