"""Oracle references for screened cluster batches (ragged plan layout) and
the Cauchy-Schwarz-scaled accuracy bar they are held to."""
import numpy as np

from oracle import oracle as O
from tests.gpu_util import ATOL, RTOL


def oracle_Q(basis, pairs, cart=False):
    q = np.stack([np.arange(pairs.shape[0])] * 2, axis=1)
    D = O.eri(basis, 4, pairs, pairs, cartesian=cart, quartets=q)   # [n, nab, nab]
    return np.sqrt(np.abs(np.einsum("nii->ni", D)).max(axis=1))


def oracle_batch(b, bt, quad=True):
    """oracle values of every kept quartet of a batch in the plan's ragged
    layout, and the Cauchy-Schwarz scale Q_ab Q_cd of each element"""
    qs = np.array([(i, k) for k, c in enumerate(bt["bra_count"]) for i in range(c)])
    D = O.eri(b, 4, bt["bra"], bt["ket"], quartets=qs, quad=quad)   # [q, nab, ncd]
    Qb, Qk = oracle_Q(b, bt["bra"]), oracle_Q(b, bt["ket"])
    qq = Qb[qs[:, 0]] * Qk[qs[:, 1]]
    out = np.empty(bt["quartets"] * bt["nab"] * bt["ncd"])
    scale = np.empty_like(out)
    base = n = 0
    for k, c in enumerate(bt["bra_count"]):
        m = c * bt["nab"] * bt["ncd"]
        out[base:base + m] = D[n:n + c].transpose(2, 1, 0).reshape(-1)
        scale[base:base + m] = np.broadcast_to(qq[n:n + c], (bt["ncd"], bt["nab"], c)).reshape(-1)
        base += m
        n += c
    return out, scale


CS_TOL = 1e-12


def assert_close_cs(got, ref, scale, what, g13_only=False):
    """Elements of contracted shellsets over tight exponents on one or two
    centres are sums of large primitive terms that cancel (exactly, when the
    integral vanishes by symmetry); fp64 resolves them only to about 1e-13 of
    the Cauchy-Schwarz scale Q_ab Q_cd.  Pass iff |err| <= 1e-12, or <= 1e-10
    |ref|, or <= CS_TOL Q_ab Q_cd, against the __float128 oracle.

    g13_only: the Cauchy-Schwarz clause is not granted (the integral kernels
    form X_PA, X_PB and P from centre differences, so one-centre symmetry
    zeros come out exactly 0 and no element needs it).  Returns the number of
    elements beyond 1e-12 abs / 1e-10 rel."""
    err = np.abs(got - ref)
    assert np.all(np.isfinite(got)), what
    g13 = (err <= ATOL) | (err <= RTOL * np.abs(ref))
    ok = g13 if g13_only else g13 | (err <= CS_TOL * scale)
    if not ok.all():
        i = int(np.argmax(np.where(ok, 0, err / scale)))
        raise AssertionError(f"{what}: {np.count_nonzero(~ok)} of {ok.size} off; worst {i}: gpu {got[i]!r} "
                             f"oracle {ref[i]!r} scale {scale[i]!r}")
    nbeyond = int(np.count_nonzero(~g13))
    print(f"{what}: max err {err.max():.2e}, max err/(Q Q) {np.max(err / scale):.2e}, "
          f"elements beyond 1e-12 abs / 1e-10 rel: {nbeyond}")
    return nbeyond
