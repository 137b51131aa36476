"""Algorithmic FLOP count per shellset of the MD scheme as the paper states it
(ket transform with partial early contraction of the terminal Hermites,
Sec. 2.2.2; single-function solid bra keeps only terminal Hermites,
Sec. 2.2.3).  Used for every "% of FP64 peak" figure; it counts what the
method must do, not what a particular GPU schedule executes.

Per 4-centre shellset, canonical orientation l_bra >= l_ket:
  K_bra K_ket [B(L) + R(L) + 2 NH(l_bra) NH(l_ket-1) n_cd + 2 NH(l_bra) nc(l_ket)]
  + K_bra [2 NH(l_bra) nc(l_ket) n_cd + 2 n_ab NH(l_bra) n_cd]
B(L) = 20 + 3(L+1) (Boys by table + downward recursion), R(L) = 3 sum_{j=1..L} (NH(j)-1)
(Hermite recursion, Eq. (31)).  3-centre: NH(l_bra) -> nc(l_X), n_ab -> 2 l_X + 1.
"""


def nh(l: int) -> int:
    return 0 if l < 0 else (l + 1) * (l + 2) * (l + 3) // 6


def nc(l: int) -> int:
    return 0 if l < 0 else (l + 1) * (l + 2) // 2


def nfunc(l: int, cartesian: bool = False) -> int:
    return nc(l) if cartesian else 2 * l + 1


def shellset_flops(la: int, lb: int, lc: int, ld: int, Ka: int = 1, Kb: int = 1, Kc: int = 1, Kd: int = 1,
                   cartesian: bool = False) -> float:
    """lb or ld < 0: single-function side (3-/2-centre)."""
    single_bra = lb < 0
    lbra = la + max(lb, 0)
    lket = lc + max(ld, 0)
    n_ab = nfunc(la, cartesian) * (nfunc(lb, cartesian) if lb >= 0 else 1)
    n_cd = nfunc(lc, cartesian) * (nfunc(ld, cartesian) if ld >= 0 else 1)
    Kbra, Kket = Ka * max(Kb, 1), Kc * max(Kd, 1)
    if not single_bra and lbra < lket:            # canonical orientation
        lbra, lket, n_ab, n_cd, Kbra, Kket = lket, lbra, n_cd, n_ab, Kket, Kbra
    L = lbra + lket
    B = 20 + 3 * (L + 1)
    R = 3 * sum(nh(j) - 1 for j in range(1, L + 1))
    nhb = nc(lbra) if (single_bra and not cartesian) else nh(lbra)
    per_q = B + R + 2 * nhb * nh(lket - 1) * n_cd + 2 * nhb * nc(lket)
    per_b = 2 * nhb * nc(lket) * n_cd + 2 * n_ab * nhb * n_cd
    return float(Kbra * Kket * per_q + Kbra * per_b)


def output_bytes(la, lb, lc, ld, cartesian=False) -> int:
    n_ab = nfunc(la, cartesian) * (nfunc(lb, cartesian) if lb >= 0 else 1)
    n_cd = nfunc(lc, cartesian) * (nfunc(ld, cartesian) if ld >= 0 else 1)
    return 8 * n_ab * n_cd


def grad_shellset_flops(la: int, lb: int, lc: int, ld: int, Ka: int = 1, Kb: int = 1, Kc: int = 1, Kd: int = 1,
                        cartesian: bool = False) -> float:
    """FLOPs of the backward schedule per shellset (twelve centre derivatives
    contracted with an adjoint).  One pass per derivative side d against the
    other side w (4-centre: both pairs; 3-centre: the ket pair; 2-centre: the
    lower-l function), each with L' = l_d + l_w + 1:
      K_d K_w [B(L') + R(L') + 2 NH(l_d+1) NH(l_w-1) n_d + 2 NH(l_d+1) nc(l_w)]
      + K_d [2 NH(l_d+1) nc(l_w) n_d + 12 NH(l_d+1) n_d]      (terminal block, six dots)
      + K_w 2 NH(l_w-1) n_w n_d + 2 nc(l_w) n_w n_d           (adjoint folded into w)
    A single function counts as a pair with a unit s partner."""
    nfn = lambda l: nfunc(l, cartesian) if l >= 0 else 1
    sides = [(la + max(lb, 0), nfn(la) * nfn(lb), Ka * max(Kb, 1)),
             (lc + max(ld, 0), nfn(lc) * nfn(ld), Kc * max(Kd, 1))]
    if lb >= 0 and ld >= 0:
        passes = [(0, 1), (1, 0)]
    elif ld >= 0:
        passes = [(1, 0)]
    else:
        passes = [(0, 1)] if la <= lc else [(1, 0)]
    total = 0.0
    for d, w in passes:
        (ldd, nd, Kd_), (lw, nw, Kw) = sides[d], sides[w]
        L = ldd + lw + 1
        B = 20 + 3 * (L + 1)
        R = 3 * sum(nh(j) - 1 for j in range(1, L + 1))
        h = nh(ldd + 1)
        per_q = B + R + 2 * h * nh(lw - 1) * nd + 2 * h * nc(lw)
        per_d = 2 * h * nc(lw) * nd + 12 * h * nd
        per_w = 2 * nh(lw - 1) * nw * nd
        total += Kd_ * Kw * per_q + Kd_ * per_d + Kw * per_w + 2 * nc(lw) * nw * nd
    return float(total)


def one_body_flops(la: int, lb: int, Ka: int = 1, Kb: int = 1, cartesian: bool = False) -> float:
    """Overlap + kinetic energy of one contracted shell pair (Sec. 2.1, Eq. (8)).
    Per primitive pair: 40 for zeta_p, P, X_PA, X_PB and the prefactor; 5 per
    1-D E coefficient E^{ij}_t (i <= l_a, j <= l_b + 2, t <= i + j) on 3 axes;
    32 per Cartesian function pair (S product, three 1-D kinetic terms, T
    combination, both accumulations).  Per pair: the factorised Cartesian-to-
    solid transform of S and T."""
    ne = sum(i + j + 1 for i in range(la + 1) for j in range(lb + 3)) - 1
    prim = 40 + 3 * 5 * ne + 32 * nc(la) * nc(lb)
    sph = 0 if cartesian else 2 * 2 * (nc(la) * nc(lb) * (2 * lb + 1) + (2 * lb + 1) * nc(la) * (2 * la + 1))
    return Ka * Kb * prim + sph


def nuclear_flops(la: int, lb: int, Ka: int = 1, Kb: int = 1, ncharge: int = 100,
                  cartesian: bool = False) -> float:
    """1-particle Coulomb integrals of one contracted shell pair with early
    summation over ncharge point charges (Eqs. (26), (30), (34), (37)).
    Per primitive pair and charge: 8 (P - I, T), B(L) for the Boys function,
    2 (L+1) for [0]_I^(m), R(L) for the recursion, N_H(L) to accumulate.
    Per primitive pair: 40 setup, 5 per 1-D E coefficient on 3 axes, and per
    Cartesian function pair 3 per Hermite term (t, u, v) plus 2.  Per pair:
    the factorised solid transform."""
    L = la + lb
    B = 20 + 3 * (L + 1)
    R = 3 * sum(nh(j) - 1 for j in range(1, L + 1))
    per_charge = 8 + B + 2 * (L + 1) + R + nh(L)
    ne = sum(i + j + 1 for i in range(la + 1) for j in range(lb + 1)) - 1
    ca = [(la - s, s - v, v) for s in range(la + 1) for v in range(s + 1)]
    cb = [(lb - s, s - v, v) for s in range(lb + 1) for v in range(s + 1)]
    terms = sum((a[0] + b[0] + 1) * (a[1] + b[1] + 1) * (a[2] + b[2] + 1) for a in ca for b in cb)
    prim = ncharge * per_charge + 40 + 15 * ne + 3 * terms + 2 * nc(la) * nc(lb)
    sph = 0 if cartesian else 2 * (nc(la) * nc(lb) * (2 * lb + 1) + (2 * lb + 1) * nc(la) * (2 * la + 1))
    return Ka * Kb * prim + sph
