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
