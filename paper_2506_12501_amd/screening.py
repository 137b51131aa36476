"""Batch planning for a whole basis: canonical shell pairs grouped by class,
Schwarz factors on the device, sorted screening prefixes, one batch per
canonical quartet class (host-side planning; no integral arithmetic here).

Canonical forms (8-fold permutational symmetry of (ab|cd)):
  - a pair (a, b) has l_a >= l_b, and a >= b when l_a == l_b;
  - pair classes are ordered by (l_a + l_b, l_a); a quartet class has its bra
    pair class at or after its ket pair class, so l_bra >= l_ket;
  - within a class whose bra and ket pair classes coincide, only quartets
    with bra position <= ket position (in the sorted order) are kept.
Screening (Sec. 3.1, batch screening on sorted data): pairs of each class
are sorted by decreasing Q; quartet (ij|kl) is kept iff Q_ij Q_kl >= tau.
For a ket pair kl the kept bra pairs are then a prefix of the sorted bra
list, which is the plan's ragged bra_count.
"""
from __future__ import annotations

import numpy as np


def pair_classes(lmax: int):
    out = [(la, lb) for la in range(lmax + 1) for lb in range(la + 1)]
    return sorted(out, key=lambda c: (c[0] + c[1], c[0]))


def canonical_pairs(l: np.ndarray, lmax: int):
    """{(la, lb): int32 [n, 2] shell pairs}"""
    l = np.asarray(l)
    res = {}
    for la, lb in pair_classes(lmax):
        A = np.nonzero(l == la)[0]
        B = np.nonzero(l == lb)[0]
        if la == lb:
            ii, jj = np.tril_indices(A.size)
            p = np.stack([A[ii], A[jj]], axis=1)
        else:
            p = np.stack(np.meshgrid(A, B, indexing="ij"), axis=-1).reshape(-1, 2)
        res[(la, lb)] = np.ascontiguousarray(p, dtype=np.int32)
    return res


def class_batches(pairs_by_class: dict, Q_by_class: dict, tau: float = 1e-12, nprim=None):
    """Sorted, screened batches.  Returns a list of dicts with keys
    name, bra, ket, bra_count, quartets, Qbra, Qket (bra pair class >= ket).

    nprim (contraction degree per shell): if given, each pair class is split
    into buckets of equal pair contraction degree K_a K_b, and there is one
    batch per (quartet class, bra bucket, ket bucket) -- so that the work items
    of a batch have equal primitive counts.  Within one pair class the bucket
    pairs (b, k) with b > k are kept whole, b == k triangular."""
    order = list(pairs_by_class)
    buckets = {}   # pair class -> [(K, sorted pairs, sorted Q)]
    for pc in order:
        P = pairs_by_class[pc]
        Q = np.asarray(Q_by_class[pc], dtype=np.float64)
        if nprim is None:
            groups = [(0, np.arange(P.shape[0]))]
        else:
            K = np.asarray(nprim)[P[:, 0]] * np.asarray(nprim)[P[:, 1]]
            groups = [(int(k), np.nonzero(K == k)[0]) for k in sorted(set(K.tolist()), reverse=True)]
        lst = []
        for k, sel in groups:
            idx = sel[np.argsort(-Q[sel], kind="stable")]
            lst.append((k, P[idx], Q[idx]))
        buckets[pc] = lst
    out = []
    ch = "spdfghik"
    for ib, pb in enumerate(order):
        for ik in range(ib + 1):
            pk = order[ik]
            for bb, (Kb, bra, Qb) in enumerate(buckets[pb]):
                for bk, (Kk, ket, Qk) in enumerate(buckets[pk]):
                    if pb == pk and bk > bb:
                        continue
                    if bra.shape[0] == 0 or ket.shape[0] == 0:
                        continue
                    # bra prefix per ket: Q_bra >= tau / Q_ket (Q_bra sorted descending)
                    with np.errstate(divide="ignore"):
                        lim = np.where(Qk > 0, tau / Qk, np.inf)
                    cnt = np.searchsorted(-Qb, -lim, side="right").astype(np.int64)
                    if pb == pk and bb == bk:
                        cnt = np.minimum(cnt, np.arange(1, ket.shape[0] + 1))
                    nz = np.nonzero(cnt)[0]
                    if nz.size == 0:
                        continue
                    nket = int(nz[-1]) + 1      # counts are nonincreasing in the ket position (up to the triangle)
                    name = f"({ch[pb[0]]}{ch[pb[1]]}|{ch[pk[0]]}{ch[pk[1]]})"
                    out.append({"name": name, "Kbra": Kb, "Kket": Kk, "bra": bra, "ket": ket[:nket],
                                "bra_count": cnt[:nket].astype(np.int32), "quartets": int(cnt[:nket].sum()),
                                "Qbra": Qb, "Qket": Qk[:nket]})
    return out


def nfunc(l, cartesian=False):
    return (l + 1) * (l + 2) // 2 if cartesian else 2 * l + 1


def with_offsets(batches, l, cartesian=False):
    """adds out_offset / nab / ncd and returns the total output size (doubles)"""
    off = 0
    for b in batches:
        la, lb = l[b["bra"][0, 0]], l[b["bra"][0, 1]]
        lc, ld = l[b["ket"][0, 0]], l[b["ket"][0, 1]]
        b["nab"] = nfunc(la, cartesian) * nfunc(lb, cartesian)
        b["ncd"] = nfunc(lc, cartesian) * nfunc(ld, cartesian)
        b["out_offset"] = off
        off += b["quartets"] * b["nab"] * b["ncd"]
    return off
