"""Host planning (no GPU): canonical pair lists and Schwarz prefixes equal a
brute-force enumeration of the kept canonical quartets."""
import itertools

import numpy as np

from paper_2506_12501_amd import screening as S, workloads as W


def test_canonical_pairs_cover_unordered_pairs_once():
    b, _ = W.water_cluster(nx=2, ny=2, nz=2)
    P = S.canonical_pairs(b.l, 2)
    seen = set()
    for (la, lb), p in P.items():
        for i, j in p:
            assert b.l[i] == la and b.l[j] == lb and (la > lb or i >= j)
            key = (min(i, j), max(i, j))
            assert key not in seen
            seen.add(key)
    n = len(b.l)
    assert len(seen) == n * (n + 1) // 2


def test_water_cluster_counts():
    b, atom = W.water_cluster()
    P = S.canonical_pairs(b.l, 2)
    assert len(b.l) == 384 and sum(v.shape[0] for v in P.values()) == 73920
    assert len(S.pair_classes(2)) == 6


def test_prefixes_equal_brute_force():
    rng = np.random.default_rng(3)
    pairs = {pc: np.stack([np.arange(n), np.arange(n)], 1).astype(np.int32) + 100 * k
             for k, (pc, n) in enumerate(zip(S.pair_classes(1), (7, 5, 4)))}
    Q = {pc: 10.0 ** rng.uniform(-9, 1, p.shape[0]) for pc, p in pairs.items()}
    tau = 1e-8
    batches = S.class_batches(pairs, Q, tau)
    got = set()
    for bt in batches:
        for k, c in enumerate(bt["bra_count"]):
            for i in range(c):
                got.add((tuple(bt["bra"][i]), tuple(bt["ket"][k])))
        assert bt["quartets"] == int(bt["bra_count"].sum())
    want = set()
    order = list(pairs)
    for ib, pb in enumerate(order):
        for ik in range(ib + 1):
            pk = order[ik]
            for i, j in itertools.product(range(pairs[pb].shape[0]), range(pairs[pk].shape[0])):
                qi, qj = Q[pb][i], Q[pk][j]
                if qi * qj < tau:
                    continue
                if pb == pk:   # one of (ij|kl), (kl|ij): the bra with the larger Q (then the lower index)
                    if (qi, -i) < (qj, -j):
                        continue
                want.add((tuple(pairs[pb][i]), tuple(pairs[pk][j])))
    assert got == want


def test_k_buckets_cover_the_same_quartets():
    """Splitting the pair classes into contraction-degree buckets keeps exactly
    the same set of screened canonical quartets."""
    b, _ = W.water_cluster(nx=2, ny=2, nz=2)
    P = S.canonical_pairs(b.l, 2)
    rng = np.random.default_rng(4)
    Q = {pc: 10.0 ** rng.uniform(-8, 1, p.shape[0]) for pc, p in P.items()}

    def kept(batches):
        out = set()
        for bt in batches:
            for k, c in enumerate(bt["bra_count"]):
                for i in range(c):
                    a, bb = tuple(bt["bra"][i]), tuple(bt["ket"][k])
                    out.add((a, bb))
        return out

    plain = S.class_batches(P, Q, 1e-9)
    bucketed = S.class_batches(P, Q, 1e-9, nprim=b.nprim)
    assert len(bucketed) > len(plain)
    assert sum(x["quartets"] for x in bucketed) == sum(x["quartets"] for x in plain)
    kp, kb = kept(plain), kept(bucketed)
    # the same unordered quartets (a same-class pair of pairs may appear as (x|y) or (y|x))
    norm = lambda s: {tuple(sorted(q)) for q in s}
    assert norm(kp) == norm(kb) and len(kb) == len(kp)
    for bt in bucketed:
        Kb = b.nprim[bt["bra"][:, 0]] * b.nprim[bt["bra"][:, 1]]
        assert np.all(Kb == bt["Kbra"])
