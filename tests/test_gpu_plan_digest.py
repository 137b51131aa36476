"""Digestion over screened plans (mdx_plan_digest, plans made with MDX_DIGEST,
as plain launches and as one graph of persistent digesting kernels): every
batch of a small water-cluster plan, ragged bra prefixes included, is
contracted with random pair-blocked densities inside the kernels, and the J
blocks are compared with the __float128 oracle's integrals of every kept
quartet contracted on the host.

Bar (a contracted sum, as for the backward kernel): |err| <= 1e-12, or <=
1e-10 |J|, or <= 1e-14 sum |I D| over the terms of that J element.
"""
import numpy as np
import pytest

from paper_2506_12501_amd import screening as S, workloads as W
from tests.cluster_util import oracle_batch

pytestmark = pytest.mark.gpu

CTOL = 1e-14


def cluster_batches(tau=1e-12, seed=5):
    from paper_2506_12501_amd import native
    b, _ = W.water_cluster(seed=seed, nx=2, ny=2, nz=2)
    sh = native.DeviceShells(b)
    P = S.canonical_pairs(b.l, 2)
    Q = {pc: native.schwarz(sh, p).cpu().numpy() for pc, p in P.items()}
    batches = S.class_batches(P, Q, tau)
    S.with_offsets(batches, b.l)
    return b, sh, batches


def host_digest(ref, bt, Db, Dk):
    """J blocks (and the sums of |terms|) from the ragged-layout integrals of a
    batch: out[base_kl + ij + n_kl*(ab + nab*cd)]; Db [nbra, nab], Dk [nket, ncd]"""
    nab, ncd = bt["nab"], bt["ncd"]
    Jb, Jk = np.zeros_like(Db), np.zeros_like(Dk)
    Sb, Sk = np.zeros_like(Db), np.zeros_like(Dk)
    base = 0
    for kl, c in enumerate(bt["bra_count"]):
        blk = ref[base:base + c * nab * ncd].reshape(ncd, nab, c)   # [cd, ab, ij]
        base += c * nab * ncd
        Jb[:c] += np.einsum("dai,d->ia", blk, Dk[kl])
        Sb[:c] += np.einsum("dai,d->ia", np.abs(blk), np.abs(Dk[kl]))
        Jk[kl] += np.einsum("dai,ia->d", blk, Db[:c])
        Sk[kl] += np.einsum("dai,ia->d", np.abs(blk), np.abs(Db[:c]))
    return Jb, Jk, Sb, Sk


def assert_digest_close(got, ref, scale, what):
    err = np.abs(got - ref)
    ok = (err <= 1e-12) | (err <= 1e-10 * np.abs(ref)) | (err <= CTOL * scale)
    assert np.all(np.isfinite(got)), what
    if not ok.all():
        i = np.unravel_index(np.argmax(np.where(ok, 0, err)), err.shape)
        raise AssertionError(f"{what}: {np.count_nonzero(~ok)} of {ok.size} off; worst {i}: gpu {got[i]!r} "
                             f"oracle {ref[i]!r} scale {scale[i]!r}")


@pytest.mark.parametrize("tau,fused", [(1e-12, False), (1e-8, False), (1e-12, True)])
def test_plan_digest_matches_oracle(tau, fused):
    """plain launches, and the digesting graph (persistent queue kernels)"""
    import torch
    from paper_2506_12501_amd import native
    b, sh, batches = cluster_batches(tau)
    nb = [native.Batch(4, bt["bra"], bt["ket"], bt["bra_count"], bt["out_offset"]) for bt in batches]
    plan = native.Plan(sh, nb, digest=True, fused=fused)
    rng = np.random.default_rng(11)
    dev, blocks, host = "cuda", [], []
    for bt in batches:
        nbra, nket = len(bt["bra"]), len(bt["ket"])
        Db = rng.standard_normal((nbra, bt["nab"]))
        Dk = rng.standard_normal((nket, bt["ncd"]))
        # device layout: D[ij + nbra*ab] (column-major), i.e. the transpose in row-major storage
        tDb = torch.as_tensor(np.ascontiguousarray(Db.T), device=dev)
        tDk = torch.as_tensor(np.ascontiguousarray(Dk.T), device=dev)
        tJb = torch.zeros_like(tDb)
        tJk = torch.zeros_like(tDk)
        blocks.append((tDb, tDk, tJb, tJk))
        host.append((Db, Dk))
    plan.digest(blocks)
    if fused:   # a second execution of the graph (replay) into fresh J blocks
        for blk in blocks:
            blk[2].zero_()
            blk[3].zero_()
        torch.cuda.synchronize()
        plan.digest(blocks)
    torch.cuda.synchronize()
    nquart = 0
    for bt, (tDb, tDk, tJb, tJk), (Db, Dk) in zip(batches, blocks, host):
        ref, _ = oracle_batch(b, bt)
        Jb, Jk, Sb, Sk = host_digest(ref, bt, Db, Dk)
        assert_digest_close(tJb.cpu().numpy().T, Jb, Sb, f"{bt['name']} Jbra")
        assert_digest_close(tJk.cpu().numpy().T, Jk, Sk, f"{bt['name']} Jket")
        nquart += bt["quartets"]
    print(f"tau {tau} fused {fused}: {len(batches)} batches, {nquart} quartets digested")


def test_plan_digest_one_side_and_accumulation():
    """Jket only (Jbra NULL), twice into the same block: twice the single result"""
    import torch
    from paper_2506_12501_amd import native
    b, sh, batches = cluster_batches(1e-10)
    bt = max(batches, key=lambda x: x["quartets"])
    plan = native.Plan(sh, [native.Batch(4, bt["bra"], bt["ket"], bt["bra_count"], 0)], digest=True)
    rng = np.random.default_rng(12)
    Db = rng.standard_normal((len(bt["bra"]), bt["nab"]))
    tDb = torch.as_tensor(np.ascontiguousarray(Db.T), device="cuda")
    tJk = torch.zeros((bt["ncd"], len(bt["ket"])), dtype=torch.float64, device="cuda")
    plan.digest([(tDb, None, None, tJk)])
    plan.digest([(tDb, None, None, tJk)])
    torch.cuda.synchronize()
    ref, _ = oracle_batch(b, bt)
    _, Jk, _, Sk = host_digest(ref, bt, Db, np.zeros((len(bt["ket"]), bt["ncd"])))
    assert_digest_close(tJk.cpu().numpy().T, 2 * Jk, 2 * Sk, f"{bt['name']} Jket x2")


def test_plan_digest_errors():
    import torch
    from paper_2506_12501_amd import native
    b, sh, batches = cluster_batches(1e-10)
    bt = batches[0]
    nb = [native.Batch(4, bt["bra"], bt["ket"], bt["bra_count"], 0)]
    dplan = native.Plan(sh, nb, digest=True)
    with pytest.raises(native.MdxError) as e:
        dplan.execute()
    assert e.value.status == native.MDX_EINVAL
    splan = native.Plan(sh, nb)
    z = torch.zeros(len(bt["bra"]) * bt["nab"], dtype=torch.float64, device="cuda")
    with pytest.raises(native.MdxError) as e:
        splan.digest([(z, None, None, None)])
    assert e.value.status == native.MDX_EINVAL
    with pytest.raises(native.MdxError) as e:   # Jbra without Dket
        dplan.digest([(z, None, z, None)])
    assert e.value.status == native.MDX_EINVAL
