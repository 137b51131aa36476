"""Plans on the GPU: Schwarz factors, screened ragged batches of a small
water-like cluster run as plain launches and as one fused graph, each checked
against the oracle; repeated graph replays; metadata and argument errors."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import screening as S, workloads as W
from tests.cluster_util import assert_close_cs, oracle_Q, oracle_batch
from tests.gpu_util import assert_close

pytestmark = pytest.mark.gpu


def small_cluster():
    return W.water_cluster(seed=5, nx=2, ny=2, nz=2)


def test_schwarz_factors():
    from paper_2506_12501_amd import native
    b, _ = small_cluster()
    sh = native.DeviceShells(b)
    for pc, pairs in S.canonical_pairs(b.l, 2).items():
        got = native.schwarz(sh, pairs).cpu().numpy()
        ref = oracle_Q(b, pairs)
        assert_close(got, ref, f"Q {pc}")


def plan_setup(tau=1e-12, seed=5, buckets=False):
    from paper_2506_12501_amd import native
    b, _ = W.water_cluster(seed=seed, nx=2, ny=2, nz=2)
    sh = native.DeviceShells(b)
    P = S.canonical_pairs(b.l, 2)
    Q = {pc: native.schwarz(sh, p).cpu().numpy() for pc, p in P.items()}
    batches = S.class_batches(P, Q, tau, nprim=b.nprim if buckets else None)
    total = S.with_offsets(batches, b.l)
    nb = [native.Batch(4, bt["bra"], bt["ket"], bt["bra_count"], bt["out_offset"]) for bt in batches]
    return b, sh, batches, nb, total


def test_plain_and_fused_plans_match_oracle():
    from paper_2506_12501_amd import native
    b, sh, batches, nb, total = plan_setup()
    assert len(batches) == 21
    plain = native.Plan(sh, nb, fused=False)
    fused = native.Plan(sh, nb, fused=True)
    assert plain.out_size == fused.out_size == total
    o1 = plain.execute().cpu().numpy()
    o2 = fused.execute().cpu().numpy()
    # the same kernel bodies with the same arithmetic order
    assert np.array_equal(o1, o2)
    for bt in batches:
        off, n = bt["out_offset"], bt["quartets"] * bt["nab"] * bt["ncd"]
        ref, scale = oracle_batch(b, bt)
        assert_close_cs(o2[off:off + n], ref, scale, bt["name"], g13_only=True)
    print("quartets", sum(bt["quartets"] for bt in batches), "doubles", total)


def test_bucketed_plans_share_pair_data():
    """contraction-degree buckets: many batches whose ket lists are prefixes of
    shared sorted lists; the fused plan computes each side's pair data once"""
    from paper_2506_12501_amd import native
    b, sh, batches, nb, total = plan_setup(buckets=True)
    assert len(batches) > 50
    plain = native.Plan(sh, nb, fused=False)
    fused = native.Plan(sh, nb, fused=True)
    o1 = plain.execute().cpu().numpy()
    o2 = fused.execute().cpu().numpy()
    assert np.array_equal(o1, o2)
    for bt in batches:
        off, n = bt["out_offset"], bt["quartets"] * bt["nab"] * bt["ncd"]
        ref, scale = oracle_batch(b, bt)
        assert_close_cs(o2[off:off + n], ref, scale, f"{bt['name']} K{bt['Kbra']}x{bt['Kket']}", g13_only=True)
    print("batches", len(batches), "quartets", sum(bt["quartets"] for bt in batches))


def test_graph_replays():
    import torch
    from paper_2506_12501_amd import native
    b, sh, batches, nb, total = plan_setup()
    fused = native.Plan(sh, nb, fused=True)
    ref = fused.execute().clone()
    out = torch.full_like(ref, float("nan"))
    for r in range(4):
        out.fill_(float("nan"))                            # eager work between replays
        fused.execute(out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {r}"
    # another output buffer rebuilds the graph
    out2 = torch.zeros_like(ref)
    fused.execute(out2)
    assert torch.equal(out2, ref)


def test_dense_batch_in_plan_equals_class_call():
    from paper_2506_12501_amd import native
    bt = W.make_class_batch("(dd|pp)", 5, 7, 2, 6.0, 0.1, 30.0, 0.1, 1.0, seed=60)
    sh = native.DeviceShells(bt.basis)
    ref = native.eri(sh, 4, bt.bra, bt.ket).permute(3, 2, 1, 0).reshape(-1)
    for fused in (False, True):
        pl = native.Plan(sh, [native.Batch(4, bt.bra, bt.ket, None, 3)], fused=fused)
        out = pl.execute()
        assert pl.out_size == 3 + ref.numel()
        assert np.array_equal(out[3:].cpu().numpy(), ref.cpu().numpy())


def test_plan_rejects_other_basis():
    from paper_2506_12501_amd import native
    b, sh, batches, nb, total = plan_setup()
    pl = native.Plan(sh, nb[:2], fused=False)
    other = native.DeviceShells(W.water_cluster(seed=6, nx=2, ny=2, nz=1)[0])
    pl.shells = other
    with pytest.raises(native.MdxError) as e:
        pl.execute()
    assert e.value.status == native.MDX_EINVAL


def test_bad_counts_rejected():
    from paper_2506_12501_amd import native
    bt = W.make_class_batch("(pp|pp)", 3, 2, 1, 6.0, 0.1, 30.0, 0.1, 1.0, seed=61)
    sh = native.DeviceShells(bt.basis)
    with pytest.raises(native.MdxError) as e:
        native.Plan(sh, [native.Batch(4, bt.bra, bt.ket, np.array([4, 1]))])
    assert e.value.status == native.MDX_EINVAL
