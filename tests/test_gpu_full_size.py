"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times (one mdx_eri_batch call over the whole batch, or the plan of
the whole cluster): sampled shellsets against the oracle, which computes them
one by one from the quartet list.  The s/p batches are small enough to check
in full."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2506_12501_amd import screening as S, workloads as W
from tests.cluster_util import oracle_Q
from tests.gpu_util import ATOL, RTOL, assert_close, assert_close_shellsets

pytestmark = pytest.mark.gpu


def sample_quartets(nbra, nket, n, seed):
    rng = np.random.default_rng(seed)
    q = np.stack([rng.integers(0, nbra, n), rng.integers(0, nket, n)], axis=1)
    q[0] = (0, 0)
    q[1] = (nbra - 1, nket - 1)          # last tile of both sides
    q[2] = (nbra - 1, 0)
    return q


def check_sampled(batch, n=96, seed=0, quad=False):
    from paper_2506_12501_amd import native
    sh = native.DeviceShells(batch.basis)
    out = native.eri(sh, batch.ncentre, batch.bra, batch.ket)      # [nbra, nab, ncd, nket] view
    q = sample_quartets(batch.bra.shape[0], batch.ket.shape[0], n, seed)
    idx = (np.asarray(q[:, 0]), np.asarray(q[:, 1]))
    import torch
    got = out[torch.as_tensor(idx[0], device=out.device), :, :, torch.as_tensor(idx[1], device=out.device)]
    ref = O.eri(batch.basis, batch.ncentre, batch.bra, batch.ket, quartets=q, quad=quad)    # [q, nab, ncd]
    assert_close_shellsets(got.cpu().numpy(), ref, f"{batch.name} full size, {n} sampled shellsets")


@pytest.mark.parametrize("name", W.C1_CLASSES)
def test_sp_classes_all_elements(name):
    from paper_2506_12501_amd import native
    b = W.config1(name, seed=0)
    sh = native.DeviceShells(b.basis)
    got = native.eri(sh, 4, b.bra, b.ket).cpu().numpy()
    assert_close(got, O.eri(b.basis, 4, b.bra, b.ket), f"{name} 16x16")


@pytest.mark.parametrize("name", ["(pp|pp)", "(pp|ps)", "(dd|ss)"])
def test_large_register_kernel_batches(name):
    """dense batches large enough for the register kernel's multi-ket mapping
    (64 bra pairs x 16 ket pairs per workgroup): 520 bra pairs (a ragged last
    tile) x 7,300 ket pairs (a last chunk of 4), sampled shellsets"""
    b = W.make_class_batch(name, 520, 7300, 1, 4.0, 0.1, 100.0, None, None, seed=31)
    check_sampled(b, n=96, seed=4)


@pytest.mark.parametrize("name", W.C2_CLASSES)
def test_contracted_classes(name):
    check_sampled(W.config2(name, seed=0), seed=1)


@pytest.mark.parametrize("name", W.C4_CLASSES_4C + W.C4_CLASSES_3C + W.HIGH_L_CLASSES_4C)
def test_high_l_classes(name):
    # l >= 4 against the __float128 oracle (the fp64 oracle's solid transform
    # loses up to ~3e-11 of the shellset maximum there); (ii|ii) costs ~25 s of
    # quad work per shellset, so it is sampled more thinly
    quad = max(W.parse_class(name)) >= 4
    check_sampled(W.config4(name, seed=0), n=16 if name == "(ii|ii)" else 48, seed=2, quad=quad)


def test_water_cluster_plan_sampled():
    """the whole screened 384-shell cluster in one fused plan (contraction-degree
    batches) against the __float128 oracle on sampled quartets of every batch,
    per element within 1e-12 abs or 1e-10 rel (no Cauchy-Schwarz clause)"""
    import torch
    from paper_2506_12501_amd import native
    b, _ = W.water_cluster(seed=0)
    sh = native.DeviceShells(b)
    P = S.canonical_pairs(b.l, 2)
    Q = {pc: native.schwarz(sh, p).cpu().numpy() for pc, p in P.items()}
    batches = S.class_batches(P, Q, 1e-12, nprim=b.nprim)
    S.with_offsets(batches, b.l)
    plan = native.Plan(sh, [native.Batch(4, bt["bra"], bt["ket"], bt["bra_count"], bt["out_offset"])
                            for bt in batches], fused=True)
    out = plan.execute()
    rng = np.random.default_rng(3)
    nchk = 0
    for bt in batches:
        cnt = bt["bra_count"]
        starts = np.concatenate([[0], np.cumsum(cnt)])
        pick = np.unique(rng.integers(0, bt["quartets"], min(6, bt["quartets"])))
        ks = np.searchsorted(starts, pick, side="right") - 1
        iis = pick - starts[ks]
        ref = O.eri(b, 4, bt["bra"], bt["ket"], quartets=np.stack([iis, ks], 1), quad=True)
        qq = oracle_Q(b, bt["bra"])[iis] * oracle_Q(b, bt["ket"])[ks]
        nab, ncd = bt["nab"], bt["ncd"]
        obase = np.concatenate([[0], np.cumsum(cnt.astype(np.int64) * nab * ncd)])
        ab, cd = np.meshgrid(np.arange(nab), np.arange(ncd), indexing="ij")
        idx = (bt["out_offset"] + obase[ks][:, None, None] + iis[:, None, None]
               + cnt[ks][:, None, None] * (ab[None] + nab * cd[None]))
        got = out[torch.as_tensor(idx.reshape(-1), device=out.device)].cpu().numpy().reshape(ref.shape)
        err = np.abs(got - ref)
        # plain per-element bar: one-centre symmetry zeros come out exactly 0
        ok = (err <= ATOL) | (err <= RTOL * np.abs(ref))
        assert ok.all(), (bt["name"], bt["Kbra"], bt["Kket"], float(np.max(err / qq[:, None, None])))
        nchk += ok.size
    print("cluster: batches", len(batches), "elements checked", nchk)
