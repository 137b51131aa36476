"""Prepared batches (mdx_eri_prepare, mdx_one_body_prepare, mdx_nuclear_prepare
and their run calls) through the C ABI.

* A run gives the plain call's result bit for bit: the same kernels read the
  same tables, which now sit in the batch's own device memory.
* A run captured into a HIP graph replays correctly when the centres (or the
  charges) are rewritten in place between replays: every replay is compared
  with the plain call on the values of that moment, with the program's own
  eager work and synchronisations in between.
* The plain calls, which copy host tables per call, refuse a capturing stream
  before doing any work.
* Argument errors: another batch kind, changed shell metadata, a short
  workspace.
"""
import ctypes

import numpy as np
import pytest

from paper_2506_12501_amd import workloads as W

pytestmark = pytest.mark.gpu

ERI_CASES = [
    # name, nbra, nket, K, paired
    ("(dd|dd)", 37, 29, 3, False),     # matrix-core kernel, ragged tiles
    ("(pp|ps)", 70, 23, 2, False),     # register kernel, a ragged second wave
    ("(ds|ps)", 41, 41, 2, True),      # paired quartets
    ("(p|dd)", 45, 33, 3, False),      # 3-centre
    ("(hh|gg)", 9, 7, 2, False),       # mixed class: single-primitive kernel by primitive expansion
]


def _native():
    from paper_2506_12501_amd import native
    return native


def _eri_batch(name, nbra, nket, K, seed):
    return W.make_class_batch(name, nbra, nket, K, 8.0, 0.05, 50.0, 0.1, 1.0, seed=seed)


@pytest.mark.parametrize("case", ERI_CASES, ids=[c[0] for c in ERI_CASES])
def test_eri_run_matches_plain_call(case):
    import torch
    native = _native()
    name, nbra, nket, K, paired = case
    b = _eri_batch(name, nbra, nket, K, seed=11)
    sh = native.DeviceShells(b.basis)
    ref = native.eri(sh, b.ncentre, b.bra, b.ket, paired=paired).permute(*reversed(range(3 if paired else 4)))
    ref = ref.contiguous().reshape(-1)
    p = native.Prepared("eri", sh, b.ncentre, b.bra, b.ket, paired=paired)
    assert p.out_size == ref.numel()
    out = p.run()[0]
    torch.cuda.synchronize()
    assert torch.equal(out[:ref.numel()], ref), name
    out2 = p.run()[0]   # a second run of the same batch
    torch.cuda.synchronize()
    assert torch.equal(out2[:ref.numel()], ref), name


def _replays(p, sh, values, write, plain, run_args=()):
    """captures p.run into a graph, then for each value set: write it in place,
    replay, and compare with the plain call (eager) on the same values"""
    import torch
    p.run(*run_args)                      # eager run first (kernel attributes set up)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            p.run(*run_args)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for i, v in enumerate(values):
        write(v)
        g.replay()
        torch.cuda.synchronize()
        got = [o.clone() for o in p.out]
        ref = plain()
        torch.cuda.synchronize()
        for a, r in zip(got, ref):
            assert torch.equal(a[:r.numel()], r), f"replay {i}"
    return g


def _moved_centres(basis, n, seed):
    rng = np.random.default_rng(seed)
    xyz = np.asarray(basis.xyz, dtype=np.float64).reshape(-1, 3)
    return [(xyz + rng.normal(scale=0.05, size=xyz.shape)).reshape(-1) for _ in range(n)]


@pytest.mark.parametrize("case", [ERI_CASES[0], ERI_CASES[1], ERI_CASES[3]], ids=["dddd", "ppps", "p_dd"])
def test_eri_run_captured_in_graph(case):
    import torch
    native = _native()
    name, nbra, nket, K, paired = case
    b = _eri_batch(name, nbra, nket, K, seed=12)
    sh = native.DeviceShells(b.basis)
    p = native.Prepared("eri", sh, b.ncentre, b.bra, b.ket)

    def write(v):
        sh.center.copy_(torch.as_tensor(v, device="cuda"))

    def plain():
        r = native.eri(sh, b.ncentre, b.bra, b.ket)
        return [r.permute(3, 2, 1, 0).contiguous().reshape(-1)]
    _replays(p, sh, _moved_centres(b.basis, 3, seed=5), write, plain)


@pytest.mark.parametrize("la,lb", [(2, 1), (3, 3), (5, 2)])
def test_one_body_run_captured_in_graph(la, lb):
    import torch
    native = _native()
    basis, pairs = W.one_body_pairs(la, lb, 13, 11, 3, seed=la * 7 + lb)
    sh = native.DeviceShells(basis)
    p = native.Prepared("one_body", sh, pairs)
    S0, T0 = native.one_body(sh, pairs)
    out = p.run()
    torch.cuda.synchronize()
    n = S0.numel()
    assert p.out_size == n
    assert torch.equal(out[0][:n], S0.permute(1, 2, 0).contiguous().reshape(-1))
    assert torch.equal(out[1][:n], T0.permute(1, 2, 0).contiguous().reshape(-1))

    def write(v):
        sh.center.copy_(torch.as_tensor(v, device="cuda"))

    def plain():
        S, T = native.one_body(sh, pairs)
        return [S.permute(1, 2, 0).contiguous().reshape(-1), T.permute(1, 2, 0).contiguous().reshape(-1)]
    _replays(p, sh, _moved_centres(basis, 3, seed=6), write, plain)


@pytest.mark.parametrize("la,lb", [(2, 1), (4, 2), (4, 3)])
def test_nuclear_run_captured_in_graph(la, lb):
    """(d|p), (g|d): the lane kernel; (g|f): the one-pair-per-wave kernel (the
    charges are read at replay time)"""
    import torch
    native = _native()
    basis, pairs = W.one_body_pairs(la, lb, 9, 7, 2, seed=la * 5 + lb)
    sh = native.DeviceShells(basis)
    nch = 70
    ch = torch.as_tensor(W.point_charges(nch, seed=3), device="cuda").reshape(-1).contiguous()
    p = native.Prepared("nuclear", sh, pairs, nch)
    V0 = native.nuclear(sh, pairs, ch)
    out = p.run(ch)
    torch.cuda.synchronize()
    assert torch.equal(out[0][:V0.numel()], V0.permute(1, 2, 0).contiguous().reshape(-1))
    news = [W.point_charges(nch, seed=10 + i).reshape(-1) for i in range(3)]

    def write(v):
        ch.copy_(torch.as_tensor(v, device="cuda"))

    def plain():
        return [native.nuclear(sh, pairs, ch).permute(1, 2, 0).contiguous().reshape(-1)]
    _replays(p, sh, news, write, plain, run_args=(ch,))


def test_plain_calls_refuse_a_capturing_stream():
    """the plain calls copy host tables per call, which a graph cannot replay:
    they return MDX_EINVAL on a capturing stream before any work, and the
    capture itself stays valid"""
    import torch
    native = _native()
    b = _eri_batch("(pp|ps)", 20, 9, 2, seed=13)
    sh = native.DeviceShells(b.basis)
    basis1, pairs1 = W.one_body_pairs(1, 1, 5, 4, 2, seed=2)
    sh1 = native.DeviceShells(basis1)
    p = native.Prepared("eri", sh, b.ncentre, b.bra, b.ket)
    p.run()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    errs = []
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for call in (lambda: native.eri(sh, b.ncentre, b.bra, b.ket),
                         lambda: native.one_body(sh1, pairs1)):
                try:
                    call()
                except native.MdxError as e:
                    errs.append(e)
            p.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    assert len(errs) == 2 and all(e.status == native.MDX_EINVAL for e in errs), errs
    assert all("captured" in str(e) for e in errs)
    g.replay()
    torch.cuda.synchronize()
    ref = native.eri(sh, b.ncentre, b.bra, b.ket).permute(3, 2, 1, 0).contiguous().reshape(-1)
    assert torch.equal(p.out[0][:ref.numel()], ref)


def test_prepared_errors():
    import torch
    native = _native()
    L = native.lib()
    b = _eri_batch("(ps|ps)", 8, 8, 2, seed=14)
    sh = native.DeviceShells(b.basis)
    p = native.Prepared("eri", sh, b.ncentre, b.bra, b.ket)
    stream = native._stream(torch)
    o = ctypes.c_void_p(p.out[0].data_ptr())
    # another kind
    st = L.mdx_one_body_run(p.handle, ctypes.byref(sh.struct), o, o, None, 0, stream)
    assert st == native.MDX_EINVAL and b"another integral kind" in L.mdx_last_error()
    # short workspace
    st = L.mdx_eri_run(p.handle, ctypes.byref(sh.struct), o, ctypes.c_void_p(p.wsp), 16, stream)
    assert st == native.MDX_EWORKSPACE
    # changed metadata (a shell's contraction degree)
    sh2 = native.DeviceShells(b.basis)
    sh2.nprim = sh2.nprim.copy()
    sh2.nprim[0] = 1
    sh2.struct.nprim = native._i32p(sh2.nprim)
    st = L.mdx_eri_run(p.handle, ctypes.byref(sh2.struct), o, ctypes.c_void_p(p.wsp), p.ws_bytes, stream)
    assert st == native.MDX_EINVAL and b"metadata" in L.mdx_last_error()
    # a failing preparation leaves the handle NULL
    h = ctypes.c_void_p(1)
    bad = np.array([[0, 10 ** 6]], dtype=np.int32)
    st = L.mdx_one_body_prepare(p.ctx.handle, ctypes.byref(sh.struct), 1, native._i32p(bad), 0, ctypes.byref(h))
    assert st == native.MDX_EINVAL and not h.value
    torch.cuda.synchronize()
