#!/usr/bin/env python
"""Benchmark: FP64 McMurchie-Davidson ERIs on one MI355X.

One step = the whole hot path for the contracted workload (bra/ket pair data
+ Boys + Hermite recursion + ket and bra transforms + store) over both classes
(dd|dd) and (pd|dd), 256 x 256 shell pairs each (65,536 shellsets per class),
K = 3 per shell, exponents log-uniform in [0.05, 50], coefficients uniform in
[0.1, 1], centres uniform in a 10 A cube (seed 0).  Inputs are resident in HBM
before the timed region; outputs are written to HBM every step.

Prints one compact JSON line on stdout (compact_record: headline, roofline,
CPU baseline, parity and one-number summaries of the other legs) and writes
the full record of every leg to --detail-out.
"""
from __future__ import annotations

import argparse
import ctypes
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X published dense FP64 (vector and matrix)
PEAK_HBM_GBS = 8000.0
METRIC = "FP64 ERI shellsets/s + % FP64 peak per L-class; fused-batch vs per-class speedup"


def log(msg):
    """progress on stderr; stdout carries only the JSON result line"""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class HipEvents:
    """Raw hipEvent_t handles for the library's profiling hook."""

    def __init__(self, n):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.ev = (ctypes.c_void_p * n)()
        for i in range(n):
            h = ctypes.c_void_p()
            assert self.hip.hipEventCreate(ctypes.byref(h)) == 0
            self.ev[i] = h
        self.n = n

    def close(self):
        for i in range(self.n):
            if self.ev[i]:
                self.hip.hipEventDestroy(ctypes.c_void_p(self.ev[i]))
                self.ev[i] = None

    def elapsed_ms(self, i):
        ms = ctypes.c_float()
        assert self.hip.hipEventSynchronize(ctypes.c_void_p(self.ev[2 * i + 1])) == 0
        r = self.hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(self.ev[2 * i]),
                                         ctypes.c_void_p(self.ev[2 * i + 1]))
        assert r == 0, r
        return ms.value


class ClassRun:
    """Preallocated buffers for repeated mdx_eri_batch calls on one class."""

    def __init__(self, native, batch, ctx, torch):
        self.native, self.batch, self.ctx, self.torch = native, batch, ctx, torch
        self.sh = native.DeviceShells(batch.basis)
        self.bra = native._pairs(batch.bra)
        self.ket = native._pairs(batch.ket)
        self.nab, self.ncd = native._class_sizes(self.sh, batch.ncentre, self.bra, self.ket, False)
        L = native.lib()
        self.wsz = L.mdx_eri_workspace_size(ctx.handle, ctypes.byref(self.sh.struct), batch.ncentre,
                                            self.bra.shape[0], native._i32p(self.bra), self.ket.shape[0],
                                            native._i32p(self.ket), 0)
        if self.wsz == 0:
            native.check(native.MDX_EINVAL, "workspace size")
        self.ws = torch.empty(self.wsz // 8 + 64, dtype=torch.float64, device="cuda")
        self.wsp = (self.ws.data_ptr() + 255) // 256 * 256
        self.n = self.bra.shape[0] * self.ket.shape[0]
        self.out = torch.empty(self.n * self.nab * self.ncd, dtype=torch.float64, device="cuda")

    def __call__(self):
        n = self.native
        n.check(n.lib().mdx_eri_batch(self.ctx.handle, ctypes.byref(self.sh.struct), self.batch.ncentre,
                                      self.bra.shape[0], n._i32p(self.bra), self.ket.shape[0], n._i32p(self.ket),
                                      0, ctypes.c_void_p(self.out.data_ptr()), ctypes.c_void_p(self.wsp),
                                      self.wsz, n._stream(self.torch)), "mdx_eri_batch")

    def view(self):
        nb, nk = self.bra.shape[0], self.ket.shape[0]
        return self.out.view(nk, self.ncd, self.nab, nb).permute(3, 2, 1, 0)


class OneBodyRun:
    """Preallocated buffers for repeated mdx_one_body_batch calls on one class."""

    def __init__(self, native, basis, pairs, ctx, torch):
        self.native, self.ctx, self.torch = native, ctx, torch
        self.sh = native.DeviceShells(basis)
        self.pairs = native._pairs(pairs)
        self.n = self.pairs.shape[0]
        L = native.lib()
        self.wsz = L.mdx_one_body_workspace_size(ctx.handle, ctypes.byref(self.sh.struct), self.n,
                                                 native._i32p(self.pairs), 0)
        if self.wsz == 0:
            native.check(native.MDX_EINVAL, "workspace size")
        self.ws = torch.empty(self.wsz // 8 + 64, dtype=torch.float64, device="cuda")
        self.wsp = (self.ws.data_ptr() + 255) // 256 * 256
        la, lb = int(basis.l[pairs[0, 0]]), int(basis.l[pairs[0, 1]])
        self.nf = native.nfunc(la, False) * native.nfunc(lb, False)
        self.S = torch.empty(self.n * self.nf, dtype=torch.float64, device="cuda")
        self.T = torch.empty_like(self.S)

    def __call__(self):
        n = self.native
        n.check(n.lib().mdx_one_body_batch(self.ctx.handle, ctypes.byref(self.sh.struct), self.n,
                                           n._i32p(self.pairs), 0, ctypes.c_void_p(self.S.data_ptr()),
                                           ctypes.c_void_p(self.T.data_ptr()), ctypes.c_void_p(self.wsp),
                                           self.wsz, n._stream(self.torch)), "mdx_one_body_batch")


class DigestRun(ClassRun):
    """Preallocated densities and J blocks for repeated mdx_eri_digest_batch
    calls on one class (both sides contracted)."""

    def __init__(self, native, batch, ctx, torch, seed=2):
        super().__init__(native, batch, ctx, torch)
        del self.out
        g = torch.Generator(device="cuda").manual_seed(seed)
        nb, nk = self.bra.shape[0], self.ket.shape[0]
        self.Db = torch.randn(nb * self.nab, dtype=torch.float64, device="cuda", generator=g)
        self.Dk = torch.randn(nk * self.ncd, dtype=torch.float64, device="cuda", generator=g)
        self.Jb = torch.zeros(nb * self.nab, dtype=torch.float64, device="cuda")
        self.Jk = torch.zeros(nk * self.ncd, dtype=torch.float64, device="cuda")

    def __call__(self):
        n = self.native
        p = lambda t: ctypes.c_void_p(t.data_ptr())
        n.check(n.lib().mdx_eri_digest_batch(self.ctx.handle, ctypes.byref(self.sh.struct), self.batch.ncentre,
                                             self.bra.shape[0], n._i32p(self.bra), self.ket.shape[0],
                                             n._i32p(self.ket), 0, p(self.Db), p(self.Dk), p(self.Jb), p(self.Jk),
                                             ctypes.c_void_p(self.wsp), self.wsz, n._stream(self.torch)),
                "mdx_eri_digest_batch")


class NuclearRun(OneBodyRun):
    """Preallocated buffers for repeated mdx_nuclear_batch calls on one class."""

    def __init__(self, native, basis, pairs, charges, ctx, torch):
        super().__init__(native, basis, pairs, ctx, torch)
        self.charges = torch.as_tensor(charges, device="cuda")
        self.nch = int(self.charges.shape[0])
        del self.T
        L = native.lib()
        self.wsz = L.mdx_nuclear_workspace_size(ctx.handle, ctypes.byref(self.sh.struct), self.n,
                                                native._i32p(self.pairs), self.nch, 0)
        if self.wsz == 0:
            native.check(native.MDX_EINVAL, "nuclear workspace size")
        self.ws = torch.empty(self.wsz // 8 + 64, dtype=torch.float64, device="cuda")
        self.wsp = (self.ws.data_ptr() + 255) // 256 * 256

    def __call__(self):
        n = self.native
        n.check(n.lib().mdx_nuclear_batch(self.ctx.handle, ctypes.byref(self.sh.struct), self.n,
                                          n._i32p(self.pairs), self.nch, ctypes.c_void_p(self.charges.data_ptr()),
                                          0, ctypes.c_void_p(self.S.data_ptr()), ctypes.c_void_p(self.wsp),
                                          self.wsz, n._stream(self.torch)), "mdx_nuclear_batch")


class GradRun:
    """Preallocated buffers for repeated mdx_eri_grad_batch calls on one class."""

    def __init__(self, native, batch, ctx, torch, seed=1):
        from paper_2506_12501_amd import workloads as W
        self.native, self.batch, self.ctx, self.torch = native, batch, ctx, torch
        self.sh = native.DeviceShells(batch.basis)
        self.bra = native._pairs(batch.bra)
        self.ket = native._pairs(batch.ket)
        nab, ncd = native._class_sizes(self.sh, batch.ncentre, self.bra, self.ket, False)
        L = native.lib()
        self.wsz = L.mdx_eri_grad_workspace_size(ctx.handle, ctypes.byref(self.sh.struct), batch.ncentre,
                                                 self.bra.shape[0], native._i32p(self.bra), self.ket.shape[0],
                                                 native._i32p(self.ket), 0)
        if self.wsz == 0:
            native.check(native.MDX_EINVAL, "gradient workspace size")
        self.ws = torch.empty(self.wsz // 8 + 64, dtype=torch.float64, device="cuda")
        self.wsp = (self.ws.data_ptr() + 255) // 256 * 256
        self.n = self.bra.shape[0] * self.ket.shape[0]
        self.W = torch.as_tensor(W.adjoint(batch, nab, ncd, seed=seed), device="cuda")
        self.grad = torch.empty(self.n * 12, dtype=torch.float64, device="cuda")

    def __call__(self):
        n = self.native
        n.check(n.lib().mdx_eri_grad_batch(self.ctx.handle, ctypes.byref(self.sh.struct), self.batch.ncentre,
                                           self.bra.shape[0], n._i32p(self.bra), self.ket.shape[0],
                                           n._i32p(self.ket), 0, ctypes.c_void_p(self.W.data_ptr()),
                                           ctypes.c_void_p(self.grad.data_ptr()), ctypes.c_void_p(self.wsp),
                                           self.wsz, n._stream(self.torch)), "mdx_eri_grad_batch")


def measure(fn, nlaunch, reps, native, ctx, torch):
    """(ms per call, [mean kernel ms of launch j of a call]) over reps calls;
    kernel times come from the library's profiling hook."""
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    ev = HipEvents(2 * nlaunch * reps)
    native.check(native.lib().mdx_set_profile_events(ctx.handle, ev.ev, ev.n), "profile hook")
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    gc.disable()   # a collection pass inside the loop would stall the enqueueing thread
    t0.record()
    for _ in range(reps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    gc.enable()
    native.check(native.lib().mdx_set_profile_events(ctx.handle, None, 0), "profile hook off")
    ks = [ev.elapsed_ms(i) for i in range(nlaunch * reps)]
    ev.close()
    return t0.elapsed_time(t1) / reps, [sum(ks[j::nlaunch]) / reps for j in range(nlaunch)]


EXTRA_LEGS = ("gradient", "high_l", "sp_classes", "sp_hbm", "digest", "one_body", "nuclear")


def extra_legs(native, ctx, torch, tune, reps, legs=EXTRA_LEGS):
    """The other measured workloads (not part of the headline step)."""
    from paper_2506_12501_amd import autotune, flops as F, workloads as W
    out = {}

    def kfl(batch, grad=False):
        la, lb, lc, ld = W.parse_class(batch.name)
        Ks = [int(batch.basis.nprim[batch.bra[0, 0]]), int(batch.basis.nprim[batch.bra[0, 1]]) if lb >= 0 else 1,
              int(batch.basis.nprim[batch.ket[0, 0]]), int(batch.basis.nprim[batch.ket[0, 1]]) if ld >= 0 else 1]
        return (F.grad_shellset_flops if grad else F.shellset_flops)(la, lb, lc, ld, *Ks)

    if "gradient" in legs:
        # backward kernel: (dd|dd) K=3, 256 x 256 pairs, adjoint N(0,1) seed 1
        g = GradRun(native, W.config2("(dd|dd)"), ctx, torch, seed=1)
        variant, vt = None, None
        if tune:
            variant, vt = autotune.tune(ctx, g.sh, 4, g.bra, g.ket, g, reps=2, cache=False, gradient=True)
        ms, kms = measure(g, 2, reps, native, ctx, torch)
        fl = kfl(g.batch, grad=True) * g.n
        log("gradient leg done")
        out["gradient"] = {
            "workload": "(dd|dd) backward, K=3, 256x256 pairs (65,536 shellsets), adjoint N(0,1) seed 1, "
                        "12 centre derivatives per shellset",
            "ms_per_call": ms, "shellsets_per_s": g.n / (ms * 1e-3), "kernel_ms_per_pass": kms,
            "algorithmic_gflop": fl / 1e9, "kernel_tflops": fl / (sum(kms) * 1e-3) / 1e12,
            "pct_fp64_peak": 100 * fl / (sum(kms) * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, "variant": variant,
            "tuning_ms": vt, "flop_model": "flops.grad_shellset_flops"}
        del g

    if "high_l" in legs:
        # high-L primitive classes: (ff|ff), (gg|gg) 128 x 128; (X|dd) 256 x 256
        hl = {}
        for name in W.C4_CLASSES_4C + W.C4_CLASSES_3C + W.HIGH_L_CLASSES_4C:
            r = ClassRun(native, W.config4(name, seed=0), ctx, torch)
            v, vt = None, None
            if tune:
                v, vt = autotune.tune(ctx, r.sh, r.batch.ncentre, r.bra, r.ket, r, reps=2, cache=False)
            ms, kms = measure(r, 1, reps, native, ctx, torch)
            fl = kfl(r.batch) * r.n
            hl[name] = {"shellsets": r.n, "ms_per_call": ms, "kernel_ms": kms[0],
                        "shellsets_per_s": r.n / (ms * 1e-3), "kernel_tflops": fl / (kms[0] * 1e-3) / 1e12,
                        "out_write_GB_per_s": r.out.numel() * 8 / (kms[0] * 1e-3) / 1e9,
                        "pct_fp64_peak": 100 * fl / (kms[0] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, "variant": v,
                        "tuning_ms": vt}
            del r
        out["high_l"] = hl

    if "sp_classes" in legs:
        # plain s/p primitive classes: 16 x 16 pairs (256 shellsets) per class
        sp = {}
        for name in W.C1_CLASSES:
            r = ClassRun(native, W.config1(name, seed=0), ctx, torch)
            ms, kms = measure(r, 1, max(reps, 20), native, ctx, torch)
            sp[name] = {"shellsets": r.n, "us_per_call": ms * 1e3, "kernel_us": kms[0] * 1e3,
                        "shellsets_per_s": r.n / (ms * 1e-3)}
        out["sp_classes"] = sp

    if "sp_hbm" in legs:
        # the same classes at 4,096 x 4,096 pairs (16.8 M shellsets): these are
        # bound by writing the output, so the evidence is HBM bandwidth
        hb = {}
        for name in W.C1_CLASSES:
            r = ClassRun(native, W.config1(name, npair=4096, seed=0), ctx, torch)
            ms, kms = measure(r, 1, 3, native, ctx, torch)
            nbytes = r.out.numel() * 8
            hb[name] = {"shellsets": r.n, "out_GB": nbytes / 1e9, "ms_per_call": ms, "kernel_ms": kms[0],
                        "shellsets_per_s": r.n / (ms * 1e-3), "out_write_GB_per_s": nbytes / (kms[0] * 1e-3) / 1e9,
                        "hbm_frac": nbytes / (kms[0] * 1e-3) / (PEAK_HBM_GBS * 1e9)}
            del r
            torch.cuda.empty_cache()
        out["sp_hbm"] = hb
        log("s/p HBM leg done")

    if "digest" in legs:
        # the same batches contracted with densities in the kernels (Jbra and
        # Jket) instead of storing the integrals: the s/p classes at 4,096 x
        # 4,096 pairs and the two contracted d classes of the headline step
        dg = {}
        cases = [(name, W.config1(name, npair=4096, seed=0)) for name in W.C1_CLASSES] + \
                [(name + " K=3", W.config2(name, seed=0)) for name in W.C2_CLASSES]
        for key, b in cases:
            r = DigestRun(native, b, ctx, torch)
            ms, kms = measure(r, 1, 3, native, ctx, torch)
            nbytes = r.n * r.nab * r.ncd * 8
            ent = {"shellsets": r.n, "ms_per_call": ms, "kernel_ms": kms[0],
                   "shellsets_per_s": r.n / (kms[0] * 1e-3),
                   "output_GB_not_written": nbytes / 1e9}
            if key in out.get("sp_hbm", {}):
                ent["store_kernel_ms"] = out["sp_hbm"][key]["kernel_ms"]
                ent["speedup_vs_store"] = ent["store_kernel_ms"] / kms[0]
            dg[key] = ent
            del r
            torch.cuda.empty_cache()
        out["digest"] = dg
        log("digest leg done")

    if "one_body" in legs:
        # overlap + kinetic energy, spherical, K=3: 1024 x 1024 shell pairs per
        # class.  ms_per_call includes the upload of the host pair list.
        ob = {}
        # l <= 3: 1024 x 1024 pairs (one pair per lane); l = 4..6: 256 x 256
        # pairs (one pair per wave)
        for la, lb in [(0, 0), (1, 1), (2, 1), (2, 2), (3, 3), (4, 4), (5, 5), (6, 6)]:
            n1 = 1024 if la <= 3 else 256
            basis, pairs = W.one_body_pairs(la, lb, n1, n1, 3, seed=la * 3 + lb)
            r = OneBodyRun(native, basis, pairs, ctx, torch)
            ms, kms = measure(r, 1, 5, native, ctx, torch)
            # the prepared form: pair records resident, a run enqueues the kernel only
            pr = native.Prepared("one_body", r.sh, r.pairs, ctx=ctx)
            msp, _ = measure(pr.run, 1, 5, native, ctx, torch)
            del pr
            nbytes = 2 * r.n * r.nf * 8
            fl = F.one_body_flops(la, lb, 3, 3) * r.n
            ob["(%s|%s)" % ("spdfghi"[la], "spdfghi"[lb])] = {
                "pairs": r.n, "ms_per_call": ms, "ms_per_call_prepared": msp, "kernel_ms": kms[0],
                "pairs_per_s": r.n / (kms[0] * 1e-3),
                "out_write_GB_per_s": nbytes / (kms[0] * 1e-3) / 1e9,
                "hbm_frac": nbytes / (kms[0] * 1e-3) / (PEAK_HBM_GBS * 1e9),
                "kernel_tflops": fl / (kms[0] * 1e-3) / 1e12,
                "pct_fp64_peak": 100 * fl / (kms[0] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                "flop_model": "flops.one_body_flops"}
            del r
            torch.cuda.empty_cache()
        out["one_body"] = ob
        log("one-body leg done")

    if "nuclear" in legs:
        # 1-particle Coulomb integrals of 100 point charges (the paper's Table 2
        # setting), early summation over charges; 256 x 256 = 65,536 pairs per
        # class, K = 1 and K = 5
        nu = {}
        charges = W.point_charges(100, 10.0, seed=0)
        for K in (1, 5):
            # l_a + l_b <= 6: 256 x 256 pairs, one per lane; beyond, one pair per
            # wave: 64 x 64 pairs, K = 1 only
            for la, lb in [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2), (3, 0), (3, 1), (3, 3), (4, 2), (6, 0),
                           (4, 4), (5, 5), (6, 6)]:
                if K > 1 and la + lb > 6:
                    continue
                n1 = 256 if la + lb <= 6 else 64
                basis, pairs = W.one_body_pairs(la, lb, n1, n1, K, seed=10 * K + la * 3 + lb)
                r = NuclearRun(native, basis, pairs, charges, ctx, torch)
                ms, kms = measure(r, 1, 5, native, ctx, torch)
                pr = native.Prepared("nuclear", r.sh, r.pairs, r.nch, ctx=ctx)
                msp, _ = measure(lambda: pr.run(r.charges), 1, 5, native, ctx, torch)
                del pr
                fl = F.nuclear_flops(la, lb, K, K, 100) * r.n
                nu["(%s|%s) K=%d" % ("spdfghi"[la], "spdfghi"[lb], K)] = {
                    "pairs": r.n, "charges": 100, "ms_per_call": ms, "ms_per_call_prepared": msp,
                    "kernel_ms": kms[0],
                    "pairs_per_s": r.n / (kms[0] * 1e-3), "kernel_tflops": fl / (kms[0] * 1e-3) / 1e12,
                    "pct_fp64_peak": 100 * fl / (kms[0] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                    "flop_model": "flops.nuclear_flops"}
                del r
        out["nuclear"] = nu
        log("nuclear-attraction leg done")

    return out


def cluster_leg(native, ctx, torch, reps, sample, tune=True):
    """Mixed-L screened batch over the 32-molecule water-like cluster: every
    canonical class in one plan; plain per-class launches vs one fused graph."""
    import numpy as np
    from oracle import oracle as O
    from paper_2506_12501_amd import flops as F, screening as S, workloads as W
    from tests.cluster_util import oracle_Q
    from tests.gpu_util import ATOL, RTOL
    b, _ = W.water_cluster(seed=0)
    sh = native.DeviceShells(b)
    P = S.canonical_pairs(b.l, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Qd = {pc: native.schwarz(sh, p) for pc, p in P.items()}
    torch.cuda.synchronize()
    schwarz_ms = (time.perf_counter() - t0) * 1e3
    Q = {pc: q.cpu().numpy() for pc, q in Qd.items()}
    batches = S.class_batches(P, Q, 1e-12, nprim=b.nprim)
    total = S.with_offsets(batches, b.l)
    nquart = sum(bt["quartets"] for bt in batches)
    log(f"cluster: {len(b.l)} shells, {sum(p.shape[0] for p in P.values())} pairs, {len(batches)} batches, "
        f"{nquart} quartets, {total * 8 / 1e9:.2f} GB output")
    # tile shapes per class for the fused plan (the plain baseline keeps the defaults)
    nb = [native.Batch(4, bt["bra"], bt["ket"], bt["bra_count"], bt["out_offset"]) for bt in batches]
    plain = native.Plan(sh, nb, fused=False)
    from paper_2506_12501_amd import autotune
    tuned = autotune.tune_batches(ctx, sh, batches) if tune else {}
    log(f"cluster tuning: { {k: v[0] for k, v in tuned.items()} }")
    fused = native.Plan(sh, nb, fused=True)
    # the same per-batch launches as `plain`, with the tuned kernels: fusion
    # alone is plain_tuned / fused
    plain_tuned = native.Plan(sh, nb, fused=False) if tuned else None
    for name, (best, _) in tuned.items():   # back to the defaults for everything after this leg
        la, lb = (int(x) for x in b.l[next(bt for bt in batches if bt["name"] == name)["bra"][0]])
        lc, ld = (int(x) for x in b.l[next(bt for bt in batches if bt["name"] == name)["ket"][0]])
        ctx.set_variant(4, la, lb, lc, ld, 0, -1)
    o_plain = torch.empty(total, dtype=torch.float64, device="cuda")
    o_fused = torch.empty(total, dtype=torch.float64, device="cuda")

    def timed(plan, out):
        plan.execute(out)                       # warm-up (graph capture for the fused plan)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        ts = []
        gc.disable()
        for _ in range(reps):
            e0.record()
            plan.execute(out)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        gc.enable()
        return ts

    t_plain = timed(plain, o_plain)
    t_fused = timed(fused, o_fused)
    t_plain_tuned = timed(plain_tuned, o_plain) if plain_tuned is not None else None
    # the same screened batches contracted with pair-blocked densities in the
    # kernels (MDX_DIGEST plan, plain launches; both J sides of every quartet)
    # instead of writing the 2.1 GB of integrals
    dplan = native.Plan(sh, nb, digest=True)
    g = torch.Generator(device="cuda").manual_seed(3)
    blocks = []
    for bt in batches:
        nbra, nket = len(bt["bra"]), len(bt["ket"])
        Db = torch.randn(nbra * bt["nab"], dtype=torch.float64, device="cuda", generator=g)
        Dk = torch.randn(nket * bt["ncd"], dtype=torch.float64, device="cuda", generator=g)
        blocks.append((Db, Dk, torch.zeros_like(Db), torch.zeros_like(Dk)))

    class _Digest:
        def __init__(self, plan):
            self.plan = plan

        def execute(self, out=None):
            self.plan.digest(blocks)
    t_digest = timed(_Digest(dplan), None)
    # and as one graph of persistent digesting kernels
    t_digest_fused = timed(_Digest(native.Plan(sh, nb, digest=True, fused=True)), None)
    log(f"cluster: digesting plan {min(t_digest):.2f} ms, digesting graph {min(t_digest_fused):.2f} ms")
    identical = bool(torch.equal(o_plain, o_fused))        # expected only where tuning kept the default kernels
    max_diff = float((o_plain - o_fused).abs().max())
    log(f"cluster: plain {min(t_plain):.2f} ms, fused {min(t_fused):.2f} ms")
    # algorithmic FLOPs with each pair's own contraction degree
    Kp = lambda pairs: b.nprim[pairs[:, 0]].astype(np.float64) * b.nprim[pairs[:, 1]]
    flops = 0.0
    for bt in batches:
        la, lb = b.l[bt["bra"][0]]
        lc, ld = b.l[bt["ket"][0]]
        f11 = F.shellset_flops(la, lb, lc, ld, 1, 1, 1, 1)
        per_q = F.shellset_flops(la, lb, lc, ld, 1, 1, 2, 1) - f11
        per_b = f11 - per_q
        kb, kk = Kp(bt["bra"]), Kp(bt["ket"])
        csum = np.concatenate([[0.0], np.cumsum(kb)])
        sb = csum[bt["bra_count"]]                      # sum of K_bra over each ket's prefix
        flops += float(np.sum(sb * kk) * per_q + np.sum(sb) * per_b)
    # stratified parity sample against the __float128 oracle
    rng = np.random.default_rng(11)
    out_h = None
    nchk = nbad = nqq_only = 0
    worst_cs = 0.0
    for bt in batches:
        cnt = bt["bra_count"]
        starts = np.concatenate([[0], np.cumsum(cnt)])
        pick = np.unique(rng.integers(0, bt["quartets"], min(sample, bt["quartets"])))
        ks = np.searchsorted(starts, pick, side="right") - 1
        iis = pick - starts[ks]
        qs = np.stack([iis, ks], axis=1)
        ref = O.eri(b, 4, bt["bra"], bt["ket"], quartets=qs, quad=True)          # [q, nab, ncd]
        qq = oracle_Q(b, bt["bra"])[iis] * oracle_Q(b, bt["ket"])[ks]
        nab, ncd = bt["nab"], bt["ncd"]
        obase = np.concatenate([[0], np.cumsum(cnt.astype(np.int64) * nab * ncd)])
        ab, cd = np.meshgrid(np.arange(nab), np.arange(ncd), indexing="ij")
        idx = (bt["out_offset"] + obase[ks][:, None, None] + iis[:, None, None]
               + cnt[ks][:, None, None] * (ab[None] + nab * cd[None]))
        got = o_fused[torch.as_tensor(idx.reshape(-1), device="cuda")].cpu().numpy().reshape(ref.shape)
        err = np.abs(got - ref)
        g13 = (err <= ATOL) | (err <= RTOL * np.abs(ref))
        ok = g13 | (err <= 1e-12 * qq[:, None, None])
        nchk += ok.size
        nbad += int(np.count_nonzero(~ok))
        nqq_only += int(np.count_nonzero(ok & ~g13))
        worst_cs = max(worst_cs, float(np.max(err / qq[:, None, None])))
    best_f, best_p = min(t_fused), min(t_plain)
    return {
        "workload": "32 water-like molecules (96 atoms, 3 A simple-cubic lattice, 384 shells, 800 primitives, "
                    "768 spherical AOs); heavy s K=(8,1,1), p K=(3,1), d K=1; light s K=(3,1), p K=1; zeta "
                    "log-U[0.1,5000]; canonical quartets with Q_ab Q_cd >= 1e-12, 21 classes split into batches of equal (K_bra, K_ket), seed 0",
        "classes": len({bt["name"] for bt in batches}), "batches": len(batches), "quartets": nquart,
        "output_gb": total * 8 / 1e9,
        "schwarz_ms": schwarz_ms,
        "plain_ms": best_p, "fused_ms": best_f, "plain_ms_all": t_plain, "fused_ms_all": t_fused,
        "digest_plain_ms": min(t_digest), "digest_plain_ms_all": t_digest,
        "digest_fused_ms": min(t_digest_fused), "digest_fused_ms_all": t_digest_fused,
        "plain_tuned_ms": min(t_plain_tuned) if t_plain_tuned else None, "plain_tuned_ms_all": t_plain_tuned,
        "fused_speedup": best_p / best_f,
        "fusion_only_speedup": min(t_plain_tuned) / best_f if t_plain_tuned else None,
        "outputs_identical": identical, "max_abs_diff_plain_fused": max_diff,
        "fused_tuning": {k: {"variant": v[0], "ms": {str(a): t for a, t in v[1].items()}} for k, v in tuned.items()},
        "plain_uses": "default kernel choice per class",
        "shellsets_per_s_fused": nquart / (best_f * 1e-3),
        "algorithmic_gflop": flops / 1e9, "fused_tflops": flops / (best_f * 1e-3) / 1e12,
        "pct_fp64_peak_fused": 100 * flops / (best_f * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
        "parity_sample": {"checked": nchk, "failed": nbad, "passed_only_by_QQ_clause": nqq_only,
                          "max_err_over_QQ": worst_cs, "reference": "__float128 oracle",
                          "tolerance": "|err| <= 1e-12 or <= 1e-10 |ref| or <= 1e-12 Q_ab Q_cd",
                          "sample": f"up to {sample} quartets per class, uniform"},
        "per_class_quartets": {n: sum(bt["quartets"] for bt in batches if bt["name"] == n)
                               for n in dict.fromkeys(bt["name"] for bt in batches)},
    }


def class_flops(batch):
    from paper_2506_12501_amd import flops as F, workloads as W
    la, lb, lc, ld = W.parse_class(batch.name)
    K = int(batch.basis.nprim[0])
    return F.shellset_flops(la, lb, lc, ld, K, K if lb >= 0 else 1, K, K if ld >= 0 else 1)


def cpu_model():
    """CPU model name of this host (from /proc/cpuinfo)"""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


_SINGLE_THREAD = """
import json, sys, time
sys.path.insert(0, {root!r})
from oracle import oracle as O
from paper_2506_12501_amd import workloads as W
n, t = 0, 0.0
for name in {names!r}:
    b = W.config2(name, npair={npair}, seed=0)
    bra, ket = b.bra[:{m}], b.ket[:{m}]
    t0 = time.perf_counter()
    O.eri(b.basis, b.ncentre, bra, ket)
    t += time.perf_counter() - t0
    n += bra.shape[0] * ket.shape[0]
print(json.dumps({{"shellsets": n, "seconds": t}}))
"""


def cpu_single_thread(names, npair, m):
    """The oracle on one thread (a child process with OMP_NUM_THREADS=1 that
    touches no GPU) over the first m x m shellsets of each class."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", _SINGLE_THREAD.format(root=ROOT, names=list(names), npair=npair, m=m)],
                       capture_output=True, text=True, env=env, timeout=600)
    if r.returncode != 0:
        log("single-thread oracle run failed: " + r.stderr[-500:])
        return None
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value": d["shellsets"] / d["seconds"], "cores": 1,
            "sample": f"{m}x{m} shellsets of each class, {d['shellsets']} shellsets, {d['seconds']:.1f} s"}


def cpu_baseline(runs, sample_pairs):
    """The oracle, as it stands, on the first sample_pairs x sample_pairs shellsets
    of each class; all host threads (OpenMP).  Also returns its parity against
    the GPU output of the same shellsets."""
    import numpy as np
    from oracle import oracle as O
    from tests.gpu_util import ATOL, RTOL
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    total_t, total_n = 0.0, 0
    worst_abs, worst_rel, nbad, nchk = 0.0, 0.0, 0, 0
    for r in runs:
        b = r.batch
        bra, ket = b.bra[:sample_pairs], b.ket[:sample_pairs]
        t0 = time.perf_counter()
        ref = O.eri(b.basis, b.ncentre, bra, ket)
        total_t += time.perf_counter() - t0
        total_n += bra.shape[0] * ket.shape[0]
        got = r.view()[:sample_pairs, :, :, :sample_pairs].cpu().numpy()
        err = np.abs(got - ref)
        ok = (err <= ATOL) | (err <= RTOL * np.abs(ref))
        nbad += int(np.count_nonzero(~ok))
        nchk += ok.size
        worst_abs = max(worst_abs, float(err.max()))
        worst_rel = max(worst_rel, float(np.max(err / np.maximum(np.abs(ref), 1e-300) * (err > ATOL))))
    return {"value": total_n / total_t, "unit": "shellsets/s", "cores": nthreads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{sample_pairs}x{sample_pairs} shellsets of each class (first pairs of the workload), "
                      f"{total_n} shellsets, {total_t:.1f} s"}, \
           {"checked": nchk, "failed": nbad, "max_abs_err": worst_abs, "max_rel_err_above_atol": worst_rel,
            "tolerance": "per element |gpu-oracle| <= 1e-12 or <= 1e-10 |oracle|"}


def load_traffic(kernel_tag):
    """HBM bytes per launch from profiles/<tag>_traffic.json, if it was
    measured on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("source_sha256_16") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


KERNEL_SOURCES = ["eri_mfma.hip", "eri_mfma.h", "mfma_common.h", "cube_layouts.h", "eri_common.h", "kernels.h",
                  "mdx_internal.h", "boys_device.h", "eri.cpp"]


def kernel_source_hash():
    """sha256 (16 hex digits) over the sources of the forward matrix-core kernel and its launch"""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2506_12501_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def _r(x, sig=5):
    """round floats (recursively) to `sig` significant digits for the compact line"""
    if isinstance(x, float):
        return float(f"{x:.{sig}g}")
    if isinstance(x, dict):
        return {k: _r(v, sig) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_r(v, sig) for v in x]
    return x


COMPACT_MAX_BYTES = 4096


def compact_record(full, detail_path=None):
    """The one JSON line printed on stdout: the headline keys, the roofline of
    the dominant kernel, the CPU baseline, parity and one-number summaries of
    the other legs (their full records go to the detail file)."""
    keys = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
            "vs_baseline", "dtype", "data", "config", "step_tflops_algorithmic", "step_pct_fp64_peak", "roofline",
            "cpu_baseline")
    rec = {k: full.get(k) for k in keys}
    rec["per_class"] = {n: {k: c[k] for k in ("kernel_ms", "pct_fp64_peak", "shellsets_per_s_kernel")}
                        for n, c in (full.get("per_class") or {}).items()}
    if full.get("parity_sample"):
        p = full["parity_sample"]
        rec["parity_sample"] = {k: p[k] for k in ("checked", "failed", "max_abs_err")}
    cl = full.get("mixed_cluster")
    if cl:
        rec["mixed_cluster"] = {k: cl.get(k) for k in ("quartets", "plain_ms", "plain_tuned_ms", "fused_ms",
                                                        "fused_speedup", "fusion_only_speedup",
                                                        "pct_fp64_peak_fused", "digest_plain_ms",
                                                        "digest_fused_ms")}
        ps = cl["parity_sample"]
        rec["mixed_cluster"]["parity"] = {k: ps.get(k) for k in ("checked", "failed", "passed_only_by_QQ_clause",
                                                                 "max_err_over_QQ")}
    ex = full.get("extras") or {}
    summ = {}
    if "gradient" in ex:
        summ["gradient_pct_fp64_peak"] = ex["gradient"]["pct_fp64_peak"]
        summ["gradient_ms_per_call"] = ex["gradient"]["ms_per_call"]
    if "high_l" in ex:
        summ["high_l_pct_fp64_peak"] = {n: v["pct_fp64_peak"] for n, v in ex["high_l"].items()}
    if "sp_hbm" in ex:
        summ["sp_hbm_frac"] = {n: v["hbm_frac"] for n, v in ex["sp_hbm"].items()}
    if "digest" in ex:
        summ["digest_kernel_ms"] = {n: v["kernel_ms"] for n, v in ex["digest"].items()}
    if "one_body" in ex:
        summ["one_body_pct_fp64_peak"] = {n: v["pct_fp64_peak"] for n, v in ex["one_body"].items()}
        pc = {n: v["ms_per_call_prepared"] / v["kernel_ms"] for n, v in ex["one_body"].items()
              if "ms_per_call_prepared" in v}
        if pc:
            summ["one_body_prepared_call_over_kernel"] = pc
    if "nuclear" in ex:
        summ["nuclear_kernel_ms"] = {n: v["kernel_ms"] for n, v in ex["nuclear"].items()}
    if summ:
        rec["extras_summary"] = summ
    rec["detail"] = detail_path
    rec = _r(rec)
    # keep the line short: drop the largest summaries first if it ever grows
    for k in ("one_body_prepared_call_over_kernel", "nuclear_kernel_ms", "digest_kernel_ms", "one_body_pct_fp64_peak",
              "sp_hbm_frac"):
        if len(json.dumps(rec, separators=(",", ":"))) <= COMPACT_MAX_BYTES:
            break
        rec.get("extras_summary", {}).pop(k, None)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--npair", type=int, default=256)
    ap.add_argument("--cpu-sample", type=int, default=224)
    ap.add_argument("--no-extras", action="store_true", help="skip the gradient / high-L / s-p legs")
    ap.add_argument("--extra-reps", type=int, default=5)
    ap.add_argument("--extras", default=",".join(EXTRA_LEGS),
                    help="comma-separated extra legs to run (default: all of %s)" % ", ".join(EXTRA_LEGS))
    ap.add_argument("--no-cluster", action="store_true", help="skip the mixed-L cluster leg")
    ap.add_argument("--cluster-sample", type=int, default=48)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only copy this many MiB device-to-device (HBM counter calibration)")
    ap.add_argument("--classes", default=None, help="comma-separated subset of the workload's classes")
    ap.add_argument("--detail-out", default=os.path.join("gpurun_out", "bench_detail.json"),
                    help="file for the full record of every leg (the stdout line is a compact summary)")
    ap.add_argument("--cpu-single-sample", type=int, default=24,
                    help="m: the single-thread oracle times m x m shellsets of each class")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the integral batches shard "
                                   "across GPUs by ket-pair blocks (see DESIGN.md), but no multi-GPU "
                                   "run is part of this build", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2506_12501_amd import native, workloads as W

    ctx = native.Context.get(0)
    names = args.classes.split(",") if args.classes else W.C2_CLASSES
    runs = [ClassRun(native, W.config2(name, npair=args.npair, seed=0), ctx, torch) for name in names]
    log("workload built")
    nshell = sum(r.n for r in runs)

    # autotuner (untimed): fastest kernel variant per class on this workload
    tuning = {}
    if not args.no_tune:
        from paper_2506_12501_amd import autotune
        for r in runs:
            best, times = autotune.tune(ctx, r.sh, r.batch.ncentre, r.bra, r.ket, r, reps=2, cache=False)
            tuning[r.batch.name] = {"variant": best, "ms": {str(k): v for k, v in times.items()}}

    log(f"tuning done: {tuning}")

    def step():
        for r in runs:
            r()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # integral-kernel events through the library hook: launch i of the timed
    # region uses pair i; classes alternate in call order
    ev = HipEvents(2 * len(runs) * args.steps)
    native.check(native.lib().mdx_set_profile_events(ctx.handle, ev.ev, ev.n), "profile hook")
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    t0.record()
    wall0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    gc.enable()
    wall = time.perf_counter() - wall0
    native.check(native.lib().mdx_set_profile_events(ctx.handle, None, 0), "profile hook off")
    ms_step = t0.elapsed_time(t1) / args.steps
    log(f"timed region done: {ms_step:.3f} ms per step")

    per_class = {}
    for ci, r in enumerate(runs):
        ks = [ev.elapsed_ms(s * len(runs) + ci) for s in range(args.steps)]
        kms = sum(ks) / len(ks)
        fl = class_flops(r.batch) * r.n
        per_class[r.batch.name] = {
            "shellsets": r.n, "kernel_ms": kms, "algorithmic_gflop": fl / 1e9,
            "kernel_tflops": fl / (kms * 1e-3) / 1e12,
            "pct_fp64_peak": 100.0 * fl / (kms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "shellsets_per_s_kernel": r.n / (kms * 1e-3),
        }
    ev.close()
    dom = runs[0].batch.name
    pc = per_class[dom]
    traffic = load_traffic("eri_mfma_dddd_k3")
    roofline = {"bound": "mfma", "achieved": pc["kernel_tflops"], "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": pc["kernel_tflops"] / PEAK_FP64_TFLOPS, "traffic": traffic,
                "kernel": "eri_mfma_kernel (dd|dd) K=3, 65,536 shellsets per launch",
                "flops_per_launch": pc["algorithmic_gflop"] * 1e9}

    extras = None
    if not args.no_extras:
        extras = extra_legs(native, ctx, torch, not args.no_tune, args.extra_reps, args.extras.split(","))
        log("extra legs done")
    cluster = None
    if not args.no_cluster:
        cluster = cluster_leg(native, ctx, torch, args.extra_reps, args.cluster_sample, not args.no_tune)
        log("cluster leg done")

    cpu, parity = (None, None)
    if not args.no_cpu:
        cpu, parity = cpu_baseline(runs, args.cpu_sample)
        cpu["single_thread"] = cpu_single_thread(names, args.npair, args.cpu_single_sample)
        log("cpu baseline done")

    total_flops = sum(class_flops(r.batch) * r.n for r in runs)
    rec = {
        "metric": METRIC,
        "value": nshell / (ms_step * 1e-3),
        "unit": "shellsets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "contracted (dd|dd) + (pd|dd), K=3 per shell, 256x256 shell pairs per class "
                               "(65,536 shellsets each), zeta log-U[0.05,50], c U[0.1,1], 10 A box, seed 0",
                   "classes": [r.batch.name for r in runs], "shellsets_per_step": nshell},
        "step_tflops_algorithmic": total_flops / (ms_step * 1e-3) / 1e12,
        "step_pct_fp64_peak": 100.0 * total_flops / (ms_step * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
        "per_class": per_class,
        "tuning": tuning,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_sample": parity,
        "extras": extras,
        "mixed_cluster": cluster,
        "wall_s_timed": wall,
    }
    detail = None
    if args.detail_out:
        try:
            os.makedirs(os.path.dirname(os.path.abspath(args.detail_out)), exist_ok=True)
            with open(args.detail_out, "w") as f:
                json.dump(rec, f, indent=1)
            detail = args.detail_out
        except OSError as e:
            log(f"could not write {args.detail_out}: {e}")
    if extras:
        for leg, v in extras.items():
            log(f"{leg}: " + json.dumps(_r(v, 4))[:2000])
    if cluster:
        log("mixed_cluster: " + json.dumps(_r({k: v for k, v in cluster.items() if k != "fused_tuning"}, 4))[:2000])
    print(json.dumps(compact_record(rec, detail), separators=(",", ":")), flush=True)


if __name__ == "__main__":
    main()
