"""Autotuner: per class, time every compiled kernel variant on the caller's
batch and keep the fastest (replaces the paper's compile-time tile choice,
Sec. 3.1).  Results are cached as JSON keyed by device architecture, class
and contraction degrees, and applied through mdx_set_variant.
"""
from __future__ import annotations

import ctypes
import json
import os

from . import native

CACHE = os.environ.get("MDX_TUNE_CACHE", os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json"))


def _class_of(shells: "native.DeviceShells", ncentre, bra, ket):
    la = int(shells.l[bra[0, 0]])
    lb = int(shells.l[bra[0, 1]]) if ncentre == 4 else -1
    lc = int(shells.l[ket[0, 0]])
    ld = int(shells.l[ket[0, 1]]) if ncentre >= 3 else -1
    Kb = int(shells.nprim[bra[0, 0]]) * (int(shells.nprim[bra[0, 1]]) if ncentre == 4 else 1)
    Kk = int(shells.nprim[ket[0, 0]]) * (int(shells.nprim[ket[0, 1]]) if ncentre >= 3 else 1)
    return la, lb, lc, ld, Kb, Kk


def key_string(arch, ncentre, la, lb, lc, ld, cartesian, Kb, Kk, gradient=False):
    kind = ("cart" if cartesian else "sph") + ("+grad" if gradient else "")
    return f"{arch}|{ncentre}|{la},{lb},{lc},{ld}|{kind}|K{Kb}x{Kk}"


def _flags(cartesian, gradient):
    return (native.MDX_CARTESIAN if cartesian else 0) | (native.MDX_GRADIENT if gradient else 0)


def variants(ctx: "native.Context", ncentre, la, lb, lc, ld, cartesian, gradient=False) -> list:
    """Variant ids the library has for this class (probing mdx_set_variant);
    gradient=True: the backward kernel's tile shapes."""
    L = native.lib()
    fl = _flags(cartesian, gradient)
    out = []
    for v in range(0, 32):
        st = L.mdx_set_variant(ctx.handle, ncentre, la, max(lb, 0), lc, max(ld, 0), fl, v)
        if st == native.MDX_OK:
            out.append(v)
        elif v > 0:
            break
    L.mdx_set_variant(ctx.handle, ncentre, la, max(lb, 0), lc, max(ld, 0), fl, -1)
    return out


def time_call(fn, reps=3):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        t0.record()
        fn()
        t1.record()
        torch.cuda.synchronize()
        best = min(best, t0.elapsed_time(t1))
    return best


def tune(ctx, shells, ncentre, bra, ket, call, cartesian=False, reps=3, cache=True, gradient=False):
    """call(): runs the batch once with the context's current variant
    (gradient=True: the backward call, tuning the backward kernel).
    Returns (best_variant, {variant: ms})."""
    import torch
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "gfx950")
    la, lb, lc, ld, Kb, Kk = _class_of(shells, ncentre, bra, ket)
    key = key_string(arch, ncentre, la, lb, lc, ld, cartesian, Kb, Kk, gradient)
    L = native.lib()
    fl = _flags(cartesian, gradient)
    times = {}
    for v in variants(ctx, ncentre, la, lb, lc, ld, cartesian, gradient):
        native.check(L.mdx_set_variant(ctx.handle, ncentre, la, max(lb, 0), lc, max(ld, 0), fl, v),
                     "mdx_set_variant")
        try:
            times[v] = time_call(call, reps)
        except native.MdxError as e:
            if e.status != native.MDX_EUNSUPPORTED:   # a variant that does not serve this batch
                raise
    best = min(times, key=times.get)
    native.check(L.mdx_set_variant(ctx.handle, ncentre, la, max(lb, 0), lc, max(ld, 0), fl, best),
                 "mdx_set_variant")
    if cache:
        data = load_cache()
        data[key] = {"variant": best, "ms": times}
        save_cache(data)
    return best, times


def load_cache(path: str = CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_cache(data: dict, path: str = CACHE) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def apply_cache(ctx, path: str = CACHE) -> int:
    """Apply every cached choice for this device; returns how many."""
    import torch
    arch = getattr(torch.cuda.get_device_properties(0), "gcnArchName", "gfx950")
    n = 0
    for key, rec in load_cache(path).items():
        a, nc, ls, kind, _ = key.split("|")
        if a != arch:
            continue
        la, lb, lc, ld = (int(x) for x in ls.split(","))
        fl = _flags(kind.startswith("cart"), kind.endswith("+grad"))
        st = native.lib().mdx_set_variant(ctx.handle, int(nc), la, max(lb, 0), lc, max(ld, 0), fl,
                                          int(rec["variant"]))
        n += st == native.MDX_OK
    return n


def tune_batches(ctx, shells, batches, cartesian=False, reps=2, fused=True):
    """Pick a kernel variant per class for a list of plan batches (dicts with
    bra, ket, bra_count, out_offset as built by screening.class_batches): for
    every class with several variants, time a plan of that class's batches
    under each variant and keep the fastest.  fused=True times the class's
    persistent work-queue launch (the form a fused plan runs), False the
    plain per-batch launches.  Returns {class name: (best, {variant: ms})};
    the choices stay set on ctx, so plans created afterwards use them."""
    import torch
    by_class = {}
    for bt in batches:
        by_class.setdefault(bt["name"], []).append(bt)
    L = native.lib()
    out = {}
    for name, bts in by_class.items():
        la, lb = (int(x) for x in shells.l[bts[0]["bra"][0]])
        lc, ld = (int(x) for x in shells.l[bts[0]["ket"][0]])
        vs = variants(ctx, 4, la, lb, lc, ld, cartesian)
        if len(vs) < 2:
            continue
        times = {}
        for v in vs:
            native.check(L.mdx_set_variant(ctx.handle, 4, la, lb, lc, ld, int(cartesian), v), "mdx_set_variant")
            off = 0
            nb = []
            for bt in bts:
                nb.append(native.Batch(4, bt["bra"], bt["ket"], bt["bra_count"], off))
                off += bt["quartets"] * bt["nab"] * bt["ncd"]
            try:
                plan = native.Plan(shells, nb, cartesian=cartesian, fused=fused, ctx=ctx)
            except native.MdxError:
                continue
            o = torch.empty(max(plan.out_size, 1), dtype=torch.float64, device=shells.center.device)
            times[v] = time_call(lambda: plan.execute(o), reps)
            del plan, o
        if not times:
            continue
        best = min(times, key=times.get)
        native.check(L.mdx_set_variant(ctx.handle, 4, la, lb, lc, ld, int(cartesian), best), "mdx_set_variant")
        out[name] = (best, times)
    return out
