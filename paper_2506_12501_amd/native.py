"""ctypes binding of libmdx.so (include/mdx.h).  Argument marshalling only:
every step of the integral evaluation runs in the library's HIP kernels.
PyTorch provides device memory and the current stream.

The library is loaded on first use; if it is missing the call raises -- there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmdx.so")

MDX_OK, MDX_EINVAL, MDX_EUNSUPPORTED, MDX_EWORKSPACE, MDX_ENOMEM, MDX_EDEVICE = range(6)
MDX_SPHERICAL, MDX_CARTESIAN, MDX_FUSED, MDX_GRADIENT, MDX_PAIRED, MDX_DIGEST = 0, 1, 2, 4, 8, 16
MDX_NOALLOC_SCRATCH_BYTES = 64 << 20     # static scratch of mdx_eri_batch_noalloc, per device

_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_pi32 = ctypes.POINTER(ctypes.c_int32)


class MdxShells(ctypes.Structure):
    _fields_ = [("nshell", _i32), ("center", _p), ("exponent", _p), ("coef", _p),
                ("l", _pi32), ("nprim", _pi32), ("prim_offset", _pi32)]


class MdxBatchDesc(ctypes.Structure):
    _fields_ = [("ncentre", ctypes.c_int), ("nbra", _i32), ("bra", _pi32), ("nket", _i32),
                ("ket", _pi32), ("bra_count", _pi32), ("out_offset", ctypes.c_int64)]


class MdxDigestBlock(ctypes.Structure):
    _fields_ = [("Dbra", _p), ("Dket", _p), ("Jbra", _p), ("Jket", _p)]


class MdxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None
_lock = threading.Lock()

EXPORTS = {
    "mdx_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_p)]),
    "mdx_destroy": (None, [_p]),
    "mdx_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "mdx_last_error": (ctypes.c_char_p, []),
    "mdx_boys": (ctypes.c_int, [_p, _i32, _p, ctypes.c_int, _p, _p]),
    "mdx_eri_workspace_size": (ctypes.c_size_t, [_p, ctypes.POINTER(MdxShells), ctypes.c_int, _i32, _pi32,
                                                 _i32, _pi32, ctypes.c_int]),
    "mdx_eri_batch": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), ctypes.c_int, _i32, _pi32, _i32, _pi32,
                                     ctypes.c_int, _p, _p, ctypes.c_size_t, _p]),
    "mdx_eri_batch_noalloc": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), ctypes.c_int, _i32, _pi32, _i32,
                                             _pi32, ctypes.c_int, _p, _p]),
    "mdx_eri_digest_batch": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), ctypes.c_int, _i32, _pi32, _i32, _pi32,
                                            ctypes.c_int, _p, _p, _p, _p, _p, ctypes.c_size_t, _p]),
    "mdx_eri_grad_workspace_size": (ctypes.c_size_t, [_p, ctypes.POINTER(MdxShells), ctypes.c_int, _i32,
                                                      _pi32, _i32, _pi32, ctypes.c_int]),
    "mdx_eri_grad_batch": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), ctypes.c_int, _i32, _pi32, _i32,
                                          _pi32, ctypes.c_int, _p, _p, _p, ctypes.c_size_t, _p]),
    "mdx_one_body_workspace_size": (ctypes.c_size_t, [_p, ctypes.POINTER(MdxShells), _i32, _pi32, ctypes.c_int]),
    "mdx_one_body_batch": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), _i32, _pi32, ctypes.c_int, _p, _p, _p,
                                          ctypes.c_size_t, _p]),
    "mdx_nuclear_workspace_size": (ctypes.c_size_t, [_p, ctypes.POINTER(MdxShells), _i32, _pi32, _i32,
                                                     ctypes.c_int]),
    "mdx_nuclear_batch": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), _i32, _pi32, _i32, _p, ctypes.c_int, _p,
                                         _p, ctypes.c_size_t, _p]),
    "mdx_schwarz_workspace_size": (ctypes.c_size_t, [_p, ctypes.POINTER(MdxShells), _i32, _pi32, ctypes.c_int]),
    "mdx_schwarz": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), _i32, _pi32, ctypes.c_int, _p, _p,
                                   ctypes.c_size_t, _p]),
    "mdx_eri_prepare": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), ctypes.c_int, _i32, _pi32, _i32, _pi32,
                                       ctypes.c_int, ctypes.POINTER(_p)]),
    "mdx_eri_run": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), _p, _p, ctypes.c_size_t, _p]),
    "mdx_one_body_prepare": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), _i32, _pi32, ctypes.c_int,
                                            ctypes.POINTER(_p)]),
    "mdx_one_body_run": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), _p, _p, _p, ctypes.c_size_t, _p]),
    "mdx_nuclear_prepare": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), _i32, _pi32, _i32, ctypes.c_int,
                                           ctypes.POINTER(_p)]),
    "mdx_nuclear_run": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), _p, _p, _p, ctypes.c_size_t, _p]),
    "mdx_batch_workspace_size": (ctypes.c_size_t, [_p]),
    "mdx_batch_output_size": (ctypes.c_int64, [_p]),
    "mdx_batch_destroy": (None, [_p]),
    "mdx_plan_create": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), ctypes.c_int,
                                       ctypes.POINTER(MdxBatchDesc), ctypes.c_int, ctypes.POINTER(_p)]),
    "mdx_plan_workspace_size": (ctypes.c_size_t, [_p]),
    "mdx_plan_output_size": (ctypes.c_int64, [_p]),
    "mdx_plan_execute": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), _p, _p, ctypes.c_size_t, _p]),
    "mdx_plan_digest": (ctypes.c_int, [_p, ctypes.POINTER(MdxShells), ctypes.POINTER(MdxDigestBlock), _p,
                                       ctypes.c_size_t, _p]),
    "mdx_plan_destroy": (None, [_p]),
    "mdx_set_profile_events": (ctypes.c_int, [_p, ctypes.POINTER(_p), ctypes.c_int]),
    "mdx_set_variant": (ctypes.c_int, [_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_int]),
}


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIBPATH):
                raise RuntimeError(f"{LIBPATH} is not built (run paper_2506_12501_amd/build.py); "
                                   "there is no fallback implementation")
            L = ctypes.CDLL(LIBPATH)
            for name, (res, args) in EXPORTS.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def check(status: int, what: str):
    if status != MDX_OK:
        L = lib()
        raise MdxError(status, f"{what}: {L.mdx_status_string(status).decode()}: {L.mdx_last_error().decode()}")


def _ptr(t) -> int:
    return t.data_ptr() if t is not None else 0


def _i32p(a: np.ndarray):
    return a.ctypes.data_as(_pi32)


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """One mdx_ctx for a device (Boys and solid-harmonic tables resident)."""
    _cache: dict = {}

    def __init__(self, device: int = 0):
        self.device = device
        h = _p()
        check(lib().mdx_create(device, ctypes.byref(h)), "mdx_create")
        self.handle = h

    @classmethod
    def get(cls, device: int = 0) -> "Context":
        if device not in cls._cache:
            cls._cache[device] = Context(device)
        return cls._cache[device]

    def set_variant(self, ncentre, la, lb, lc, ld, cartesian, variant):
        check(lib().mdx_set_variant(self.handle, ncentre, la, lb, lc, ld, int(cartesian), variant),
              "mdx_set_variant")


class DeviceShells:
    """Shell table: numeric arrays on the device, metadata on the host."""

    def __init__(self, basis, device="cuda", center=None):
        import torch
        self.l = np.ascontiguousarray(basis.l, dtype=np.int32)
        self.nprim = np.ascontiguousarray(basis.nprim, dtype=np.int32)
        self.poff = np.ascontiguousarray(basis.poff, dtype=np.int32)
        if center is None:
            center = torch.as_tensor(np.ascontiguousarray(basis.xyz, dtype=np.float64).reshape(-1), device=device)
        self.center = center.reshape(-1).contiguous()
        self.exps = torch.as_tensor(np.ascontiguousarray(basis.exps, dtype=np.float64), device=device)
        self.coefs = torch.as_tensor(np.ascontiguousarray(basis.coefs, dtype=np.float64), device=device)
        self.struct = MdxShells(int(self.l.size), _ptr(self.center), _ptr(self.exps), _ptr(self.coefs),
                                _i32p(self.l), _i32p(self.nprim), _i32p(self.poff))

    def with_center(self, center):
        new = object.__new__(DeviceShells)
        new.__dict__.update(self.__dict__)
        new.center = center.reshape(-1).contiguous()
        new.struct = MdxShells(int(self.l.size), _ptr(new.center), _ptr(self.exps), _ptr(self.coefs),
                               _i32p(self.l), _i32p(self.nprim), _i32p(self.poff))
        return new


def nfunc(l: int, cartesian: bool) -> int:
    return (l + 1) * (l + 2) // 2 if cartesian else 2 * l + 1


def _pairs(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32).reshape(-1, 2))
    return a


def _class_sizes(shells: DeviceShells, ncentre, bra, ket, cartesian):
    la = int(shells.l[bra[0, 0]])
    lb = int(shells.l[bra[0, 1]]) if ncentre == 4 else -1
    lc = int(shells.l[ket[0, 0]])
    ld = int(shells.l[ket[0, 1]]) if ncentre >= 3 else -1
    nab = nfunc(la, cartesian) * (nfunc(lb, cartesian) if lb >= 0 else 1)
    ncd = nfunc(lc, cartesian) * (nfunc(ld, cartesian) if ld >= 0 else 1)
    return nab, ncd


def boys(x, mmax: int, ctx: Context | None = None):
    """F[m, i] = F_m(x[i]) on the device."""
    import torch
    ctx = ctx or Context.get(x.device.index or 0)
    x = x.contiguous().to(torch.float64)
    F = torch.empty((mmax + 1, x.numel()), dtype=torch.float64, device=x.device)
    check(lib().mdx_boys(ctx.handle, x.numel(), _ptr(x), mmax, _ptr(F), _stream(torch)), "mdx_boys")
    return F


def eri(shells: DeviceShells, ncentre: int, bra, ket, cartesian: bool = False, ctx: Context | None = None,
        out=None, paired: bool = False):
    """Dense batch; returns a view of shape [nbra, nab, ncd, nket] over the
    library's [ij,ab,cd,kl] column-major buffer.  paired=True: only the
    quartets q = (bra q, ket q), a view of shape [n, nab, ncd]."""
    import torch
    dev = shells.center.device
    ctx = ctx or Context.get(dev.index or 0)
    bra = _pairs(bra)
    ket = _pairs(ket)
    nbra, nket = bra.shape[0], ket.shape[0]
    nab, ncd = _class_sizes(shells, ncentre, bra, ket, cartesian)
    flags = (MDX_CARTESIAN if cartesian else MDX_SPHERICAL) | (MDX_PAIRED if paired else 0)
    L = lib()
    wsz = L.mdx_eri_workspace_size(ctx.handle, ctypes.byref(shells.struct), ncentre, nbra, _i32p(bra), nket,
                                   _i32p(ket), flags)
    if wsz == 0:
        # planning failed: the batch call reports the planning status
        check(L.mdx_eri_batch(ctx.handle, ctypes.byref(shells.struct), ncentre, nbra, _i32p(bra), nket,
                              _i32p(ket), flags, None, None, 0, _stream(torch)), "mdx_eri_batch")
    ws = torch.empty(wsz // 8 + 32, dtype=torch.float64, device=dev)
    base = _ptr(ws)
    aligned = (base + 255) // 256 * 256
    if out is None:
        out = torch.empty((nbra if paired else nbra * nket) * nab * ncd, dtype=torch.float64, device=dev)
    check(L.mdx_eri_batch(ctx.handle, ctypes.byref(shells.struct), ncentre, nbra, _i32p(bra), nket, _i32p(ket),
                          flags, _ptr(out), ctypes.c_void_p(aligned), wsz, _stream(torch)), "mdx_eri_batch")
    if paired:
        return out.view(ncd, nab, nbra).permute(2, 1, 0)
    return out.view(nket, ncd, nab, nbra).permute(3, 2, 1, 0)


def eri_noalloc(shells: DeviceShells, ncentre: int, bra, ket, out, cartesian: bool = False,
                ctx: Context | None = None, paired: bool = False):
    """mdx_eri_batch_noalloc into the caller's `out` (a device tensor of at
    least nbra*nket*nab*ncd doubles, or nbra*nab*ncd with paired=True); the
    library's static scratch replaces the workspace.  Returns the same view
    as eri()."""
    import torch
    dev = shells.center.device
    ctx = ctx or Context.get(dev.index or 0)
    bra = _pairs(bra)
    ket = _pairs(ket)
    nbra, nket = bra.shape[0], ket.shape[0]
    nab, ncd = _class_sizes(shells, ncentre, bra, ket, cartesian)
    n = (nbra if paired else nbra * nket) * nab * ncd
    if out.dtype != torch.float64 or out.device != dev or not out.is_contiguous() or out.numel() < n:
        raise ValueError(f"out must be a contiguous float64 tensor of >= {n} elements on {dev}")
    flags = (MDX_CARTESIAN if cartesian else MDX_SPHERICAL) | (MDX_PAIRED if paired else 0)
    check(lib().mdx_eri_batch_noalloc(ctx.handle, ctypes.byref(shells.struct), ncentre, nbra, _i32p(bra), nket,
                                      _i32p(ket), flags, _ptr(out), _stream(torch)), "mdx_eri_batch_noalloc")
    if paired:
        return out[:n].view(ncd, nab, nbra).permute(2, 1, 0)
    return out[:n].view(nket, ncd, nab, nbra).permute(3, 2, 1, 0)


def eri_digest(shells: DeviceShells, ncentre: int, bra, ket, Dbra=None, Dket=None, cartesian: bool = False,
               ctx: Context | None = None):
    """Dense batch contracted with pair-blocked densities inside the kernels;
    Dbra [nbra, nab] and Dket [nket, ncd] device tensors (row = pair).
    Returns (Jbra, Jket), same shapes (None where the other side's density
    is None)."""
    import torch
    dev = shells.center.device
    ctx = ctx or Context.get(dev.index or 0)
    bra = _pairs(bra)
    ket = _pairs(ket)
    nbra, nket = bra.shape[0], ket.shape[0]
    if nbra and nket:
        nab, ncd = _class_sizes(shells, ncentre, bra, ket, cartesian)
    else:   # an empty side: the densities carry the function counts
        nab = Dbra.shape[1] if Dbra is not None else 0
        ncd = Dket.shape[1] if Dket is not None else 0
    flags = MDX_CARTESIAN if cartesian else MDX_SPHERICAL
    L = lib()
    sp = ctypes.byref(shells.struct)
    wsz = L.mdx_eri_workspace_size(ctx.handle, sp, ncentre, nbra, _i32p(bra), nket, _i32p(ket), flags)
    if wsz == 0:
        check(L.mdx_eri_digest_batch(ctx.handle, sp, ncentre, nbra, _i32p(bra), nket, _i32p(ket), flags, None,
                                     None, None, None, None, 0, _stream(torch)), "mdx_eri_digest_batch")
    ws = torch.empty(wsz // 8 + 32, dtype=torch.float64, device=dev)
    aligned = (_ptr(ws) + 255) // 256 * 256
    # library layout: D[pair + npair*f], i.e. the transpose of [pair, f]
    Db = Dbra.t().contiguous() if Dbra is not None else None
    Dk = Dket.t().contiguous() if Dket is not None else None
    Jb = torch.zeros(nab, nbra, dtype=torch.float64, device=dev) if Dk is not None else None
    Jk = torch.zeros(ncd, nket, dtype=torch.float64, device=dev) if Db is not None else None
    check(L.mdx_eri_digest_batch(ctx.handle, sp, ncentre, nbra, _i32p(bra), nket, _i32p(ket), flags, _ptr(Db),
                                 _ptr(Dk), _ptr(Jb), _ptr(Jk), ctypes.c_void_p(aligned), wsz, _stream(torch)),
          "mdx_eri_digest_batch")
    return (Jb.t() if Jb is not None else None), (Jk.t() if Jk is not None else None)


def eri_grad(shells: DeviceShells, ncentre: int, bra, ket, adjoint, cartesian: bool = False,
             ctx: Context | None = None):
    """grad[ij, 12, kl] = sum W d(ab|cd)/dX_i; adjoint in the [ij,ab,cd,kl]
    column-major layout (flat tensor or the [nbra,nab,ncd,nket] view)."""
    import torch
    dev = shells.center.device
    ctx = ctx or Context.get(dev.index or 0)
    bra = _pairs(bra)
    ket = _pairs(ket)
    nbra, nket = bra.shape[0], ket.shape[0]
    flags = MDX_CARTESIAN if cartesian else MDX_SPHERICAL
    L = lib()
    wsz = L.mdx_eri_grad_workspace_size(ctx.handle, ctypes.byref(shells.struct), ncentre, nbra, _i32p(bra),
                                        nket, _i32p(ket), flags)
    if wsz == 0:
        check(L.mdx_eri_grad_batch(ctx.handle, ctypes.byref(shells.struct), ncentre, nbra, _i32p(bra), nket,
                                   _i32p(ket), flags, None, None, None, 0, _stream(torch)), "mdx_eri_grad_batch")
    ws = torch.empty(wsz // 8 + 32, dtype=torch.float64, device=dev)
    aligned = (_ptr(ws) + 255) // 256 * 256
    if adjoint.dim() == 4:
        adjoint = adjoint.permute(3, 2, 1, 0)
    W = adjoint.contiguous().reshape(-1)
    grad = torch.empty(nbra * 12 * nket, dtype=torch.float64, device=dev)
    check(L.mdx_eri_grad_batch(ctx.handle, ctypes.byref(shells.struct), ncentre, nbra, _i32p(bra), nket,
                               _i32p(ket), flags, _ptr(W), _ptr(grad), ctypes.c_void_p(aligned), wsz,
                               _stream(torch)), "mdx_eri_grad_batch")
    return grad.view(nket, 12, nbra).permute(2, 1, 0)


def one_body(shells: DeviceShells, pairs, cartesian: bool = False, ctx: Context | None = None,
             overlap: bool = True, kinetic: bool = True):
    """Overlap and kinetic-energy integrals of a batch of shell pairs of one
    class; returns (S, T), each a view of shape [npair, na, nb] over the
    library's [ij, ab] column-major buffer (None for a matrix not asked for)."""
    import torch
    dev = shells.center.device
    ctx = ctx or Context.get(dev.index or 0)
    pairs = _pairs(pairs)
    npair = pairs.shape[0]
    flags = MDX_CARTESIAN if cartesian else MDX_SPHERICAL
    L = lib()
    sp = ctypes.byref(shells.struct)
    wsz = L.mdx_one_body_workspace_size(ctx.handle, sp, npair, _i32p(pairs), flags)
    if wsz == 0:
        check(L.mdx_one_body_batch(ctx.handle, sp, npair, _i32p(pairs), flags, None, None, None, 0,
                                   _stream(torch)), "mdx_one_body_batch")
    if npair:
        la, lb = int(shells.l[pairs[0, 0]]), int(shells.l[pairs[0, 1]])
        na, nb = nfunc(la, cartesian), nfunc(lb, cartesian)
    else:
        na = nb = 0
    ws = torch.empty(wsz // 8 + 32, dtype=torch.float64, device=dev)
    aligned = (_ptr(ws) + 255) // 256 * 256
    S = torch.empty(npair * na * nb, dtype=torch.float64, device=dev) if overlap else None
    T = torch.empty(npair * na * nb, dtype=torch.float64, device=dev) if kinetic else None
    check(L.mdx_one_body_batch(ctx.handle, sp, npair, _i32p(pairs), flags, _ptr(S) if S is not None else None,
                               _ptr(T) if T is not None else None, ctypes.c_void_p(aligned), wsz,
                               _stream(torch)), "mdx_one_body_batch")

    def view(x):
        return None if x is None else x.view(na, nb, npair).permute(2, 0, 1)
    return view(S), view(T)


def nuclear(shells: DeviceShells, pairs, charges, cartesian: bool = False, ctx: Context | None = None):
    """1-particle Coulomb integrals of a batch of shell pairs of one class in
    the field of point charges (a [n, 4] device tensor of x, y, z, q rows);
    returns a view of shape [npair, na, nb] over the library's [ij, ab]
    column-major buffer."""
    import torch
    dev = shells.center.device
    ctx = ctx or Context.get(dev.index or 0)
    pairs = _pairs(pairs)
    npair = pairs.shape[0]
    charges = charges.reshape(-1, 4).contiguous()
    flags = MDX_CARTESIAN if cartesian else MDX_SPHERICAL
    L = lib()
    sp = ctypes.byref(shells.struct)
    wsz = L.mdx_nuclear_workspace_size(ctx.handle, sp, npair, _i32p(pairs), charges.shape[0], flags)
    if wsz == 0:
        check(L.mdx_nuclear_batch(ctx.handle, sp, npair, _i32p(pairs), charges.shape[0], _ptr(charges), flags,
                                  None, None, 0, _stream(torch)), "mdx_nuclear_batch")
    if npair:
        na = nfunc(int(shells.l[pairs[0, 0]]), cartesian)
        nb = nfunc(int(shells.l[pairs[0, 1]]), cartesian)
    else:
        na = nb = 0
    ws = torch.empty(wsz // 8 + 32, dtype=torch.float64, device=dev)
    aligned = (_ptr(ws) + 255) // 256 * 256
    V = torch.empty(npair * na * nb, dtype=torch.float64, device=dev)
    check(L.mdx_nuclear_batch(ctx.handle, sp, npair, _i32p(pairs), charges.shape[0], _ptr(charges), flags,
                              _ptr(V), ctypes.c_void_p(aligned), wsz, _stream(torch)), "mdx_nuclear_batch")
    return V.view(na, nb, npair).permute(2, 0, 1)


def schwarz(shells: DeviceShells, pairs, cartesian: bool = False, ctx: Context | None = None):
    """Q[i] = sqrt(max_ab |(ab|ab)|) of each shell pair (one class), on the device."""
    import torch
    dev = shells.center.device
    ctx = ctx or Context.get(dev.index or 0)
    pairs = _pairs(pairs)
    n = pairs.shape[0]
    flags = MDX_CARTESIAN if cartesian else MDX_SPHERICAL
    L = lib()
    Q = torch.empty(n, dtype=torch.float64, device=dev)
    wsz = L.mdx_schwarz_workspace_size(ctx.handle, ctypes.byref(shells.struct), n, _i32p(pairs), flags)
    if wsz == 0:
        check(L.mdx_schwarz(ctx.handle, ctypes.byref(shells.struct), n, _i32p(pairs), flags, None, None, 0,
                            _stream(torch)), "mdx_schwarz")
    ws = torch.empty(wsz // 8 + 32, dtype=torch.float64, device=dev)
    aligned = (_ptr(ws) + 255) // 256 * 256
    check(L.mdx_schwarz(ctx.handle, ctypes.byref(shells.struct), n, _i32p(pairs), flags, _ptr(Q),
                        ctypes.c_void_p(aligned), wsz, _stream(torch)), "mdx_schwarz")
    return Q


class Batch:
    """One class batch of a plan: pair lists, optional ragged bra prefix
    counts per ket pair, and the offset of its output block."""

    def __init__(self, ncentre, bra, ket, bra_count=None, out_offset=0):
        self.ncentre = ncentre
        self.bra = _pairs(bra)
        self.ket = _pairs(ket)
        self.bra_count = None if bra_count is None else np.ascontiguousarray(bra_count, dtype=np.int32)
        self.out_offset = int(out_offset)


class Plan:
    """mdx_plan over a list of Batch; fused=True -> one captured graph with
    persistent work-queue kernels."""

    def __init__(self, shells: DeviceShells, batches, cartesian=False, fused=False, ctx: Context | None = None,
                 digest=False):
        import torch
        self.ctx = ctx or Context.get(shells.center.device.index or 0)
        self.shells = shells
        self.batches = list(batches)
        n = len(self.batches)
        descs = (MdxBatchDesc * max(n, 1))()
        for i, b in enumerate(self.batches):
            descs[i] = MdxBatchDesc(b.ncentre, b.bra.shape[0], _i32p(b.bra), b.ket.shape[0], _i32p(b.ket),
                                    _i32p(b.bra_count) if b.bra_count is not None else None, b.out_offset)
        flags = (MDX_CARTESIAN if cartesian else 0) | (MDX_FUSED if fused else 0) | (MDX_DIGEST if digest else 0)
        h = _p()
        check(lib().mdx_plan_create(self.ctx.handle, ctypes.byref(shells.struct), n, descs, flags, ctypes.byref(h)),
              "mdx_plan_create")
        self.handle = h
        self.ws_bytes = lib().mdx_plan_workspace_size(h)
        self.out_size = lib().mdx_plan_output_size(h)
        self.ws = torch.empty(self.ws_bytes // 8 + 32, dtype=torch.float64, device=shells.center.device)
        self.wsp = (_ptr(self.ws) + 255) // 256 * 256

    def execute(self, out=None):
        import torch
        if out is None:
            out = torch.empty(max(self.out_size, 1), dtype=torch.float64, device=self.shells.center.device)
        check(lib().mdx_plan_execute(self.handle, ctypes.byref(self.shells.struct), ctypes.c_void_p(_ptr(out)),
                                     ctypes.c_void_p(self.wsp), self.ws_bytes, _stream(torch)), "mdx_plan_execute")
        return out

    def digest(self, blocks):
        """mdx_plan_digest (plan made with digest=True): blocks is one
        (Dbra, Dket, Jbra, Jket) tuple of device tensors (or None) per batch;
        the J tensors are accumulated in place."""
        import torch
        n = len(self.batches)
        arr = (MdxDigestBlock * max(n, 1))()
        for i, blk in enumerate(blocks):
            arr[i] = MdxDigestBlock(*[_ptr(t) for t in blk])
        check(lib().mdx_plan_digest(self.handle, ctypes.byref(self.shells.struct), arr, ctypes.c_void_p(self.wsp),
                                    self.ws_bytes, _stream(torch)), "mdx_plan_digest")

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().mdx_plan_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


class Prepared:
    """A prepared batch (mdx_eri_prepare, mdx_one_body_prepare,
    mdx_nuclear_prepare): planned and its index tables copied to the device
    once; run() enqueues kernels only, so it can be captured into a graph.
    kind: "eri" (args ncentre, bra, ket; paired), "one_body" (args pairs) or
    "nuclear" (args pairs, ncharge).  Output buffers and the workspace are
    allocated here once and reused by every run."""

    def __init__(self, kind, shells: DeviceShells, *args, cartesian: bool = False, paired: bool = False,
                 ctx: Context | None = None):
        import torch
        self.kind = kind
        self.shells = shells
        dev = shells.center.device
        self.ctx = ctx or Context.get(dev.index or 0)
        flags = (MDX_CARTESIAN if cartesian else MDX_SPHERICAL) | (MDX_PAIRED if paired else 0)
        L = lib()
        h = _p()
        sp = ctypes.byref(shells.struct)
        if kind == "eri":
            ncentre, bra, ket = args
            self.bra, self.ket = _pairs(bra), _pairs(ket)
            self.ncentre, self.paired = ncentre, paired
            self.nab, self.ncd = _class_sizes(shells, ncentre, self.bra, self.ket, cartesian)
            st = L.mdx_eri_prepare(self.ctx.handle, sp, ncentre, self.bra.shape[0], _i32p(self.bra),
                                   self.ket.shape[0], _i32p(self.ket), flags, ctypes.byref(h))
        elif kind == "one_body":
            (pairs,) = args
            self.pairs = _pairs(pairs)
            st = L.mdx_one_body_prepare(self.ctx.handle, sp, self.pairs.shape[0], _i32p(self.pairs), flags,
                                        ctypes.byref(h))
        elif kind == "nuclear":
            pairs, ncharge = args
            self.pairs = _pairs(pairs)
            self.ncharge = int(ncharge)
            st = L.mdx_nuclear_prepare(self.ctx.handle, sp, self.pairs.shape[0], _i32p(self.pairs), self.ncharge,
                                       flags, ctypes.byref(h))
        else:
            raise ValueError(f"unknown kind {kind!r}")
        check(st, f"mdx_{kind}_prepare")
        self.handle = h
        self.ws_bytes = L.mdx_batch_workspace_size(h)
        self.out_size = L.mdx_batch_output_size(h)
        self.ws = torch.empty(self.ws_bytes // 8 + 32, dtype=torch.float64, device=dev)
        self.wsp = (_ptr(self.ws) + 255) // 256 * 256
        nout = 2 if kind == "one_body" else 1
        self.out = [torch.empty(max(self.out_size, 1), dtype=torch.float64, device=dev) for _ in range(nout)]

    def run(self, charges=None):
        """Enqueues the batch on the current stream into self.out; returns
        the output tensors (flat, the plain calls' layouts)."""
        import torch
        L = lib()
        sp = ctypes.byref(self.shells.struct)
        ws = ctypes.c_void_p(self.wsp)
        if self.kind == "eri":
            check(L.mdx_eri_run(self.handle, sp, _ptr(self.out[0]), ws, self.ws_bytes, _stream(torch)),
                  "mdx_eri_run")
        elif self.kind == "one_body":
            check(L.mdx_one_body_run(self.handle, sp, _ptr(self.out[0]), _ptr(self.out[1]), ws, self.ws_bytes,
                                     _stream(torch)), "mdx_one_body_run")
        else:
            check(L.mdx_nuclear_run(self.handle, sp, _ptr(charges) if charges is not None else None,
                                    _ptr(self.out[0]), ws, self.ws_bytes, _stream(torch)), "mdx_nuclear_run")
        return self.out

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                lib().mdx_batch_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

