"""Seeded synthetic inputs: Gaussian shells, shell pairs and adjoints.

This module draws random numbers and lays out shell tables.  It holds none of
the integral arithmetic, so both the GPU path and the CPU oracle can be fed
the same bytes from it.

Draw order is fixed and documented: shells are generated one after another;
for each shell its centre (3 uniforms), then its K exponents (log-uniform),
then its K coefficients.  Coefficients are multiplied by the normalisation
constant of an x^l primitive Cartesian Gaussian,
N(zeta, l) = (2 zeta/pi)^{3/4} (4 zeta)^{l/2} / sqrt((2l-1)!!),
so that integrals are O(1); the library itself applies coefficients as given.
Lengths are in bohr; box sizes are given in Angstrom and converted with
1 A = 1/0.529177210903 bohr.

The workloads mirror the paper's benchmark method (random Gaussians that
mimic basis-set values and randomise the Boys arguments, Sec. 4) and the
five configurations this library is measured on.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ANGSTROM = 1.0 / 0.529177210903


def _dfact(n: int) -> float:
    r = 1.0
    while n > 1:
        r *= n
        n -= 2
    return r


def prim_norm(zeta: np.ndarray, l: int) -> np.ndarray:
    """Normalisation of x^l exp(-zeta r^2)."""
    return (2 * zeta / math.pi) ** 0.75 * (4 * zeta) ** (l / 2) / math.sqrt(_dfact(2 * l - 1))


@dataclasses.dataclass
class Basis:
    xyz: np.ndarray      # [nshell, 3] float64, bohr
    l: np.ndarray        # [nshell] int32
    nprim: np.ndarray    # [nshell] int32
    poff: np.ndarray     # [nshell] int32 offset into exps/coefs
    exps: np.ndarray     # [nprim_total] float64
    coefs: np.ndarray    # [nprim_total] float64

    @property
    def nshell(self) -> int:
        return int(self.l.size)

    def moved(self, shell: int, axis: int, h: float) -> "Basis":
        xyz = self.xyz.copy()
        xyz[shell, axis] += h
        return dataclasses.replace(self, xyz=xyz)


class ShellBuilder:
    def __init__(self):
        self.xyz, self.l, self.K, self.exps, self.coefs = [], [], [], [], []

    def add(self, center, l, exps, coefs) -> int:
        self.xyz.append(np.asarray(center, dtype=np.float64))
        self.l.append(int(l))
        self.K.append(len(exps))
        self.exps.extend(float(e) for e in exps)
        self.coefs.extend(float(c) for c in coefs)
        return len(self.l) - 1

    def basis(self) -> Basis:
        K = np.asarray(self.K, dtype=np.int32)
        poff = np.zeros_like(K)
        if K.size:
            poff[1:] = np.cumsum(K)[:-1]
        return Basis(np.asarray(self.xyz, dtype=np.float64).reshape(-1, 3),
                     np.asarray(self.l, dtype=np.int32), K, poff.astype(np.int32),
                     np.asarray(self.exps, dtype=np.float64),
                     np.asarray(self.coefs, dtype=np.float64))


def random_shell(rng, sb: ShellBuilder, l: int, K: int, box_bohr: float, zeta_lo: float,
                 zeta_hi: float, coef_lo: float | None = None, coef_hi: float | None = None,
                 center=None) -> int:
    """One shell: centre, then K log-uniform exponents, then K coefficients.

    coef_lo None means coefficient 1 (before normalisation)."""
    c = rng.uniform(0.0, box_bohr, 3) if center is None else np.asarray(center, dtype=np.float64)
    z = np.exp(rng.uniform(math.log(zeta_lo), math.log(zeta_hi), K))
    if coef_lo is None:
        co = np.ones(K)
    else:
        co = rng.uniform(coef_lo, coef_hi, K)
    return sb.add(c, l, z, co * prim_norm(z, l))


@dataclasses.dataclass
class ClassBatch:
    """One same-class batch: dense outer product of bra x ket pairs."""
    name: str
    ncentre: int
    basis: Basis
    bra: np.ndarray      # [nbra, 2] int32 (second column -1 for a 1-centre side)
    ket: np.ndarray      # [nket, 2] int32

    @property
    def nshellsets(self) -> int:
        return int(self.bra.shape[0] * self.ket.shape[0])


_LCHAR = "spdfghik"


def parse_class(name: str):
    """'(pd|dd)' -> (1, 2, 2, 2); '(i|dd)' -> (6, -1, 2, 2); '(s|p)' -> (0,-1,1,-1)."""
    s = name.strip("()")
    b, k = s.split("|")
    lv = [_LCHAR.index(ch) for ch in b] + [-1] * (2 - len(b))
    lv += [_LCHAR.index(ch) for ch in k] + [-1] * (2 - len(k))
    return tuple(lv)


def make_class_batch(name: str, nbra: int, nket: int, K: int, box_A: float, zeta_lo: float,
                     zeta_hi: float, coef_lo=None, coef_hi=None, seed: int = 0) -> ClassBatch:
    """Random shells for one class: each pair gets fresh shells (own centres).

    Bra shells are drawn first (pair by pair, first shell then second),
    then ket shells."""
    la, lb, lc, ld = parse_class(name)
    ncentre = 4 if lb >= 0 and ld >= 0 else (3 if ld >= 0 else 2)
    rng = np.random.default_rng(seed)
    sb = ShellBuilder()
    box = box_A * ANGSTROM
    bra = np.full((nbra, 2), -1, dtype=np.int32)
    ket = np.full((nket, 2), -1, dtype=np.int32)
    for i in range(nbra):
        bra[i, 0] = random_shell(rng, sb, la, K, box, zeta_lo, zeta_hi, coef_lo, coef_hi)
        if lb >= 0:
            bra[i, 1] = random_shell(rng, sb, lb, K, box, zeta_lo, zeta_hi, coef_lo, coef_hi)
    for i in range(nket):
        ket[i, 0] = random_shell(rng, sb, lc, K, box, zeta_lo, zeta_hi, coef_lo, coef_hi)
        if ld >= 0:
            ket[i, 1] = random_shell(rng, sb, ld, K, box, zeta_lo, zeta_hi, coef_lo, coef_hi)
    return ClassBatch(name, ncentre, sb.basis(), bra, ket)


def one_body_pairs(la: int, lb: int, na: int, nb: int, K: int, seed: int = 0):
    """Shell pairs for the overlap/kinetic batches: na shells of l_a and nb of
    l_b, each with its own centre in a 10 A box, K exponents log-uniform in
    [0.05, 50] and coefficients in [0.1, 1]; all na x nb pairs (a outer,
    b inner).  Returns (basis, pairs [na*nb, 2])."""
    rng = np.random.default_rng(seed)
    sb = ShellBuilder()
    box = 10.0 * ANGSTROM
    A = [random_shell(rng, sb, la, K, box, 0.05, 50.0, 0.1, 1.0) for _ in range(na)]
    B = [random_shell(rng, sb, lb, K, box, 0.05, 50.0, 0.1, 1.0) for _ in range(nb)]
    pairs = np.stack(np.meshgrid(np.asarray(A, np.int32), np.asarray(B, np.int32), indexing="ij"), -1)
    return sb.basis(), np.ascontiguousarray(pairs.reshape(-1, 2))


def point_charges(n: int = 100, box_A: float = 10.0, q_lo: float = 1.0, q_hi: float = 8.0, seed: int = 0):
    """n point charges, positions uniform in a box_A Angstrom cube, charges
    uniform in [q_lo, q_hi]: rows (x, y, z, q) in bohr, the layout the
    1-particle Coulomb entry point takes."""
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(0.0, box_A * ANGSTROM, (n, 3))
    q = rng.uniform(q_lo, q_hi, n)
    return np.ascontiguousarray(np.c_[xyz, q], dtype=np.float64)


# ---------------------------------------------------------------------------
# The five measured configurations
# ---------------------------------------------------------------------------
C1_CLASSES = ["(ss|ss)", "(ps|ss)", "(ps|ps)", "(pp|ss)", "(pp|ps)", "(pp|pp)"]
C2_CLASSES = ["(dd|dd)", "(pd|dd)"]
C4_CLASSES_4C = ["(ff|ff)", "(gg|gg)"]
C4_CLASSES_3C = ["(s|dd)", "(p|dd)", "(d|dd)", "(f|dd)", "(g|dd)", "(h|dd)", "(i|dd)"]
# beyond l = 4 per 4-centre shell (same recipe as the high-L classes above)
HIGH_L_CLASSES_4C = ["(hh|hh)", "(ii|ii)"]


def config1(name: str, npair: int = 16, seed: int = 0) -> ClassBatch:
    """Plain MD s/p primitive quartets: 16 x 16 pairs, 4 A box, zeta in
    [0.1, 100], coefficient 1."""
    return make_class_batch(name, npair, npair, 1, 4.0, 0.1, 100.0, None, None, seed)


def config2(name: str, npair: int = 256, seed: int = 0) -> ClassBatch:
    """Contracted K=3 shells: 256 x 256 pairs, 10 A box, zeta in [0.05, 50],
    coefficients in [0.1, 1]."""
    return make_class_batch(name, npair, npair, 3, 10.0, 0.05, 50.0, 0.1, 1.0, seed)


def config4(name: str, nbra: int | None = None, nket: int | None = None, seed: int = 0) -> ClassBatch:
    """High-L primitive: 4-centre 128 x 128, 3-centre 256 aux x 256 pairs;
    zeta in [0.1, 20], 4 A box."""
    la, lb, lc, ld = parse_class(name)
    if lb >= 0:
        nbra = nbra or 128
        nket = nket or 128
    else:
        nbra = nbra or 256
        nket = nket or 256
    return make_class_batch(name, nbra, nket, 1, 4.0, 0.1, 20.0, None, None, seed)


def adjoint(batch: ClassBatch, nab: int, ncd: int, seed: int = 1) -> np.ndarray:
    """W ~ N(0,1) in the dense output layout [nbra, nab, ncd, nket] (Fortran)."""
    rng = np.random.default_rng(seed)
    n = batch.bra.shape[0] * nab * ncd * batch.ket.shape[0]
    return rng.standard_normal(n)


# ---------------------------------------------------------------------------
# Configuration 3: water-like cluster
# ---------------------------------------------------------------------------
def water_cluster(seed: int = 0, nx: int = 4, ny: int = 4, nz: int = 6, spacing_A: float = 3.0):
    """96 atoms on a simple-cubic lattice (3 A spacing); atom i is heavy iff
    i % 3 == 0.  Heavy: s K=(8,1,1), p K=(3,1), one d K=1.  Light: s K=(3,1),
    one p K=1.  Exponents log-uniform in [0.1, 5000]; coefficients uniform in
    [0.1, 1] (times normalisation).  Returns (basis, atom_of_shell)."""
    rng = np.random.default_rng(seed)
    sb = ShellBuilder()
    atom_of = []
    n = 0
    for ix in range(nx):
        for iy in range(ny):
            for iz in range(nz):
                center = np.array([ix, iy, iz], dtype=np.float64) * spacing_A * ANGSTROM
                heavy = (n % 3 == 0)
                shells = [(0, 8), (0, 1), (0, 1), (1, 3), (1, 1), (2, 1)] if heavy else \
                         [(0, 3), (0, 1), (1, 1)]
                for (l, K) in shells:
                    random_shell(rng, sb, l, K, 0.0, 0.1, 5000.0, 0.1, 1.0, center=center)
                    atom_of.append(n)
                n += 1
    return sb.basis(), np.asarray(atom_of, dtype=np.int32)
