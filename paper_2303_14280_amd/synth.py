"""Seeded synthetic inputs for the sn-K exchange build.

This module produces the *inputs* of the method and nothing else: a molecular
geometry, a contracted Cartesian Gaussian basis (Sec. II.A: atom-centred,
contracted GTOs; Sec. II.B for the primitive form), an atom-centred molecular
quadrature (Sec. II.C: Mura-Knowles radial x Lebedev-Laikov angular grids with
a fuzzy-cell weight partition) and a density matrix P = 2 C_occ C_occ^T built
from random S-orthonormal occupied orbitals.  It holds none of the arithmetic
of the exchange build itself (collocation, 3c-CP integrals, G, K): both the
HIP library and the CPU oracle consume what it returns.

The paper's molecules, basis sets (6-31G(d)) and grids are not reproduced;
seeded water-like clusters of matching shape stand in for them (Table mol,
Table grids).  All lengths are in bohr.

Seeds: ``numpy.random.default_rng([config_id, stream])`` with stream 0 for
the geometry, 1 for the basis and 2 for the orbitals.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

ANGSTROM = 1.0 / 0.529177210903  # bohr per angstrom

Z_O, Z_H = 8, 1

# Per-config recipe: atoms, box, basis flavour, grid (radial x angular) and occupied orbitals.
BASIS_SEED = {"sp": 1, "spd": 2}

CONFIGS: Dict[int, dict] = {
    1: dict(n_triads=2, extra=None, box=None, basis="sp", grid=(50, 110), density="delocalised"),
    2: dict(n_triads=10, extra=None, box=9.0, basis="spd", grid=(75, 302), density="delocalised"),
    3: dict(n_triads=50, extra=None, box=20.0, basis="spd", grid=(75, 302), density="delocalised"),
    4: dict(n_triads=166, extra="OH", box=30.0, basis="spd", grid=(75, 302), density="local"),
    5: dict(n_triads=333, extra="O", box=38.0, basis="spd", grid=(50, 194), density="local"),
}

# Lebedev degree giving a number of angular points.
_LEBEDEV_DEGREE = {6: 3, 14: 5, 26: 7, 38: 9, 50: 11, 86: 15, 110: 17, 146: 19, 170: 21,
                   194: 23, 302: 29, 350: 31, 434: 35, 590: 41, 770: 47, 974: 53, 1202: 59}

# Shell l sequences per element and basis flavour.
_SHELLS = {
    ("sp", Z_O): [0, 0, 0, 1, 1],            # O 3s2p
    ("sp", Z_H): [0, 0, 1],                  # H 2s1p
    ("spd", Z_O): [0, 0, 0, 0, 1, 1, 1, 2],  # O 4s3p1d
    ("spd", Z_H): [0, 0, 1],                 # H 2s1p
}

NPRIM = 3
EXP_RANGE = (0.1, 5000.0)
COEF_RANGE = (0.1, 1.0)


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def cart_components(l: int) -> List[Tuple[int, int, int]]:
    """Cartesian exponents of a shell in lexicographic order (x,y,z; xx,xy,xz,yy,yz,zz)."""
    out = []
    for lx in range(l, -1, -1):
        for ly in range(l - lx, -1, -1):
            out.append((lx, ly, l - lx - ly))
    return out


def _dfact(n: int) -> float:
    """(n)!! with (-1)!! = 0!! = 1."""
    r = 1.0
    while n > 1:
        r *= n
        n -= 2
    return r


@dataclasses.dataclass
class System:
    """One sn-K problem: basis (SoA), grid, weights and density."""
    config_id: int
    atom_Z: np.ndarray
    atom_xyz: np.ndarray          # (n_atom, 3) bohr
    molecule_of_atom: np.ndarray  # (n_atom,)
    shell_center: np.ndarray      # (nshell, 3)
    shell_l: np.ndarray           # int32
    shell_nprim: np.ndarray       # int32
    shell_prim_off: np.ndarray    # int32
    shell_atom: np.ndarray        # int32
    exps: np.ndarray              # float64
    coefs: np.ndarray             # float64, normalised for the axis-aligned component
    grid_xyz: np.ndarray          # (npts, 3)
    grid_w: np.ndarray            # (npts,)
    grid_atom: np.ndarray         # int32 (npts,)
    P: np.ndarray                 # (nbf, nbf)
    n_occ: int
    density: str

    @property
    def nshell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def nbf(self) -> int:
        return int(sum(ncart(int(l)) for l in self.shell_l))

    @property
    def npts(self) -> int:
        return int(self.grid_w.shape[0])

    def shell_offsets(self) -> np.ndarray:
        off = np.zeros(self.nshell + 1, dtype=np.int64)
        off[1:] = np.cumsum([ncart(int(l)) for l in self.shell_l])
        return off

    def with_grid(self, xyz: np.ndarray, w: np.ndarray, atom: Optional[np.ndarray] = None) -> "System":
        atom = np.zeros(len(w), np.int32) if atom is None else np.asarray(atom, np.int32)
        return dataclasses.replace(self, grid_xyz=np.ascontiguousarray(xyz, np.float64),
                                   grid_w=np.ascontiguousarray(w, np.float64), grid_atom=atom)

    def with_density(self, P: np.ndarray) -> "System":
        return dataclasses.replace(self, P=np.ascontiguousarray(P, np.float64))

    def subset_points(self, idx: np.ndarray) -> "System":
        idx = np.asarray(idx)
        return self.with_grid(self.grid_xyz[idx], self.grid_w[idx], self.grid_atom[idx])


# ----------------------------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------------------------

def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _water(rng: np.random.Generator, o_pos: np.ndarray) -> np.ndarray:
    r1 = rng.uniform(0.94, 0.98) * ANGSTROM
    r2 = rng.uniform(0.94, 0.98) * ANGSTROM
    th = math.radians(rng.uniform(101.5, 107.5))
    loc = np.array([[0.0, 0.0, 0.0], [r1, 0.0, 0.0], [r2 * math.cos(th), r2 * math.sin(th), 0.0]])
    return o_pos + loc @ _random_rotation(rng).T


def _unit(rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def make_geometry(config_id: int, variant: int = 0) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Atoms (Z, xyz in bohr, molecule index) of a seeded water-like cluster.

    ``variant`` > 0 draws another cluster of the same recipe (other seed)."""
    cfg = CONFIGS[config_id]
    rng = np.random.default_rng([config_id, 0] + ([variant] if variant else []))
    n_tri = cfg["n_triads"]
    if cfg["box"] is None:
        # two triads with O-O = 3.0 A along a random direction
        o = [np.zeros(3), 3.0 * ANGSTROM * _unit(rng)]
    else:
        box = cfg["box"] * ANGSTROM
        dmin = 2.5 * ANGSTROM
        n_o = n_tri + (1 if cfg["extra"] else 0)
        o = []
        tries = 0
        while len(o) < n_o:
            tries += 1
            if tries > 10_000_000:
                raise RuntimeError("could not place oxygens")
            p = rng.uniform(0.0, box, size=3)
            if all(np.linalg.norm(p - q) >= dmin for q in o):
                o.append(p)
    Z, xyz, mol = [], [], []
    for t in range(n_tri):
        w = _water(rng, o[t])
        Z += [Z_O, Z_H, Z_H]
        xyz += list(w)
        mol += [t, t, t]
    if cfg["extra"] == "OH":
        Z += [Z_O, Z_H]
        xyz += [o[n_tri], o[n_tri] + 0.96 * ANGSTROM * _unit(rng)]
        mol += [n_tri, n_tri]
    elif cfg["extra"] == "O":
        Z += [Z_O]
        xyz += [o[n_tri]]
        mol += [n_tri]
    return np.array(Z, np.int32), np.array(xyz, np.float64), np.array(mol, np.int32)


# ----------------------------------------------------------------------------------------------
# basis
# ----------------------------------------------------------------------------------------------

def _normalised_coefs(l: int, exps: np.ndarray, raw: np.ndarray) -> np.ndarray:
    """Fold primitive normalisation of the axis-aligned component x^l e^{-a r^2} and the
    contraction normalisation into the coefficients (unit self-overlap of that component)."""
    prim_n = (2 * exps / math.pi) ** 0.75 * (4 * exps) ** (l / 2.0) / math.sqrt(_dfact(2 * l - 1))
    c = raw * prim_n
    a = exps[:, None]
    b = exps[None, :]
    # overlap of normalised primitives of the axis-aligned component
    s = (2.0 * np.sqrt(a * b) / (a + b)) ** (l + 1.5)
    norm = float(raw @ s @ raw)
    return c / math.sqrt(norm)


def make_element_basis(flavour: str, rng: np.random.Generator) -> Dict[int, List[Tuple[int, np.ndarray, np.ndarray]]]:
    """Random contracted basis per element: 3 primitives per shell, exponents iid
    log-uniform on [0.1, 5000] (sorted descending), coefficients iid U(0.1, 1)."""
    out = {}
    lo, hi = math.log(EXP_RANGE[0]), math.log(EXP_RANGE[1])
    for Z in (Z_O, Z_H):
        shells = []
        for l in _SHELLS[(flavour, Z)]:
            e = np.sort(np.exp(rng.uniform(lo, hi, size=NPRIM)))[::-1].copy()
            c = rng.uniform(*COEF_RANGE, size=NPRIM)
            shells.append((l, e, _normalised_coefs(l, e, c)))
        out[Z] = shells
    return out


def assemble_basis(atom_Z, atom_xyz, per_element):
    cen, ls, npr, off, sat, ex, co = [], [], [], [], [], [], []
    k = 0
    for a, (Z, R) in enumerate(zip(atom_Z, atom_xyz)):
        for (l, e, c) in per_element[int(Z)]:
            cen.append(R)
            ls.append(l)
            npr.append(len(e))
            off.append(k)
            sat.append(a)
            ex.append(e)
            co.append(c)
            k += len(e)
    return (np.array(cen, np.float64).reshape(-1, 3), np.array(ls, np.int32), np.array(npr, np.int32),
            np.array(off, np.int32), np.array(sat, np.int32),
            np.concatenate(ex).astype(np.float64), np.concatenate(co).astype(np.float64))


# ----------------------------------------------------------------------------------------------
# molecular grid
# ----------------------------------------------------------------------------------------------

def mura_knowles(n_rad: int, alpha: float = 5.0) -> Tuple[np.ndarray, np.ndarray]:
    """Mura-Knowles radial rule r = -alpha ln(1 - x^3), x = k/(n+1); weights include r^2."""
    k = np.arange(1, n_rad + 1, dtype=np.float64)
    x = k / (n_rad + 1)
    r = -alpha * np.log1p(-x ** 3)
    w = 3.0 * alpha * x ** 2 * r ** 2 / ((1.0 - x ** 3) * (n_rad + 1))
    return r, w


def lebedev(n_ang: int) -> Tuple[np.ndarray, np.ndarray]:
    from scipy.integrate import lebedev_rule
    x, w = lebedev_rule(_LEBEDEV_DEGREE[n_ang])
    return np.ascontiguousarray(x.T), np.asarray(w, np.float64)


def _becke_s(mu: np.ndarray) -> np.ndarray:
    f = mu
    for _ in range(3):
        f = f * (1.5 - 0.5 * (f * f))
    return 0.5 - 0.5 * f


def becke_partition(points: np.ndarray, parent: int, atoms: np.ndarray, cand: np.ndarray) -> np.ndarray:
    """Becke fuzzy-cell weight (3-fold iterated cell function, no size adjustment) of the
    parent atom at the given points, over the candidate atom set ``cand`` (contains parent).
    Uses s(-mu) = 1 - s(mu), so each unordered atom pair is evaluated once."""
    A = atoms[cand]
    k = len(cand)
    d = [np.linalg.norm(points - A[b], axis=1) for b in range(k)]
    Pc = [np.ones(len(points)) for _ in range(k)]
    for b in range(k):
        for c in range(b + 1, k):
            s = _becke_s((d[b] - d[c]) * (1.0 / float(np.linalg.norm(A[b] - A[c]))))
            Pc[b] *= s
            Pc[c] *= 1.0 - s
    ip = int(np.nonzero(cand == parent)[0][0])
    return Pc[ip] / np.sum(Pc, axis=0)


_SSF_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grid_ssf.c")
_SSF_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgridssf.so")
_ssf = None


def build_ssf(force: bool = False) -> str:
    """Compile the Stratmann-weight helper (``grid_ssf.c``) with gcc."""
    if force or not os.path.exists(_SSF_LIB) or os.path.getmtime(_SSF_LIB) < os.path.getmtime(_SSF_SRC):
        tmp = _SSF_LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O3", "-fno-math-errno", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", tmp, _SSF_SRC, "-lm"],
                       check=True)
        os.replace(tmp, _SSF_LIB)
    return _SSF_LIB


def ssf_partition(points: np.ndarray, parent: np.ndarray, atoms: np.ndarray) -> np.ndarray:
    """Stratmann-Scuseria-Frisch partition factor of each point's parent atom over all atoms
    (a = 0.64), evaluated exactly: the scheme's cell function is exactly 0 or 1 outside
    |mu| < a, which bounds the atoms that can contribute (see grid_ssf.c)."""
    global _ssf
    if _ssf is None:
        L = ctypes.CDLL(build_ssf())
        L.ssf_weights.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p]
        L.ssf_weights.restype = ctypes.c_int
        _ssf = L
    A = np.ascontiguousarray(atoms, np.float64)
    X = np.ascontiguousarray(points, np.float64)
    par = np.ascontiguousarray(parent, np.int32)
    out = np.empty(len(X), np.float64)
    rc = _ssf.ssf_weights(len(A), A.ctypes.data, len(X), X.ctypes.data, par.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise MemoryError("ssf_weights: out of memory")
    return out


def make_grid(atom_xyz: np.ndarray, n_rad: int, n_ang: int, exact_below: int = 64
              ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Atom-centred grid: Mura-Knowles x Lebedev per atom with fuzzy-cell partition weights.

    Up to ``exact_below`` atoms: Becke's partition (3-fold iterated cell function) over all
    atoms.  Above: the Stratmann-Scuseria-Frisch partition (the paper's choice, Sec. II.C)
    over all atoms, evaluated exactly with its own cut-offs, so the cell weights of every
    point add up to one."""
    r, wr = mura_knowles(n_rad)
    u, wa = lebedev(n_ang)
    loc = (r[:, None, None] * u[None, :, :]).reshape(-1, 3)
    wloc = (wr[:, None] * wa[None, :]).reshape(-1)
    n_atom = len(atom_xyz)
    xyz = np.concatenate([atom_xyz[a] + loc for a in range(n_atom)]) if n_atom else np.zeros((0, 3))
    at = np.repeat(np.arange(n_atom, dtype=np.int32), len(loc))
    if n_atom <= 1:
        wb = np.ones(len(xyz))
    elif n_atom <= exact_below:
        wb = np.concatenate([becke_partition(atom_xyz[a] + loc, a, atom_xyz, np.arange(n_atom))
                             for a in range(n_atom)])
    else:
        wb = ssf_partition(xyz, at, atom_xyz)
    w = np.tile(wloc, n_atom) * wb
    return xyz, w, at


# ----------------------------------------------------------------------------------------------
# overlap (for S-orthonormal orbitals) and density
# ----------------------------------------------------------------------------------------------

def _overlap_1d(lmax_a: int, lmax_b: int, PA: np.ndarray, PB: np.ndarray, oo2p: np.ndarray, s00: np.ndarray):
    """Obara-Saika 1-D overlap table s[i][j] (arrays over primitive pairs)."""
    s = [[None] * (lmax_b + 1) for _ in range(lmax_a + 1)]
    s[0][0] = s00
    for i in range(lmax_a + 1):
        for j in range(lmax_b + 1):
            if i == 0 and j == 0:
                continue
            if i > 0:
                v = PA * s[i - 1][j]
                if i > 1:
                    v = v + (i - 1) * oo2p * s[i - 2][j]
                if j > 0:
                    v = v + j * oo2p * s[i - 1][j - 1]
            else:
                v = PB * s[i][j - 1]
                if j > 1:
                    v = v + (j - 1) * oo2p * s[i][j - 2]
            s[i][j] = v
    return s


def overlap_matrix(sys: System, shells: Optional[np.ndarray] = None) -> np.ndarray:
    """Overlap S over the functions of ``shells`` (all shells by default)."""
    if shells is None:
        shells = np.arange(sys.nshell)
    shells = np.asarray(shells)
    offs = [0]
    for s in shells:
        offs.append(offs[-1] + ncart(int(sys.shell_l[s])))
    n = offs[-1]
    S = np.zeros((n, n))
    comps = {l: cart_components(l) for l in range(3)}
    cnorm = {l: [math.sqrt(_dfact(2 * l - 1) / (_dfact(2 * a - 1) * _dfact(2 * b - 1) * _dfact(2 * c - 1)))
                 for (a, b, c) in comps[l]] for l in range(3)}
    for ii, sa in enumerate(shells):
        la = int(sys.shell_l[sa])
        A = sys.shell_center[sa]
        pa = slice(sys.shell_prim_off[sa], sys.shell_prim_off[sa] + sys.shell_nprim[sa])
        ea, ca = sys.exps[pa], sys.coefs[pa]
        for jj in range(ii + 1):
            sb = shells[jj]
            lb = int(sys.shell_l[sb])
            B = sys.shell_center[sb]
            pb = slice(sys.shell_prim_off[sb], sys.shell_prim_off[sb] + sys.shell_nprim[sb])
            eb, cb = sys.exps[pb], sys.coefs[pb]
            a = ea[:, None]
            b = eb[None, :]
            p = a + b
            P = (a[..., None] * A + b[..., None] * B) / p[..., None]
            mu = a * b / p
            oo2p = 0.5 / p
            cc = ca[:, None] * cb[None, :]
            tabs = []
            for q in range(3):
                s00 = np.sqrt(math.pi / p) * np.exp(-mu * (A[q] - B[q]) ** 2)
                tabs.append(_overlap_1d(la, lb, P[..., q] - A[q], P[..., q] - B[q], oo2p, s00))
            blk = np.zeros((ncart(la), ncart(lb)))
            for ia, (ax, ay, az) in enumerate(comps[la]):
                for ib, (bx, by, bz) in enumerate(comps[lb]):
                    v = tabs[0][ax][bx] * tabs[1][ay][by] * tabs[2][az][bz]
                    blk[ia, ib] = float((cc * v).sum()) * cnorm[la][ia] * cnorm[lb][ib]
            S[offs[ii]:offs[ii + 1], offs[jj]:offs[jj + 1]] = blk
            S[offs[jj]:offs[jj + 1], offs[ii]:offs[ii + 1]] = blk.T
    return S


def _orthonormal_orbitals(S: np.ndarray, n_occ: int, rng: np.random.Generator) -> np.ndarray:
    """C with C^T S C = I: seeded Gaussian coefficients C0, then C = C0 L^{-T} with
    L L^T = C0^T S C0 (Cholesky of a small, well-conditioned matrix).  Unlike an
    eigendecomposition of S, this is a smooth function of the inputs, so the same
    seed gives the same density on every machine to rounding."""
    nb = S.shape[0]
    if n_occ > nb:
        raise ValueError("more occupied orbitals than basis functions")
    C0 = rng.normal(size=(nb, n_occ))
    M = C0.T @ S @ C0
    L = np.linalg.cholesky(0.5 * (M + M.T))
    return np.linalg.solve(L, C0.T).T


def make_density(sys_wo_P: System, n_occ: int, kind: str, seed: Sequence[int]) -> np.ndarray:
    rng = np.random.default_rng(list(seed))
    nb = sys_wo_P.nbf
    if kind == "delocalised":
        S = overlap_matrix(sys_wo_P)
        C = _orthonormal_orbitals(S, n_occ, rng)
        Q = C @ C.T
        return Q + Q.T          # 2 C C^T, exactly symmetric
    if kind != "local":
        raise ValueError(kind)
    # molecule-local: ceil(electrons/2) orbitals per molecule on its own functions
    P = np.zeros((nb, nb))
    offs = sys_wo_P.shell_offsets()
    mol_of_shell = sys_wo_P.molecule_of_atom[sys_wo_P.shell_atom]
    total = 0
    for m in np.unique(mol_of_shell):
        shells = np.nonzero(mol_of_shell == m)[0]
        idx = np.concatenate([np.arange(offs[s], offs[s + 1]) for s in shells])
        atoms = np.unique(sys_wo_P.shell_atom[shells])
        n_el = int(sum(sys_wo_P.atom_Z[a] for a in atoms))
        k = (n_el + 1) // 2
        S = overlap_matrix(sys_wo_P, shells)
        C = _orthonormal_orbitals(S, k, rng)
        Q = C @ C.T
        P[np.ix_(idx, idx)] += Q + Q.T
        total += k
    if total != n_occ:
        raise AssertionError((total, n_occ))
    return P


# ----------------------------------------------------------------------------------------------
# public entry points
# ----------------------------------------------------------------------------------------------

def n_occupied(atom_Z: np.ndarray) -> int:
    return (int(np.sum(atom_Z)) + 1) // 2


def make_system(config_id: int, density: Optional[str] = None, grid: Optional[Tuple[int, int]] = None,
                with_density: bool = True, variant: int = 0) -> System:
    """Seeded system for config 1..5 (see ``CONFIGS``).

    ``variant`` > 0 gives another geometry and density of the same recipe; the element
    basis sets stay those of the config (as a fixed basis-set library would)."""
    cfg = CONFIGS[config_id]
    Z, xyz, mol = make_geometry(config_id, variant)
    # one element basis library per shell set: every "spd" config shares the one drawn for config 2
    per_el = make_element_basis(cfg["basis"], np.random.default_rng([BASIS_SEED[cfg["basis"]], 1]))
    cen, ls, npr, off, sat, ex, co = assemble_basis(Z, xyz, per_el)
    n_rad, n_ang = grid if grid is not None else cfg["grid"]
    gx, gw, ga = make_grid(xyz, n_rad, n_ang)
    kind = density or cfg["density"]
    sys = System(config_id, Z, xyz, mol, cen, ls, npr, off, sat, ex, co, gx, gw, ga,
                 np.zeros((0, 0)), n_occupied(Z), kind)
    if with_density:
        sys = sys.with_density(make_density(sys, sys.n_occ, kind, [config_id, 2] + ([variant] if variant else [])))
    return sys


def make_custom(atom_Z, atom_xyz, shells_per_atom, grid: Optional[Tuple[int, int]] = (30, 110),
                n_occ: Optional[int] = None, seed: int = 0, molecule_of_atom=None) -> System:
    """A hand-specified system: ``shells_per_atom[a]`` is a list of (l, exps, raw_coefs)."""
    atom_Z = np.asarray(atom_Z, np.int32)
    atom_xyz = np.asarray(atom_xyz, np.float64).reshape(-1, 3)
    cen, ls, npr, off, sat, ex, co = [], [], [], [], [], [], []
    k = 0
    for a, shells in enumerate(shells_per_atom):
        for (l, e, c) in shells:
            e = np.asarray(e, np.float64)
            c = _normalised_coefs(l, e, np.asarray(c, np.float64))
            cen.append(atom_xyz[a]); ls.append(l); npr.append(len(e)); off.append(k); sat.append(a)
            ex.append(e); co.append(c); k += len(e)
    mol = np.zeros(len(atom_Z), np.int32) if molecule_of_atom is None else np.asarray(molecule_of_atom, np.int32)
    if grid is not None:
        gx, gw, ga = make_grid(atom_xyz, *grid)
    else:
        gx, gw, ga = np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.int32)
    sys = System(0, atom_Z, atom_xyz, mol, np.array(cen).reshape(-1, 3), np.array(ls, np.int32),
                 np.array(npr, np.int32), np.array(off, np.int32), np.array(sat, np.int32),
                 np.concatenate(ex), np.concatenate(co), gx, gw, ga, np.zeros((0, 0)), 0, "delocalised")
    n = n_occ if n_occ is not None else max(1, min(n_occupied(atom_Z), sys.nbf))
    sys = dataclasses.replace(sys, n_occ=n)
    return sys.with_density(make_density(sys, n, "delocalised", [1000 + seed, 2]))


def random_symmetric(n: int, seed: int) -> np.ndarray:
    """A seeded symmetric matrix (for linearity tests)."""
    rng = np.random.default_rng([9000 + seed])
    X = rng.normal(size=(n, n))
    return 0.5 * (X + X.T)


# ----------------------------------------------------------------------------------------------
# auxiliary (density-fitting) basis
# ----------------------------------------------------------------------------------------------

# one-primitive auxiliary shells per element: even-tempered exponents (l, first, ratio, count)
# spanning the products of the orbital exponents (0.1 .. 5000), jittered per seed
_AUX_SETS = {
    Z_O: [(0, 0.2, 3.0, 10), (1, 0.3, 3.5, 5), (2, 0.4, 4.0, 3)],
    Z_H: [(0, 0.2, 3.5, 8), (1, 0.3, 4.0, 3)],
}


@dataclasses.dataclass
class AuxBasis:
    """Auxiliary (density-fitting) basis in the same SoA layout as the orbital basis."""
    shell_center: np.ndarray
    shell_l: np.ndarray
    shell_nprim: np.ndarray
    shell_prim_off: np.ndarray
    shell_atom: np.ndarray
    exps: np.ndarray
    coefs: np.ndarray

    @property
    def nshell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def nfunc(self) -> int:
        return int(sum(ncart(int(l)) for l in self.shell_l))


def make_aux_basis(s: "System", seed: int = 0) -> AuxBasis:
    """A seeded even-tempered auxiliary basis on the atoms of `s`: one-primitive s, p, d shells
    per element (O: 10s5p3d, H: 8s3p), exponents first * ratio^k, each scaled by a factor drawn
    log-uniformly from [0.85, 1.15] per element and seed, normalised like the orbital shells."""
    rng = np.random.default_rng([7000 + seed])
    per_element = {}
    for Z in (Z_O, Z_H):
        shells = []
        for (l, first, ratio, count) in _AUX_SETS[Z]:
            for k in range(count):
                e = np.array([first * ratio ** k * math.exp(rng.uniform(math.log(0.85), math.log(1.15)))])
                shells.append((l, e, _normalised_coefs(l, e, np.ones(1))))
        per_element[Z] = shells
    cen, ls, npr, off, sat, ex, co = assemble_basis(s.atom_Z, s.atom_xyz, per_element)
    return AuxBasis(cen, ls, npr, off, sat, ex, co)
