"""Molecular grids of the large clusters (more than 64 atoms): the Stratmann-Scuseria-Frisch
partition (Sec. II.C) evaluated exactly over all atoms.

Pins: the cell weights of every point add up to one; the C evaluation equals a brute-force
product over every atom pair; normalised Gaussians at atoms across the cluster integrate to
one; the electron density integrates to 2 N_occ."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2303_14280_amd import synth

A_SSF = 0.64


def _ssf_brute(r, atoms):
    """Every atom's cell weight P_B(r) / sum_C P_C(r) from the full double product."""
    d = np.linalg.norm(r - atoms, axis=1)
    R = np.linalg.norm(atoms[:, None] - atoms[None], axis=2)
    np.fill_diagonal(R, 1.0)
    x = np.clip((d[:, None] - d[None, :]) / R / A_SSF, -1.0, 1.0)
    s = 0.5 * (1.0 - (35 * x - 35 * x ** 3 + 21 * x ** 5 - 5 * x ** 7) / 16.0)
    np.fill_diagonal(s, 1.0)
    P = np.prod(s, axis=1)
    return P / P.sum()


@pytest.fixture(scope="module")
def cluster3():
    Z, xyz, mol = synth.make_geometry(3)
    return Z, xyz, mol


def test_ssf_matches_brute_force_and_sums_to_one(cluster3):
    _, atoms, _ = cluster3
    rng = np.random.default_rng(11)
    lo, hi = atoms.min(0) - 6.0, atoms.max(0) + 6.0
    pts = rng.uniform(lo, hi, size=(60, 3))
    # points next to atoms and in the bonds too
    pts = np.concatenate([pts, atoms[rng.integers(0, len(atoms), 60)] + rng.normal(scale=0.8, size=(60, 3))])
    for r in pts:
        ref = _ssf_brute(r, atoms)
        got = np.array([synth.ssf_partition(r[None], np.array([a], np.int32), atoms)[0]
                        for a in range(len(atoms))])
        assert np.all(got >= 0) and np.all(got <= 1)
        assert np.max(np.abs(got - ref)) < 1e-14
        assert abs(got.sum() - 1.0) < 1e-13


def test_large_grid_integrates_gaussians_and_density(cluster3):
    Z, xyz, mol = cluster3
    gx, gw, ga = synth.make_grid(xyz, 50, 194)
    assert np.all(gw >= 0)
    for a in (0, 37, len(xyz) // 2, len(xyz) - 1):
        for al in (0.2, 1.0, 5.0):
            f = (2 * al / np.pi) ** 1.5 * np.exp(-2 * al * np.sum((gx - xyz[a]) ** 2, axis=1))
            assert abs(np.dot(gw, f) - 1.0) < 2e-5, (a, al)
    # electron count of the molecule-local density on the same grid, molecule by molecule
    s = synth.make_system(3, density="local", with_density=False)
    s = s.with_grid(gx, gw, ga)
    s = s.with_density(synth.make_density(s, s.n_occ, "local", [3, 2]))
    offs = s.shell_offsets()
    mol_of_shell = s.molecule_of_atom[s.shell_atom]
    for m in np.unique(mol_of_shell)[:4]:
        shells = np.nonzero(mol_of_shell == m)[0]
        idx = np.concatenate([np.arange(offs[k], offs[k + 1]) for k in shells])
        atoms_m = np.unique(s.shell_atom[shells])
        sub = _shell_subset(s, shells)
        # the molecule's functions are below 1e-12 beyond 14 bohr of its atoms
        near = np.min(np.linalg.norm(gx[:, None] - s.atom_xyz[atoms_m][None], axis=2), axis=1) < 14.0
        Phi = O.collocate(sub, gx[near])
        rho = np.einsum("mi,mn,ni->i", Phi, s.P[np.ix_(idx, idx)], Phi)
        nel_m = float(np.dot(gw[near], rho))
        n_el = int(sum(s.atom_Z[a] for a in atoms_m))
        assert abs(nel_m - 2 * ((n_el + 1) // 2)) < 1e-4, (m, nel_m)


def _shell_subset(s, shells):
    """The system restricted to the given shells (primitive arrays re-based)."""
    ex, co, off = [], [], []
    k = 0
    for sh in shells:
        o, n = int(s.shell_prim_off[sh]), int(s.shell_nprim[sh])
        ex.append(s.exps[o:o + n])
        co.append(s.coefs[o:o + n])
        off.append(k)
        k += n
    import dataclasses
    return dataclasses.replace(s, shell_center=s.shell_center[shells], shell_l=s.shell_l[shells],
                               shell_nprim=s.shell_nprim[shells], shell_prim_off=np.array(off, np.int32),
                               shell_atom=s.shell_atom[shells], exps=np.concatenate(ex), coefs=np.concatenate(co))
