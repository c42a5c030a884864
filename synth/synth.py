"""Python side of the seeded input generators (ctypes over synth.c).

Everything here produces plain numpy arrays.  Nothing here docks anything.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")

MASTER_SEED = 2209050690


def build(force: bool = True) -> str:
    """Compile libsynth.so in place (gcc, OpenMP for the grid sums)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, u64, f64 = ctypes.c_int, ctypes.c_uint64, ctypes.c_double
        lib.synth_pocket.argtypes = [u64, i32, i32, f64, i32, f64, f64, f64, f64, f64, P, P]
        lib.synth_sizes_uniform.argtypes = [u64, i32, i32, i32, i32, i32, P, P]
        lib.synth_sizes_lognormal.argtypes = [u64, i32, f64, f64, i32, i32, f64, i32, P, P]
        lib.synth_library.argtypes = [u64, i32, P, P, i32, f64, i32, P, P, P, P, P, P, P, P, P]
        lib.synth_start_quats.argtypes = [u64, i32, P]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


@dataclass
class Pocket:
    """Per-atom-type score grids, values[t, z, y, x] (float32), point (i,j,k) at
    origin + spacing*(i,j,k)."""
    values: np.ndarray
    spacing: float
    origin: tuple
    gaussians: np.ndarray | None = None

    @property
    def ntypes(self):
        return self.values.shape[0]

    @property
    def shape_xyz(self):
        t, nz, ny, nx = self.values.shape
        return nx, ny, nz


@dataclass
class Library:
    """CSR ligand library (host arrays)."""
    atom_off: np.ndarray          # int32 [L+1]
    xyz: np.ndarray               # float32 [A, 3], ligand frame, Angstrom
    type: np.ndarray              # uint8 [A]
    bond_off: np.ndarray          # int32 [L+1]
    bonds: np.ndarray             # int32 [Nb, 2] local atom indices
    rot_off: np.ndarray           # int32 [L+1]
    rot_bond: np.ndarray          # int32 [Nr, 2] (fixed atom a, moving atom b), sweep order
    rot_mask: np.ndarray          # uint64 [Nr, mask_words], bit i = atom i moves
    mask_words: int
    n_rot_requested: np.ndarray = field(default=None)

    @property
    def n_ligands(self):
        return len(self.atom_off) - 1

    def n_atoms(self, l=None):
        d = np.diff(self.atom_off)
        return d if l is None else int(d[l])

    def n_rot(self, l=None):
        d = np.diff(self.rot_off)
        return d if l is None else int(d[l])

    def ligand(self, l):
        """Views of ligand l: (xyz [n,3], type [n], bonds [nb,2], rot_bond [B,2], rot_mask [B,W])."""
        a0, a1 = self.atom_off[l], self.atom_off[l + 1]
        b0, b1 = self.bond_off[l], self.bond_off[l + 1]
        r0, r1 = self.rot_off[l], self.rot_off[l + 1]
        return (self.xyz[a0:a1], self.type[a0:a1], self.bonds[b0:b1], self.rot_bond[r0:r1],
                self.rot_mask[r0:r1])

    def subset(self, idx):
        """New library holding ligands idx (in that order)."""
        idx = list(int(i) for i in idx)
        xs, ts, bs, rb, rm = [], [], [], [], []
        ao, bo, ro = [0], [0], [0]
        for l in idx:
            x, t, b, r, m = self.ligand(l)
            xs.append(x); ts.append(t); bs.append(b); rb.append(r); rm.append(m)
            ao.append(ao[-1] + len(x)); bo.append(bo[-1] + len(b)); ro.append(ro[-1] + len(r))
        W = self.mask_words
        return Library(
            atom_off=np.array(ao, np.int32),
            xyz=np.ascontiguousarray(np.concatenate(xs) if xs else np.zeros((0, 3), np.float32)),
            type=np.ascontiguousarray(np.concatenate(ts) if ts else np.zeros(0, np.uint8)),
            bond_off=np.array(bo, np.int32),
            bonds=np.ascontiguousarray(np.concatenate(bs) if bs else np.zeros((0, 2), np.int32)),
            rot_off=np.array(ro, np.int32),
            rot_bond=np.ascontiguousarray(np.concatenate(rb) if rb else np.zeros((0, 2), np.int32)),
            rot_mask=np.ascontiguousarray(np.concatenate(rm) if rm else np.zeros((0, W), np.uint64)),
            mask_words=W)


def pocket_gaussians(seed: int, ntypes: int, n: int, spacing: float, ngauss: int,
                     centre_half: float, sigma=(1.0, 2.0), amp=(-1.0, 1.0)) -> Pocket:
    vals = np.zeros((ntypes, n, n, n), np.float32)
    g = np.zeros((ntypes, ngauss, 5), np.float64)
    rc = _L().synth_pocket(seed, ntypes, n, spacing, ngauss, centre_half, sigma[0], sigma[1],
                           amp[0], amp[1], _p(vals), _p(g))
    if rc:
        raise ValueError(f"synth_pocket failed ({rc})")
    o = -spacing * (n - 1) / 2.0
    return Pocket(values=vals, spacing=float(spacing), origin=(o, o, o), gaussians=g)


@dataclass
class PocketAtoms:
    """Pocket atoms for the pairwise rescoring stand-in: positions in the grid's
    frame (float32 [n, 3]), types (uint8 [n]), the integer pair weight of a
    ligand atom of grid type t and a pocket atom of type u (int32 [t, u]), and
    the contact distance (Angstrom)."""
    xyz: np.ndarray
    type: np.ndarray
    ntypes: int
    weight: np.ndarray
    contact_dist: float


def pocket_atoms(seed: int, pocket: Pocket, density: float = 0.04, cavity_frac: float = 0.4,
                 ntypes: int = 4, contact_dist: float = 4.0, weights=(-2, 3)) -> PocketAtoms:
    """Atoms uniform in the grid box (density per cubic Angstrom) outside a central
    cavity sphere (radius cavity_frac times the half extent), where the docked
    ligands sit; types U{0..ntypes-1}; weights U{weights[0]..weights[1]}."""
    rng = np.random.default_rng([seed, 0x6A70])
    nx, ny, nz = pocket.shape_xyz
    half = pocket.spacing * (np.array([nx, ny, nz]) - 1) / 2.0
    centre = np.array(pocket.origin) + half
    rc = cavity_frac * float(half.min())
    vol = float(np.prod(2 * half)) - 4.0 / 3.0 * np.pi * rc ** 3
    n = int(round(density * vol))
    pts = np.zeros((0, 3))
    while len(pts) < n:
        cand = rng.uniform(-half, half, size=(2 * n + 16, 3))
        cand = cand[np.linalg.norm(cand, axis=1) >= rc]
        pts = np.concatenate([pts, cand])
    xyz = (pts[:n] + centre).astype(np.float32)
    typ = rng.integers(0, ntypes, size=n).astype(np.uint8)
    w = rng.integers(weights[0], weights[1] + 1, size=(pocket.ntypes, ntypes)).astype(np.int32)
    return PocketAtoms(xyz=xyz, type=typ, ntypes=int(ntypes), weight=w,
                       contact_dist=float(contact_dist))


def library_from_sizes(seed: int, n_atoms, n_rot, ntypes: int = 4, clash_dist: float = 2.05,
                       mask_words: int | None = None) -> Library:
    n_atoms = np.ascontiguousarray(n_atoms, np.int32)
    n_rot = np.ascontiguousarray(n_rot, np.int32)
    L = len(n_atoms)
    if mask_words is None:
        mask_words = max(1, (int(n_atoms.max(initial=1)) + 63) // 64)
    A = int(n_atoms.sum())
    Br = int(n_rot.sum())
    atom_off = np.zeros(L + 1, np.int32)
    xyz = np.zeros((A, 3), np.float32)
    typ = np.zeros(A, np.uint8)
    bond_off = np.zeros(L + 1, np.int32)
    bonds = np.zeros((max(A - L, 0), 2), np.int32)
    rot_off = np.zeros(L + 1, np.int32)
    rot_bond = np.zeros((Br, 2), np.int32)
    rot_mask = np.zeros((Br, mask_words), np.uint64)
    b_act = np.zeros(L, np.int32)
    rc = _L().synth_library(seed, L, _p(n_atoms), _p(n_rot), ntypes, clash_dist, mask_words,
                            _p(atom_off), _p(xyz), _p(typ), _p(bond_off), _p(bonds), _p(rot_off),
                            _p(rot_bond), _p(rot_mask), _p(b_act))
    if rc:
        raise ValueError(f"synth_library failed ({rc})")
    nr = int(rot_off[-1])
    return Library(atom_off=atom_off, xyz=xyz, type=typ, bond_off=bond_off, bonds=bonds,
                   rot_off=rot_off, rot_bond=rot_bond[:nr].copy(), rot_mask=rot_mask[:nr].copy(),
                   mask_words=mask_words, n_rot_requested=n_rot)


def library_uniform(seed: int, L: int, atoms: tuple, rot: tuple, ntypes: int = 4,
                    mask_words: int | None = None) -> Library:
    n = np.zeros(L, np.int32)
    b = np.zeros(L, np.int32)
    rc = _L().synth_sizes_uniform(seed, L, atoms[0], atoms[1], rot[0], rot[1], _p(n), _p(b))
    if rc:
        raise ValueError("bad size ranges")
    return library_from_sizes(seed, n, b, ntypes, mask_words=mask_words)


def library_lognormal(seed: int, L: int, median=40.0, sigma_log=0.5, atoms=(12, 150), lam=6.0,
                      bmax=30, ntypes: int = 4) -> Library:
    n = np.zeros(L, np.int32)
    b = np.zeros(L, np.int32)
    rc = _L().synth_sizes_lognormal(seed, L, median, sigma_log, atoms[0], atoms[1], lam, bmax,
                                    _p(n), _p(b))
    if rc:
        raise ValueError("bad size ranges")
    return library_from_sizes(seed, n, b, ntypes)


def start_quats(seed: int, R: int) -> np.ndarray:
    """R uniformly random unit quaternions (w, x, y, z), float32 [R, 4]."""
    q = np.zeros((R, 4), np.float32)
    _L().synth_start_quats(seed, R, _p(q))
    return q


# ---------------------------------------------------------------------------
# Workload recipes (sizes, distributions and search settings of the paper-shaped
# synthetic workloads).
CONFIGS = {
    1: dict(name="c1-plain-small", pocket=dict(ntypes=4, n=32, spacing=0.5, ngauss=40,
                                               centre_half=4.0),
            ligands=dict(L=8, atoms=(20, 20), rot=(3, 3)),
            search=dict(restarts=16, torsion_steps=64, sweep_passes=2, align_steps=30, top_k=16,
                        dedup_rmsd=2.0)),
    2: dict(name="c2-plain-paper-scale", pocket=dict(ntypes=4, n=96, spacing=0.375, ngauss=160,
                                                     centre_half=9.0),
            ligands=dict(L=10000, atoms=(20, 80), rot=(2, 12)),
            search=dict(restarts=256, torsion_steps=256, sweep_passes=3, align_steps=30, top_k=30,
                        dedup_rmsd=2.0)),
    3: dict(name="c3-batched", pocket=dict(ntypes=4, n=96, spacing=0.375, ngauss=160,
                                           centre_half=9.0),
            ligands=dict(L=200000, atoms=(20, 100), rot=(0, 20)),
            search=dict(restarts=256, torsion_steps=256, sweep_passes=3, align_steps=30, top_k=30,
                        dedup_rmsd=2.0)),
}


def config(idx: int, n_ligands: int | None = None):
    """(pocket, library, quats, search) for a workload recipe; the seed is
    MASTER_SEED + idx.  n_ligands truncates the library (same per-ligand streams)."""
    c = CONFIGS[idx]
    seed = MASTER_SEED + idx
    pk = pocket_gaussians(seed, **c["pocket"])
    lg = dict(c["ligands"])
    L = lg.pop("L") if n_ligands is None else n_ligands
    lib = library_uniform(seed, L, lg["atoms"], lg["rot"], ntypes=c["pocket"]["ntypes"])
    q = start_quats(seed, c["search"]["restarts"])
    return pk, lib, q, dict(c["search"])
