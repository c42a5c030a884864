"""ctypes binding of the FP64 docking oracle (dock_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  The GPU library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dock_oracle.c")
_LIBPATH = os.path.join(_HERE, "liboracle.so")
NONE_ACCEPTED = 0xFFFF
# class of a followed decision (decision_class / final_class)
EXACT, SCORE_TIE, BUMP_TIE, MISMATCH, NOT_FOLLOWED = 0, 1, 2, 3, 255
ABS_TIE = 1e-5


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIBPATH):
        tmp = _LIBPATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIBPATH)
    return _LIBPATH


P = ctypes.c_void_p


class _Grid(ctypes.Structure):
    _fields_ = [("ntypes", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("spacing", ctypes.c_double),
                ("origin", ctypes.c_double * 3), ("values", P)]


class _Ligand(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("xyz", P), ("type", P), ("nbonds", ctypes.c_int),
                ("bonds", P), ("nrot", ctypes.c_int), ("rot_bond", P), ("rot_mask", P),
                ("mask_words", ctypes.c_int)]


class _Params(ctypes.Structure):
    _fields_ = [("restarts", ctypes.c_int), ("start_quat", P), ("torsion_steps", ctypes.c_int),
                ("sweep_passes", ctypes.c_int), ("align_steps", ctypes.c_int),
                ("top_k", ctypes.c_int), ("final_align", ctypes.c_int),
                ("bump_min_bonds", ctypes.c_int), ("bump_dist", ctypes.c_double),
                ("dedup_rmsd", ctypes.c_double)]


class _Follow(ctypes.Structure):
    _fields_ = [("trace", P), ("nsel", ctypes.c_int), ("sel_restart", P), ("final_trace", P),
                ("tie_rel", ctypes.c_double), ("bump_tol", ctypes.c_double)]


class _PocketAtoms(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int), ("ntypes", ctypes.c_int), ("xyz", P), ("type", P),
                ("contact_dist", ctypes.c_double), ("lig_ntypes", ctypes.c_int), ("weight", P)]


class _Result(ctypes.Structure):
    _fields_ = [("restart_score", P), ("restart_pose", P), ("decision_score", P), ("trace", P),
                ("n_sel", ctypes.c_int32), ("sel_restart", P), ("pose_score", P),
                ("pose_xyz", P), ("final_trace", P), ("decision_class", P),
                ("final_class", P), ("stats", ctypes.c_double * 8)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            build(force=True)
        lib = ctypes.CDLL(_LIBPATH)
        G = ctypes.POINTER(_Grid)
        lib.oracle_interp.argtypes = [G, ctypes.c_int, P]
        lib.oracle_interp.restype = ctypes.c_double
        lib.oracle_score.argtypes = [G, ctypes.c_int, P, P]
        lib.oracle_score.restype = ctypes.c_double
        lib.oracle_topo.argtypes = [ctypes.c_int, ctypes.c_int, P, P]
        lib.oracle_check_ligand.argtypes = [G, ctypes.POINTER(_Ligand)]
        lib.oracle_quat_matrix.argtypes = [P, P]
        lib.oracle_align_matrix.argtypes = [ctypes.c_int, ctypes.c_int, P]
        lib.oracle_select.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int,
                                      ctypes.c_double, P]
        lib.oracle_contacts.argtypes = [ctypes.POINTER(_PocketAtoms), ctypes.c_int, P, P,
                                        ctypes.c_double, P]
        lib.oracle_contacts.restype = ctypes.c_longlong
        lib.oracle_dock_ligand.argtypes = [G, ctypes.POINTER(_Ligand), ctypes.POINTER(_Params),
                                           ctypes.POINTER(_Follow), ctypes.POINTER(_Result)]
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


class Grid:
    """Holds the ctypes grid struct and keeps the value array alive."""

    def __init__(self, values, spacing, origin):
        self.values = np.ascontiguousarray(values, np.float32)
        t, nz, ny, nx = self.values.shape
        self.s = _Grid(t, nx, ny, nz, float(spacing), (ctypes.c_double * 3)(*origin),
                       _ptr(self.values))

    @classmethod
    def of(cls, pocket):
        return cls(pocket.values, pocket.spacing, pocket.origin)


def _grid(g):
    return g if isinstance(g, Grid) else Grid.of(g)


def interp(grid, t, p):
    g = _grid(grid)
    p = np.ascontiguousarray(p, np.float64)
    return _L().oracle_interp(ctypes.byref(g.s), int(t), _ptr(p))


def score(grid, types, xyz):
    g = _grid(grid)
    types = np.ascontiguousarray(types, np.uint8)
    xyz = np.ascontiguousarray(xyz, np.float64)
    return _L().oracle_score(ctypes.byref(g.s), len(types), _ptr(types), _ptr(xyz))


def topo(n, bonds):
    bonds = np.ascontiguousarray(bonds, np.int32).reshape(-1, 2)
    d = np.zeros((n, n), np.int32)
    _L().oracle_topo(n, len(bonds), _ptr(bonds), _ptr(d))
    return d


def quat_matrix(q):
    q = np.ascontiguousarray(q, np.float32)
    M = np.zeros(9, np.float64)
    _L().oracle_quat_matrix(_ptr(q), _ptr(M))
    return M.reshape(3, 3)


def align_matrix(A, o):
    M = np.zeros(9, np.float64)
    _L().oracle_align_matrix(A, o, _ptr(M))
    return M.reshape(3, 3)


def select(scores, poses, K, delta):
    scores = np.ascontiguousarray(scores, np.float64)
    poses = np.ascontiguousarray(poses, np.float64)
    R = len(scores)
    n = poses.shape[1]
    sel = np.zeros(max(K, R), np.int32)
    ns = _L().oracle_select(R, n, _ptr(scores), _ptr(poses), K, float(delta), _ptr(sel))
    return sel[:ns].copy()


class PocketAtoms:
    """Pocket atoms of the pairwise rescoring stand-in (keeps the arrays alive)."""

    def __init__(self, xyz, types, ntypes, weight, contact_dist):
        self.xyz = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
        self.type = np.ascontiguousarray(types, np.uint8)
        self.weight = np.ascontiguousarray(weight, np.int32)
        lig_ntypes, nt = self.weight.shape
        assert nt == ntypes
        self.s = _PocketAtoms(len(self.type), int(ntypes), _ptr(self.xyz), _ptr(self.type),
                              float(contact_dist), int(lig_ntypes), _ptr(self.weight))

    @classmethod
    def of(cls, pa):
        return cls(pa.xyz, pa.type, pa.ntypes, pa.weight, pa.contact_dist)


def contacts(pocket_atoms, types, xyz, tol=0.0):
    """(contact score, boundary weight) of a pose: see oracle_contacts."""
    pa = pocket_atoms if isinstance(pocket_atoms, PocketAtoms) else PocketAtoms.of(pocket_atoms)
    types = np.ascontiguousarray(types, np.uint8)
    xyz = np.ascontiguousarray(xyz, np.float64).reshape(-1, 3)
    b = ctypes.c_longlong(0)
    v = _L().oracle_contacts(ctypes.byref(pa.s), len(types), _ptr(types), _ptr(xyz), float(tol),
                             ctypes.byref(b))
    return int(v), int(b.value)


class LigandArrays:
    def __init__(self, xyz, types, bonds, rot_bond, rot_mask, mask_words=None):
        self.xyz = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
        self.type = np.ascontiguousarray(types, np.uint8)
        self.bonds = np.ascontiguousarray(bonds, np.int32).reshape(-1, 2)
        self.rot_bond = np.ascontiguousarray(rot_bond, np.int32).reshape(-1, 2)
        n = len(self.xyz)
        W = mask_words if mask_words is not None else max(1, (n + 63) // 64)
        self.rot_mask = np.ascontiguousarray(rot_mask, np.uint64).reshape(-1, W)
        self.s = _Ligand(n, _ptr(self.xyz), _ptr(self.type), len(self.bonds), _ptr(self.bonds),
                         len(self.rot_bond), _ptr(self.rot_bond), _ptr(self.rot_mask), W)

    @property
    def n(self):
        return len(self.xyz)

    @property
    def nrot(self):
        return len(self.rot_bond)


def ligand_from_library(lib, l):
    x, t, b, r, m = lib.ligand(l)
    return LigandArrays(x, t, b, r, m, lib.mask_words)


def check_ligand(grid, lig):
    g = _grid(grid)
    return _L().oracle_check_ligand(ctypes.byref(g.s), ctypes.byref(lig.s))


DEFAULTS = dict(torsion_steps=64, sweep_passes=2, align_steps=30, top_k=16, final_align=1,
                bump_min_bonds=4, bump_dist=2.0, dedup_rmsd=2.0)


def dock_ligand(grid, lig, quats, follow=None, decisions=False, **params):
    """Dock one ligand.  params: torsion_steps, sweep_passes, align_steps, top_k,
    final_align, bump_min_bonds, bump_dist, dedup_rmsd (defaults in DEFAULTS).
    follow: dict(trace=[R, 1+P*B] u16, sel_restart=[ns] i32, final_trace=[ns] u16,
    tie_rel, bump_tol) to replay another implementation's decisions."""
    g = _grid(grid)
    p = dict(DEFAULTS)
    p.update({k: v for k, v in params.items() if k in DEFAULTS})
    quats = np.ascontiguousarray(quats, np.float32).reshape(-1, 4)
    R = len(quats)
    n, B = lig.n, lig.nrot
    D = 1 + p["sweep_passes"] * B
    K = p["top_k"]
    ps = _Params(R, _ptr(quats), p["torsion_steps"], p["sweep_passes"], p["align_steps"], K,
                 p["final_align"], p["bump_min_bonds"], p["bump_dist"], p["dedup_rmsd"])
    out = dict(
        restart_score=np.zeros(R, np.float64),
        restart_pose=np.zeros((R, n, 3), np.float64),
        decision_score=np.zeros((R, 1 + D), np.float64) if decisions else None,
        trace=np.zeros((R, D), np.uint16),
        sel_restart=np.zeros(max(K, 1), np.int32),
        pose_score=np.zeros(max(K, 1), np.float64),
        pose_xyz=np.zeros((max(K, 1), n, 3), np.float64),
        final_trace=np.zeros(max(K, 1), np.uint16),
        decision_class=np.zeros((R, D), np.uint8),
        final_class=np.zeros(max(K, 1), np.uint8),
    )
    res = _Result(_ptr(out["restart_score"]), _ptr(out["restart_pose"]),
                  _ptr(out["decision_score"]), _ptr(out["trace"]), 0, _ptr(out["sel_restart"]),
                  _ptr(out["pose_score"]), _ptr(out["pose_xyz"]), _ptr(out["final_trace"]),
                  _ptr(out["decision_class"]), _ptr(out["final_class"]))
    fs = None
    keep = []
    if follow is not None:
        tr = np.ascontiguousarray(follow["trace"], np.uint16).reshape(R, D)
        sel = follow.get("sel_restart")
        ft = follow.get("final_trace")
        keep += [tr]
        sel_a = np.ascontiguousarray(sel, np.int32) if sel is not None else None
        ft_a = np.ascontiguousarray(ft, np.uint16) if ft is not None else None
        keep += [sel_a, ft_a]
        fs = _Follow(_ptr(tr), 0 if sel_a is None else len(sel_a), _ptr(sel_a), _ptr(ft_a),
                     float(follow.get("tie_rel", 1e-5)), float(follow.get("bump_tol", 1e-4)))
    rc = _L().oracle_dock_ligand(ctypes.byref(g.s), ctypes.byref(lig.s), ctypes.byref(ps),
                                 ctypes.byref(fs) if fs is not None else None, ctypes.byref(res))
    if rc:
        raise ValueError(f"oracle_dock_ligand rejected the input ({rc})")
    ns = res.n_sel
    out["n_sel"] = ns
    for k in ("sel_restart", "pose_score", "pose_xyz", "final_trace", "final_class"):
        out[k] = out[k][:ns].copy()
    st = list(res.stats)
    # score_ties: gap within tie_rel*max(1,|best|); score_ties_beyond_abs: of those, the
    # ties whose gap exceeds ABS_TIE (they would be mismatches under an absolute tolerance)
    out["stats"] = dict(decisions=int(st[0]), exact=int(st[1]), score_ties=int(st[2]),
                        bump_ties=int(st[3]), mismatches=int(st[4]), above_applied=int(st[5]),
                        max_tie_gap=st[6], score_ties_beyond_abs=int(st[7]))
    out["best_score"] = float(out["pose_score"][0]) if ns else float("-inf")
    return out
