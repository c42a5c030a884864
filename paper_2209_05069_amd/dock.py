"""Thin ctypes binding of the C ABI in include/dock.h (same names).

Argument marshalling only: every docking step runs in the HIP library
(libdock.so).  PyTorch provides device memory and streams.  Importing this
module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libdock.so")

DOCK_OK, DOCK_EINVAL, DOCK_ENOMEM, DOCK_EAGAIN, DOCK_ENOENT, DOCK_EDEVICE, DOCK_EBUSY = \
    0, -1, -2, -3, -4, -5, -6
DOCK_MODE_BATCHED, DOCK_MODE_PLAIN = 0, 1
DOCK_TRACE_NONE = 0xFFFF
LIG_STATUS = {0: "ok", 1: "bad_size", 2: "bad_type", 3: "bad_bond", 4: "bad_mask", 5: "bad_offsets"}

P = ctypes.c_void_p


class DockError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dock error {code}: {msg}")
        self.code = code


class GridDesc(ctypes.Structure):
    _fields_ = [("ntypes", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("spacing", ctypes.c_float),
                ("origin", ctypes.c_float * 3), ("values", P)]


class Library(ctypes.Structure):
    _fields_ = [("n_ligands", ctypes.c_int32), ("mask_words", ctypes.c_int32),
                ("n_atoms_total", ctypes.c_int64), ("n_bonds_total", ctypes.c_int64),
                ("n_rot_total", ctypes.c_int64), ("atom_off", P), ("xyz", P), ("type", P),
                ("bond_off", P), ("bond", P), ("rot_off", P), ("rot_bond", P), ("rot_mask", P)]


class Params(ctypes.Structure):
    _fields_ = [("restarts", ctypes.c_int32), ("torsion_steps", ctypes.c_int32),
                ("sweep_passes", ctypes.c_int32), ("align_steps", ctypes.c_int32),
                ("top_k", ctypes.c_int32), ("final_align", ctypes.c_int32),
                ("bump_min_bonds", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("bump_prune", ctypes.c_int32), ("bin_mode", ctypes.c_int32),
                ("bump_dist", ctypes.c_float),
                ("dedup_rmsd", ctypes.c_float), ("start_quat", P)]


class Results(ctypes.Structure):
    _fields_ = [("best_score", P), ("n_poses", P), ("status", P), ("pose_score", P),
                ("pose_restart", P), ("pose_xyz", P), ("restart_score", P), ("trace", P),
                ("final_trace", P), ("pose_contacts", P)]


class PocketAtoms(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("ntypes", ctypes.c_int32),
                ("contact_dist", ctypes.c_float), ("xyz", P), ("type", P), ("weight", P)]


class BinTuning(ctypes.Structure):
    _fields_ = [("ligands", ctypes.c_int32), ("dock_waves", ctypes.c_int32),
                ("select_waves", ctypes.c_int32), ("falign_waves", ctypes.c_int32),
                ("falign_per_cu", ctypes.c_int32), ("falign_xcd", ctypes.c_int32),
                ("dock_ms", ctypes.c_float),
                ("select_ms", ctypes.c_float), ("falign_ms", ctypes.c_float),
                ("dock_ms_default", ctypes.c_float), ("select_ms_default", ctypes.c_float),
                ("falign_ms_default", ctypes.c_float)]


NUM_BINS = 8


class Timing(ctypes.Structure):
    _fields_ = [("prep_ms", ctypes.c_double), ("dock_ms", ctypes.c_double),
                ("align_ms", ctypes.c_double), ("final_ms", ctypes.c_double),
                ("calls", ctypes.c_int64),
                ("scored_samples", ctypes.c_int64)]


EXPORTS = ["dock_autotune", "dock_create", "dock_destroy", "dock_get_timing", "dock_last_error",
           "dock_ligands_batch", "dock_ligands_batch_noalloc", "dock_pocket_load",
           "dock_pocket_set_atoms", "dock_pocket_unload", "dock_poll",
           "dock_request_bytes", "dock_set_timing", "dock_set_tuning", "dock_submit", "dock_wait"]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} is missing: build it with "
                              "`python -m paper_2209_05069_amd.build`")
        # torch ships its own HIP runtime (SONAME libamdhip64.so.7); loading it first
        # makes libdock.so bind to that same runtime instead of a second copy.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIBPATH)
        L.dock_create.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(P)]
        L.dock_destroy.argtypes = [P]
        L.dock_last_error.restype = ctypes.c_char_p
        L.dock_pocket_load.argtypes = [P, ctypes.POINTER(GridDesc), ctypes.POINTER(ctypes.c_int32)]
        L.dock_pocket_unload.argtypes = [P, ctypes.c_int32]
        L.dock_pocket_set_atoms.argtypes = [P, ctypes.c_int32, ctypes.POINTER(PocketAtoms)]
        L.dock_ligands_batch.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Library),
                                         ctypes.POINTER(Params), ctypes.POINTER(Results), P]
        L.dock_ligands_batch_noalloc.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Library),
                                                 ctypes.POINTER(Params), ctypes.POINTER(Results),
                                                 P]
        L.dock_submit.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Library),
                                  ctypes.POINTER(Params), ctypes.POINTER(Results),
                                  ctypes.POINTER(ctypes.c_uint64)]
        L.dock_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]
        L.dock_request_bytes.argtypes = [ctypes.POINTER(Library), ctypes.POINTER(Params),
                                         ctypes.POINTER(Results), ctypes.POINTER(ctypes.c_uint64)]
        L.dock_wait.argtypes = [P, ctypes.c_uint64]
        L.dock_autotune.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Library),
                                    ctypes.POINTER(Params), ctypes.POINTER(BinTuning), P]
        L.dock_set_tuning.argtypes = [P, ctypes.POINTER(Params), ctypes.POINTER(BinTuning)]
        L.dock_set_timing.argtypes = [P, ctypes.c_int]
        L.dock_get_timing.argtypes = [P, ctypes.POINTER(Timing)]
        _lib = L
    return _lib


def _check(rc):
    if rc != DOCK_OK:
        raise DockError(rc, lib().dock_last_error().decode())
    return rc


def dock_last_error() -> str:
    return lib().dock_last_error().decode()


def dock_create(device: int = 0, hbm_budget_bytes: int = 0):
    h = P()
    _check(lib().dock_create(device, int(hbm_budget_bytes), ctypes.byref(h)))
    return h


def dock_destroy(ctx):
    _check(lib().dock_destroy(ctx))


def dock_pocket_load(ctx, values, spacing, origin) -> int:
    v = np.ascontiguousarray(values, np.float32)
    t, nz, ny, nx = v.shape
    gd = GridDesc(t, nx, ny, nz, float(spacing), (ctypes.c_float * 3)(*origin),
                  ctypes.c_void_p(v.ctypes.data))
    pid = ctypes.c_int32()
    _check(lib().dock_pocket_load(ctx, ctypes.byref(gd), ctypes.byref(pid)))
    return pid.value


def dock_pocket_unload(ctx, pocket_id: int):
    _check(lib().dock_pocket_unload(ctx, pocket_id))


def dock_pocket_set_atoms(ctx, pocket_id: int, xyz, types, ntypes: int, weight,
                          contact_dist: float):
    """Pocket atoms of the pairwise rescoring stand-in (see include/dock.h)."""
    x = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
    t = np.ascontiguousarray(types, np.uint8)
    w = np.ascontiguousarray(weight, np.int32)
    pa = PocketAtoms(len(t), int(ntypes), float(contact_dist), _np_ptr(x), _np_ptr(t),
                     ctypes.c_void_p(w.ctypes.data))
    _check(lib().dock_pocket_set_atoms(ctx, pocket_id, ctypes.byref(pa)))


DEFAULT_PARAMS = dict(torsion_steps=256, sweep_passes=3, align_steps=30, top_k=30, final_align=1,
                      bump_min_bonds=4, bump_dist=2.0, dedup_rmsd=2.0, mode=DOCK_MODE_BATCHED,
                      bump_prune=1, bin_mode=0)


class SearchParams:
    """dock_params plus the start orientations it points to (kept alive here)."""

    def __init__(self, start_quat, **kw):
        p = dict(DEFAULT_PARAMS)
        self.quat = np.ascontiguousarray(start_quat, np.float32).reshape(-1, 4)
        R = kw.pop("restarts", len(self.quat))
        if R != len(self.quat):
            raise ValueError(f"restarts={R} but {len(self.quat)} start orientations given")
        unknown = set(kw) - set(p)
        if unknown:
            raise TypeError(f"unknown params {unknown}")
        p.update(kw)
        self.values = p
        self.s = Params(len(self.quat), p["torsion_steps"], p["sweep_passes"], p["align_steps"],
                        p["top_k"], p["final_align"], p["bump_min_bonds"], p["mode"],
                        p["bump_prune"], p["bin_mode"], p["bump_dist"], p["dedup_rmsd"],
                        ctypes.c_void_p(self.quat.ctypes.data))

    def __getattr__(self, k):
        v = self.__dict__.get("values")
        if v is not None and k in v:
            return v[k]
        raise AttributeError(k)

    @property
    def restarts(self):
        return len(self.quat)


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else None


def _t_ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


class DeviceLibrary:
    """A CSR ligand library copied to device memory (torch tensors)."""

    def __init__(self, host, device="cuda:0"):
        import torch
        self.host = host
        self.n_ligands = int(len(host.atom_off) - 1)
        self.mask_words = int(host.mask_words)
        self.atom_off = torch.from_numpy(np.ascontiguousarray(host.atom_off, np.int32)).to(device)
        self.xyz = torch.from_numpy(np.ascontiguousarray(host.xyz, np.float32)).to(device)
        self.type = torch.from_numpy(np.ascontiguousarray(host.type, np.uint8)).to(device)
        self.bond_off = torch.from_numpy(np.ascontiguousarray(host.bond_off, np.int32)).to(device)
        self.bond = torch.from_numpy(np.ascontiguousarray(host.bonds, np.int32)).to(device)
        self.rot_off = torch.from_numpy(np.ascontiguousarray(host.rot_off, np.int32)).to(device)
        self.rot_bond = torch.from_numpy(np.ascontiguousarray(host.rot_bond, np.int32)).to(device)
        self.rot_mask = torch.from_numpy(
            np.ascontiguousarray(host.rot_mask, np.uint64).view(np.int64)).to(device)
        self.n_atoms_total = int(host.atom_off[-1])
        self.n_bonds_total = int(host.bond_off[-1])
        self.n_rot_total = int(host.rot_off[-1])
        self.s = Library(self.n_ligands, self.mask_words, self.n_atoms_total, self.n_bonds_total,
                         self.n_rot_total, _t_ptr(self.atom_off), _t_ptr(self.xyz),
                         _t_ptr(self.type), _t_ptr(self.bond_off), _t_ptr(self.bond),
                         _t_ptr(self.rot_off), _t_ptr(self.rot_bond), _t_ptr(self.rot_mask))


def host_library_struct(host):
    """dock_library over host numpy arrays (kept alive by the returned tuple)."""
    arrs = [np.ascontiguousarray(host.atom_off, np.int32), np.ascontiguousarray(host.xyz, np.float32),
            np.ascontiguousarray(host.type, np.uint8), np.ascontiguousarray(host.bond_off, np.int32),
            np.ascontiguousarray(host.bonds, np.int32), np.ascontiguousarray(host.rot_off, np.int32),
            np.ascontiguousarray(host.rot_bond, np.int32),
            np.ascontiguousarray(host.rot_mask, np.uint64)]
    L = len(arrs[0]) - 1
    s = Library(L, int(host.mask_words), int(arrs[0][-1]), int(arrs[3][-1]), int(arrs[5][-1]),
                *[_np_ptr(a) for a in arrs])
    return s, arrs


class DeviceResults:
    """Device result buffers for a library and params (torch tensors)."""

    def __init__(self, n_ligands, n_atoms_total, n_rot_total, params: SearchParams,
                 device="cuda:0", restart_scores=False, trace=False, final_trace=False,
                 contacts=False, poses=True):
        import torch
        L, K, R, Pp = n_ligands, params.top_k, params.restarts, params.sweep_passes
        self.L, self.K, self.R = L, K, R
        f32, i32, i16 = torch.float32, torch.int32, torch.int16
        self.best_score = torch.empty(L, dtype=f32, device=device)
        self.n_poses = torch.empty(L, dtype=i32, device=device)
        self.status = torch.empty(L, dtype=i32, device=device)
        self.pose_score = torch.empty(L * K, dtype=f32, device=device)
        self.pose_restart = torch.empty(L * K, dtype=i32, device=device)
        self.pose_xyz = (torch.empty(n_atoms_total * K * 3, dtype=f32, device=device)
                         if poses else None)
        self.restart_score = torch.empty(L * R, dtype=f32, device=device) if restart_scores else None
        self.trace = (torch.empty(R * (L + Pp * n_rot_total), dtype=i16, device=device)
                      if trace else None)
        self.final_trace = torch.empty(L * K, dtype=i16, device=device) if final_trace else None
        self.pose_contacts = torch.empty(L * K, dtype=i32, device=device) if contacts else None
        self.s = Results(_t_ptr(self.best_score), _t_ptr(self.n_poses), _t_ptr(self.status),
                         _t_ptr(self.pose_score), _t_ptr(self.pose_restart), _t_ptr(self.pose_xyz),
                         _t_ptr(self.restart_score), _t_ptr(self.trace), _t_ptr(self.final_trace),
                         _t_ptr(self.pose_contacts))

    def to_host(self):
        """numpy copies of every buffer (traces as uint16)."""
        out = {}
        for k in ("best_score", "n_poses", "status", "pose_score", "pose_restart", "pose_xyz",
                  "restart_score", "trace", "final_trace", "pose_contacts"):
            t = getattr(self, k)
            if t is None:
                out[k] = None
                continue
            a = t.cpu().numpy()
            if k in ("trace", "final_trace"):
                a = a.view(np.uint16)
            out[k] = a
        return out


class HostResults:
    """Host (numpy) result buffers for dock_submit."""

    def __init__(self, n_ligands, n_atoms_total, n_rot_total, params: SearchParams,
                 restart_scores=False, trace=False, final_trace=False, contacts=False,
                 poses=True):
        L, K, R, Pp = n_ligands, params.top_k, params.restarts, params.sweep_passes
        self.best_score = np.zeros(L, np.float32)
        self.n_poses = np.zeros(L, np.int32)
        self.status = np.zeros(L, np.int32)
        self.pose_score = np.zeros(L * K, np.float32)
        self.pose_restart = np.zeros(L * K, np.int32)
        self.pose_xyz = np.zeros(n_atoms_total * K * 3, np.float32) if poses else None
        self.restart_score = np.zeros(L * R, np.float32) if restart_scores else None
        self.trace = np.zeros(R * (L + Pp * n_rot_total), np.uint16) if trace else None
        self.final_trace = np.zeros(L * K, np.uint16) if final_trace else None
        self.pose_contacts = np.zeros(L * K, np.int32) if contacts else None
        self.s = Results(*[_np_ptr(getattr(self, k)) for k in (
            "best_score", "n_poses", "status", "pose_score", "pose_restart", "pose_xyz",
            "restart_score", "trace", "final_trace", "pose_contacts")])

    def to_host(self):
        return {k: getattr(self, k) for k in ("best_score", "n_poses", "status", "pose_score",
                                               "pose_restart", "pose_xyz", "restart_score",
                                               "trace", "final_trace", "pose_contacts")}


def dock_ligands_batch(ctx, pocket: int, dlib: DeviceLibrary, params: SearchParams,
                       res: DeviceResults, stream=None):
    """Enqueue docking of a device-resident library on `stream` (a torch stream,
    a raw hipStream_t int, or None for torch's current stream)."""
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    elif hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    _check(lib().dock_ligands_batch(ctx, pocket, ctypes.byref(dlib.s), ctypes.byref(params.s),
                                    ctypes.byref(res.s), ctypes.c_void_p(stream)))


NOALLOC_SCRATCH_BYTES = 64 << 20  # DOCK_NOALLOC_SCRATCH_BYTES


def dock_ligands_batch_noalloc(ctx, pocket: int, dlib: DeviceLibrary, params: SearchParams,
                               res: DeviceResults, stream=None):
    """dock_ligands_batch that allocates no device memory (tables and workspace in
    the library's fixed scratch array; batched form only, see include/dock.h)."""
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    elif hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    _check(lib().dock_ligands_batch_noalloc(ctx, pocket, ctypes.byref(dlib.s),
                                            ctypes.byref(params.s), ctypes.byref(res.s),
                                            ctypes.c_void_p(stream)))


class Submission:
    def __init__(self, ticket, keep):
        self.ticket = ticket
        self._keep = keep


def dock_submit(ctx, pocket: int, host_lib, params: SearchParams, res: HostResults):
    s, arrs = host_library_struct(host_lib)
    t = ctypes.c_uint64()
    _check(lib().dock_submit(ctx, pocket, ctypes.byref(s), ctypes.byref(params.s),
                             ctypes.byref(res.s), ctypes.byref(t)))
    return t.value


def dock_request_bytes(host_lib, params: SearchParams, res: HostResults) -> int:
    """Device bytes a dock_submit of this request needs (see include/dock.h)."""
    s, arrs = host_library_struct(host_lib)
    b = ctypes.c_uint64()
    _check(lib().dock_request_bytes(ctypes.byref(s), ctypes.byref(params.s), ctypes.byref(res.s),
                                    ctypes.byref(b)))
    return b.value


def dock_poll(ctx, ticket: int) -> bool:
    d = ctypes.c_int32()
    _check(lib().dock_poll(ctx, ticket, ctypes.byref(d)))
    return bool(d.value)


def dock_wait(ctx, ticket: int):
    _check(lib().dock_wait(ctx, ticket))


_TUNE_FIELDS = [f[0] for f in BinTuning._fields_]


def dock_autotune(ctx, pocket: int, dlib: DeviceLibrary, params: SearchParams, stream=None):
    """Tune the batched tiles per size bin on a device-resident sample; returns the
    per-bin table (list of dicts, see include/dock.h)."""
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    elif hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    out = (BinTuning * NUM_BINS)()
    _check(lib().dock_autotune(ctx, pocket, ctypes.byref(dlib.s), ctypes.byref(params.s), out,
                               ctypes.c_void_p(stream)))
    return [{k: getattr(t, k) for k in _TUNE_FIELDS} for t in out]


def dock_set_tuning(ctx, params: SearchParams, table=None):
    """Use `table` (as returned by dock_autotune) for these search settings; None
    restores the default tiles."""
    if table is None:
        _check(lib().dock_set_tuning(ctx, ctypes.byref(params.s), None))
        return
    arr = (BinTuning * NUM_BINS)()
    for i, t in enumerate(table):
        for k in _TUNE_FIELDS:
            setattr(arr[i], k, t.get(k, 0))
    _check(lib().dock_set_tuning(ctx, ctypes.byref(params.s), arr))


def dock_set_timing(ctx, enable: bool):
    _check(lib().dock_set_timing(ctx, 1 if enable else 0))


def dock_get_timing(ctx) -> dict:
    t = Timing()
    _check(lib().dock_get_timing(ctx, ctypes.byref(t)))
    return dict(prep_ms=t.prep_ms, dock_ms=t.dock_ms, align_ms=t.align_ms, final_ms=t.final_ms,
                calls=t.calls, scored_samples=t.scored_samples)


def trace_offset(l, R, P, rot_off):
    """Start of ligand l's block in the trace array."""
    return R * (l + P * int(rot_off[l]))


def ligand_outputs(h, l, atom_off, rot_off, params: SearchParams):
    """Slice ligand l's outputs out of host result arrays (dict from to_host)."""
    K, R, Pp = params.top_k, params.restarts, params.sweep_passes
    a0, a1 = int(atom_off[l]), int(atom_off[l + 1])
    n = a1 - a0
    B = int(rot_off[l + 1]) - int(rot_off[l])
    npose = int(h["n_poses"][l])
    out = dict(status=int(h["status"][l]), best_score=float(h["best_score"][l]), n_poses=npose,
               pose_score=h["pose_score"][l * K:l * K + npose].copy(),
               pose_restart=h["pose_restart"][l * K:l * K + npose].copy())
    if h.get("pose_xyz") is not None:
        out["pose_xyz"] = h["pose_xyz"][3 * a0 * K:3 * (a0 * K + npose * n)].reshape(npose, n, 3).copy()
    if h.get("restart_score") is not None:
        out["restart_score"] = h["restart_score"][l * R:(l + 1) * R].copy()
    if h.get("trace") is not None:
        b = trace_offset(l, R, Pp, rot_off)
        out["trace"] = h["trace"][b:b + R * (1 + Pp * B)].reshape(R, 1 + Pp * B).copy()
    if h.get("final_trace") is not None:
        out["final_trace"] = h["final_trace"][l * K:l * K + npose].copy()
    if h.get("pose_contacts") is not None:
        out["pose_contacts"] = h["pose_contacts"][l * K:(l + 1) * K].copy()
    return out
