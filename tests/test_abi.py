"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/dock.h, and rejects bad arguments before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dock.h")
LIB = os.path.join(ROOT, "paper_2209_05069_amd", "libdock.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(dock_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        from paper_2209_05069_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(L, n), n
    from paper_2209_05069_amd import dock
    assert sorted(dock.EXPORTS) == names


def test_null_arguments_are_rejected_with_a_message(L):
    L.dock_last_error.restype = ctypes.c_char_p
    L.dock_create.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p]
    assert L.dock_create(0, 0, None) == -1
    assert b"NULL" in L.dock_last_error()
    L.dock_destroy.argtypes = [ctypes.c_void_p]
    assert L.dock_destroy(None) == -1
    L.dock_ligands_batch.argtypes = [ctypes.c_void_p] * 6
    assert L.dock_ligands_batch(None, None, None, None, None, None) == -1
    L.dock_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
    assert L.dock_poll(None, 1, None) == -1


def test_header_structs_match_binding_layout():
    from paper_2209_05069_amd import dock
    # field order/size of the ctypes mirrors (checked against the header's fields)
    src = open(HEADER).read()
    for struct, cls in (("dock_library", dock.Library), ("dock_params", dock.Params),
                        ("dock_results", dock.Results), ("dock_grid_desc", dock.GridDesc),
                        ("dock_timing", dock.Timing), ("dock_bin_tuning", dock.BinTuning),
                        ("dock_pocket_atoms", dock.PocketAtoms)):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + struct + ";", src).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            names = decl.split(None, 1)[1] if not decl.startswith("const") else decl.split(None, 2)[2]
            for nm in names.split(","):
                nm = nm.strip().lstrip("*").strip()
                nm = re.sub(r"\[.*\]", "", nm)
                fields.append(nm)
        assert fields == [f[0] for f in cls._fields_], (struct, fields)


def test_request_bytes_needs_no_device():
    """dock_request_bytes reads sizes only: it answers on a machine without a GPU,
    grows with the library and with the optional outputs, and checks its params."""
    import numpy as np
    import synth
    from paper_2209_05069_amd import dock
    lib = synth.library_uniform(5, 6, (10, 30), (1, 4))
    big = synth.library_uniform(5, 60, (10, 30), (1, 4))
    q = synth.start_quats(5, 8)
    p = dock.SearchParams(q, torsion_steps=16, top_k=4)
    b_small = dock.dock_request_bytes(lib, p, dock.HostResults(6, int(lib.atom_off[-1]),
                                                               int(lib.rot_off[-1]), p))
    b_big = dock.dock_request_bytes(big, p, dock.HostResults(60, int(big.atom_off[-1]),
                                                             int(big.rot_off[-1]), p))
    b_trace = dock.dock_request_bytes(lib, p, dock.HostResults(
        6, int(lib.atom_off[-1]), int(lib.rot_off[-1]), p, restart_scores=True))
    assert 0 < b_small < b_big and b_small < b_trace
    bad = dock.SearchParams(q, torsion_steps=16, top_k=4, bump_prune=2)
    with pytest.raises(dock.DockError):
        dock.dock_request_bytes(lib, bad, dock.HostResults(6, int(lib.atom_off[-1]),
                                                           int(lib.rot_off[-1]), bad))
    assert np.isfinite(b_small)
