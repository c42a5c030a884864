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
    L.dock_create.argtypes = [ctypes.c_int, ctypes.c_void_p]
    assert L.dock_create(0, None) == -1
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
                        ("dock_timing", dock.Timing)):
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
