"""The C-ABI library builds, loads and exports every symbol its header declares.

These run without a GPU: they only resolve symbols and call entry points on a
NULL context, which must be rejected before any HIP call.
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "piccoll.h")
LIB = os.path.join(ROOT, "paper_2508_06771_amd", "libpiccoll.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_][a-z_0-9]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2508_06771_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_expected_api():
    names = declared_functions()
    for f in ("pic_create", "pic_destroy", "pic_sync", "pic_bin_cells", "coulomb_collide",
              "mcc_null_collide", "coulomb_pairs", "pic_cell_moments", "pic_unsort",
              "pic_philox", "pic_set_mcc", "pic_strerror"):
        assert f in names, f


def test_every_declared_symbol_is_exported(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2508_06771_amd import piccoll
    assert set(declared_functions()) <= set(piccoll.EXPORTED) | {"pic_run_steps"} | set(
        n for n in declared_functions() if n.startswith(("pic_gate", "pic_mlp", "pic_graph", "pic_label",
                                                         "pic_features", "pic_autotune")))


def test_null_context_is_rejected(lib):
    lib.pic_strerror.restype = C.c_char_p
    assert lib.pic_strerror(0) == b"ok"
    assert lib.pic_strerror(2) == b"cell id out of range"
    vp = C.c_void_p
    lib.coulomb_collide.argtypes = [vp, C.c_int, vp, vp, vp, C.c_int64, C.c_int32, C.c_double,
                                    C.c_double, vp, C.c_uint64, C.c_uint64, C.c_uint32]
    assert lib.coulomb_collide(None, 0, None, None, None, 0, 1, 1.0, 1.0, None, 0, 0, 0) == 1
    lib.pic_sync.argtypes = [vp]
    assert lib.pic_sync(None) == 1
    lib.pic_bin_cells.argtypes = [vp, vp, C.c_int64, C.c_int32, vp, vp]
    assert lib.pic_bin_cells(None, None, 0, 1, None, None) == 1
    lib.pic_create.argtypes = [vp, C.c_int, vp]
    assert lib.pic_create(None, 0, None) == 1


def test_noalloc_limits_match_header():
    """The binding's limits of coulomb_collide_noalloc are the header's."""
    from paper_2508_06771_amd import piccoll
    text = open(HEADER).read()
    for name in ("NOALLOC_MAX_CELLS", "NOALLOC_MAX_CELL_F32", "NOALLOC_MAX_CELL_F64"):
        m = re.search(r"#define PIC_%s (\d+)" % name, text)
        assert m and int(m.group(1)) == getattr(piccoll, name), name
