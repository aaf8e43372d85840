"""C-ABI checks that need no GPU: the library loads, and it exports every
function that include/flashann.h declares (no compute calls here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flashann.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ann_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ann_index_create", "ann_search", "ann_index_free", "ann_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2507_10070_amd import flashann

    if not os.path.exists(flashann.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    lib = ctypes.CDLL(flashann.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), "missing export " + name


def test_binding_lists_match_header():
    from paper_2507_10070_amd import flashann

    assert sorted(flashann.EXPORTED) == declared_functions()
