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


STRUCTS = {"ann_search_opts": "SearchOptions", "ann_index_info": "IndexInfo",
           "ann_server_opts": "ServerOptions", "ann_result": "Result",
           "ann_server_stats": "ServerStats"}


def test_struct_layouts_match_header(tmp_path):
    """Every struct of the header has the size and field offsets of its
    ctypes mirror (gcc compiles the header and prints them)."""
    import subprocess

    from paper_2507_10070_amd import flashann

    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "flashann.h"',
             "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        cls = getattr(flashann, pyname)
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(line.rsplit(" ", 1) for line in
               subprocess.run([str(exe)], check=True, capture_output=True, text=True)
               .stdout.splitlines())
    for cname, pyname in STRUCTS.items():
        cls = getattr(flashann, pyname)
        assert int(out["%s size" % cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(out["%s.%s" % (cname, fname)]) == getattr(cls, fname).offset, (cname, fname)
