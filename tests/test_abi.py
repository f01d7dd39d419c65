"""Host-side checks of the C ABI: the library and the oracle build, load, and
export every entry point include/msc.h declares (no GPU work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ms_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("ms_gradient", "ms_critical", "ms_connect", "ms_complex", "ms_ctx_create", "ms_ctx_destroy",
              "ms_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2009_03707_amd import msc
    if not os.path.exists(msc.LIB_PATH):
        pytest.skip("libmsc.so not built")
    lib = ctypes.CDLL(msc.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert sorted(msc.EXPORTED) == sorted(n for n in declared_functions())


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2009_03707_amd import msc
    monkeypatch.setattr(msc, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(msc, "_LIB", None)
    with pytest.raises(RuntimeError):
        msc.lib()


def header_struct(name):
    """(field, C type) in declaration order of `typedef struct { ... } name;`
    in the header, for structs of scalar fields."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", text)
    assert m, name
    fields = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, rest = decl.split(None, 1)
        fields += [(n.strip(), ctype) for n in rest.split(",")]
    return fields


@pytest.mark.parametrize("cname,pyname", [("ms_stats", "Stats"), ("ms_timing", "Timing")])
def test_binding_structs_match_the_header(cname, pyname):
    """The ctypes mirrors of the header's result structs list the same fields
    in the same order with the same widths (a missing or moved field would
    shift every later one)."""
    from paper_2009_03707_amd import msc
    want = header_struct(cname)
    got = getattr(msc, pyname)._fields_
    assert [n for n, _ in got] == [n for n, _ in want]
    ctypes_of = {"double": ctypes.c_double, "int64_t": ctypes.c_int64, "uint64_t": ctypes.c_uint64,
                 "int32_t": ctypes.c_int32, "uint32_t": ctypes.c_uint32}
    for (n, t), (_, ct) in zip(got, want):
        assert ctypes.sizeof(t) == ctypes.sizeof(ctypes_of[ct]), n
