"""The C-ABI library loads and exports every symbol include/dock.h declares;
host-side argument checks work without a GPU (no compute call is made)."""
import ctypes
import os
import re

import pytest

from paper_1901_06229_amd import build as dock_build
from paper_1901_06229_amd import dock

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(dock_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(dock_build.LIB_PATH):
        dock_build.build()
    return dock.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_functions("dock.h")
    assert {"dock_init_pocket", "dock_batch", "dock_batch_async", "dock_free_pocket"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_strerror_and_workspace_size(lib):
    assert lib.dock_strerror(0) == b"ok"
    assert lib.dock_strerror(dock.DOCK_E_LIMIT) == b"outside a documented limit"
    a = dock.dock_workspace_size(100, 700, 256, 256)
    b = dock.dock_workspace_size(100, 700, 256, 512)
    assert 0 < a < b
    assert a >= 700 * 256 * 2 + 100 * 8
    assert lib.dock_workspace_size(-1, 0, 1, 1, 1, 0) == 0
    assert lib.dock_workspace_size(1, 0, 1, 1, 1, -1) == 0
    # alignment: a 48-byte transform and a 2-byte index per item
    assert dock.dock_workspace_size(100, 700, 256, 256, n_align=64) - a == 50 * 100 * 256


def test_null_arguments_are_rejected_on_the_host(lib):
    h = ctypes.c_void_p()
    assert lib.dock_init_pocket(None, 4, 4, 4, None, 0.5, ctypes.byref(h)) == dock.DOCK_E_INVAL
    assert b"NULL" in lib.dock_last_error()
    g = (ctypes.c_float * 8)()
    o = (ctypes.c_float * 3)()
    assert lib.dock_init_pocket(g, 0, 2, 2, o, 0.5, ctypes.byref(h)) == dock.DOCK_E_LIMIT
    assert lib.dock_init_pocket(g, 2, 2, 2, o, -1.0, ctypes.byref(h)) == dock.DOCK_E_INVAL
    assert lib.dock_batch(None, None, None, 1, 1, None, None) == dock.DOCK_E_INVAL
    assert lib.dock_batch_async(None, None, None, 1, 1, None, None, None, 0, None) == dock.DOCK_E_INVAL
    assert lib.dock_batch_async_static(None, None, None, 1, 1, None, None, None) == dock.DOCK_E_INVAL
    lib.dock_free_pocket(None)


def test_bench_traffic_is_reported_only_for_the_measured_kernel(tmp_path, monkeypatch):
    """roofline.traffic comes from the committed counter summary, and only
    while the kernel code still hashes to the digest recorded with it."""
    import bench
    digest = bench.kernel_sources_digest()
    good = tmp_path / "good.md"
    good.write_text(f"# x\n\ntraffic_bytes_per_launch: 1234\nsources_sha256: {digest}\n")
    stale = tmp_path / "stale.md"
    stale.write_text("traffic_bytes_per_launch: 1234\nsources_sha256: " + "0" * 64 + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {3: str(good)})
    assert bench.measured_traffic(3) == 1234.0
    assert bench.measured_traffic(2) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {3: str(stale)})
    assert bench.measured_traffic(3) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {3: str(tmp_path / "missing.md")})
    assert bench.measured_traffic(3) is None


def test_binding_structs_match_the_header():
    """Every struct the header typedefs has a ctypes mirror in the binding
    with the same fields, in the same order and of the same sizes, so a field
    added on one side only cannot shift the others silently."""
    import ctypes
    import re
    from paper_1901_06229_amd import dock as binding
    header = open(os.path.join(ROOT, "include", "dock.h")).read()
    header = re.sub(r"/\*.*?\*/", " ", header, flags=re.S)
    sizes = {"int8_t": 1, "int16_t": 2, "int32_t": 4, "uint32_t": 4, "int": 4, "float": 4,
             "int64_t": 8, "uint64_t": 8, "double": 8, "size_t": 8}
    structs = re.findall(r"typedef struct \{(.*?)\}\s*(\w+);", header, flags=re.S)
    assert len(structs) >= 6
    for body, name in structs:
        fields = []
        for decl in body.split(";"):
            decl = decl.replace("const ", " ").strip()
            if not decl:
                continue
            base, rest = decl.split(None, 1)
            for d in rest.split(","):
                d = d.strip()
                fields.append((d.lstrip("*").strip(), 8 if d.startswith("*") else sizes[base]))
        mirror = getattr(binding, name)
        got = [(f, ctypes.sizeof(t)) for f, t in mirror._fields_]
        assert got == fields, (name, got, fields)
        # natural alignment: the C layout's size
        off = 0
        for _, sz in fields:
            off = (off + sz - 1) // sz * sz + sz
        align = max(sz for _, sz in fields)
        assert ctypes.sizeof(mirror) == (off + align - 1) // align * align, name
