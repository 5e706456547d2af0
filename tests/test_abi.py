"""CPU-only checks of the C ABI boundary: the library loads and exports
every function include/gsi.h declares, and the binding covers all of them."""
import os
import re

import pytest

import paper_1906_03420_amd as gsi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gsi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsi_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gsi_ctx_create", "gsi_graph_load", "gsi_query_run", "gsi_result_rows", "gsi_result_count",
                 "gsi_result_digest", "gsi_result_free", "gsi_graph_free", "gsi_ctx_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = gsi.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    names = declared_functions()
    assert sorted(gsi.binding.SIGNATURES) == names
    for name in names:
        assert callable(getattr(gsi.binding, name)), name


def test_binding_constants_match_header():
    text = open(os.path.join(ROOT, "include", "gsi.h")).read()
    defs = re.findall(r"#define\s+(GSI_[A-Z0-9_]+)\s+(0x[0-9a-fA-F]+|\d+)u?\b", text)
    assert len(defs) >= 10
    for name, val in defs:
        assert getattr(gsi.binding, name) == int(val, 0), name
    enum = re.search(r"typedef enum \{(.*?)\} gsi_status;", text, flags=re.S).group(1)
    for name, val in re.findall(r"(GSI_[A-Z_]+)\s*=\s*(\d+)", enum):
        assert getattr(gsi.binding, name) == int(val), name


def test_host_side_errors_without_gpu():
    assert "gfx950" in gsi.gsi_version()
    with pytest.raises(gsi.GsiError) as e:
        gsi.gsi_ctx_create(0, 0, 0, 1 << 20)
    assert e.value.status == gsi.GSI_E_INVALID
    assert gsi.gsi_graph_bytes_needed(1000, 5000) > 64 * 1000


def test_no_cpu_fallback_path():
    # the package imports nothing from the oracle
    import ast
    for fn in ("__init__.py", "binding.py", "build.py"):
        tree = ast.parse(open(os.path.join(ROOT, "paper_1906_03420_amd", fn)).read())
        for node in ast.walk(tree):
            if isinstance(node, (ast.Import, ast.ImportFrom)):
                mods = [a.name for a in node.names] if isinstance(node, ast.Import) else [node.module or ""]
                assert not any(m.split(".")[0] == "oracle" for m in mods)
