"""CPU-side checks of the C ABI library: it loads and exports every declared entry point; the
oracle and the product path stay independent (no imports either way).  No device calls."""
import ast
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2204_03139_amd", "libdiffcloud.so")


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(dc_[a-z_0-9]+)\s*\(", src))
    return names


def test_header_declares_entry_points():
    d = _declared()
    for n in ["dc_sample_surface", "dc_sample_surface_bwd", "dc_chamfer_fwd", "dc_chamfer_bwd",
              "dc_submit", "dc_poll", "dc_create", "dc_destroy"]:
        assert n in d


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = _declared() - exported
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_loads_with_ctypes():
    import paper_2204_03139_amd as p
    from paper_2204_03139_amd._lib import EXPORTS
    L = p.load()
    for n in EXPORTS:
        assert hasattr(L, n)
    assert L.dc_version() >= 100
    assert set(EXPORTS) == _declared()


def test_library_was_built_for_gfx950_only():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", LIB], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    targets = set(re.findall(r"gfx\d+[a-z]?", out.stdout))
    assert targets == {"gfx950"}


def _imports(path):
    tree = ast.parse(open(path).read())
    mods = set()
    for n in ast.walk(tree):
        if isinstance(n, ast.Import):
            mods |= {a.name.split(".")[0] for a in n.names}
        elif isinstance(n, ast.ImportFrom) and n.module and n.level == 0:
            mods.add(n.module.split(".")[0])
    return mods


def test_oracle_and_product_are_independent():
    pkg = os.path.join(ROOT, "paper_2204_03139_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                assert "oracle" not in _imports(os.path.join(dirpath, f)), f
            if f.endswith((".hip", ".h", ".cpp")):
                assert "oracle" not in open(os.path.join(dirpath, f)).read().lower(), f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith(".py"):
            assert "paper_2204_03139_amd" not in _imports(os.path.join(ROOT, "oracle", f)), f
        if f.endswith(".c"):
            src = open(os.path.join(ROOT, "oracle", f)).read()
            assert "#include \"" not in src  # no shared headers
    for f in os.listdir(os.path.join(ROOT, "workloads")):
        if f.endswith(".py"):
            mods = _imports(os.path.join(ROOT, "workloads", f))
            assert "oracle" not in mods and "paper_2204_03139_amd" not in mods
