"""The oracle and the HIP path share no code, and the product path never
uses the oracle: no source of one names the other, the built libraries
export none of each other's symbols, and only the CPU baseline of bench.py,
smoke() and (to build it) build() touch the oracle package. The seeded input
generators (fixtures/) import neither side."""
import ast
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1906_01128_amd")


def _sources(top, exts):
    for d, _, files in os.walk(top):
        if "__pycache__" in d or os.sep + "_lib" in d:
            continue
        for f in files:
            if f.endswith(exts):
                yield os.path.join(d, f)


def test_product_sources_do_not_name_the_oracle():
    for p in _sources(PKG, (".py", ".cpp", ".hip", ".h")):
        text = open(p).read()
        assert not re.search(r"\boracle\b|liboracle|\bor_[a-z_]+\(", text, re.I), p


def _imports(path):
    out = set()
    for node in ast.walk(ast.parse(open(path).read())):
        if isinstance(node, ast.Import):
            out |= {a.name for a in node.names}
        elif isinstance(node, ast.ImportFrom):
            out.add(node.module or "")
        elif isinstance(node, ast.Call) and getattr(node.func, "attr", "") == "import_module":
            out |= {a.value for a in node.args if isinstance(a, ast.Constant)}
    return out


def test_oracle_sources_do_not_use_the_library():
    for p in _sources(os.path.join(ROOT, "oracle"), (".py", ".c", ".h")):
        if p.endswith(".py"):
            assert not any(m.startswith("paper_1906_01128_amd") for m in _imports(p)), p
        else:
            text = open(p).read()
            assert not re.search(r"#include\s*[<\"](hip/|dc)", text), p
            assert not re.search(r"\bdc_[a-z_]+\(", text), p


def test_fixtures_import_neither_side():
    for p in _sources(os.path.join(ROOT, "fixtures"), (".py", ".c", ".h")):
        text = open(p).read()
        assert "paper_1906_01128_amd" not in text and not re.search(r"import oracle|from oracle", text), p
        assert not re.search(r"#include\s*[<\"](hip/|dc|oracle)", text), p


def _exports(lib):
    r = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True)
    if r.returncode:
        pytest.skip(f"nm failed on {lib}")
    return {ln.split()[-1] for ln in r.stdout.splitlines() if ln.strip()}


def test_built_libraries_do_not_export_each_others_symbols():
    libdc = os.path.join(PKG, "_lib", "libdc.so")
    liboracle = os.path.join(ROOT, "oracle", "liboracle.so")
    if not (os.path.exists(libdc) and os.path.exists(liboracle)):
        pytest.skip("libraries not built")
    dc_syms, or_syms = _exports(libdc), _exports(liboracle)
    assert not any(s.startswith("or_") for s in dc_syms)
    assert not any(s.startswith("dc_") for s in or_syms)


def _functions_importing_oracle(path):
    tree = ast.parse(open(path).read())
    found = []
    for node in ast.walk(tree):
        if isinstance(node, ast.FunctionDef):
            for sub in ast.walk(node):
                names = []
                if isinstance(sub, ast.Import):
                    names = [a.name for a in sub.names]
                elif isinstance(sub, ast.ImportFrom):
                    names = [sub.module or ""]
                elif isinstance(sub, ast.Call) and getattr(sub.func, "attr", "") == "import_module":
                    names = [a.value for a in sub.args if isinstance(a, ast.Constant)]
                if any(n == "oracle" or n.startswith("oracle.") for n in names):
                    found.append(node.name)
    module_level = [n for n in tree.body if isinstance(n, (ast.Import, ast.ImportFrom))
                    and any(getattr(a, "name", "") == "oracle" for a in getattr(n, "names", []))]
    return sorted(set(found)), module_level


def test_only_the_baseline_smoke_and_build_touch_the_oracle():
    fns, top = _functions_importing_oracle(os.path.join(ROOT, "bench.py"))
    assert fns == ["cpu_baseline_linear", "cpu_baseline_md"] and not top
    fns, top = _functions_importing_oracle(os.path.join(ROOT, "__graft_entry__.py"))
    assert set(fns) <= {"build", "smoke"} and not top
