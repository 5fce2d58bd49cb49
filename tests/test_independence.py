"""The oracle and the product path share nothing, and the product path has no fallback.

- No module of the package imports the oracle, and no oracle module imports the package (the
  seeded input generators in `paper_2412_20884_amd/inputs.py` are the one shared module; it
  imports neither side and holds none of the method's arithmetic).
- No HIP source includes anything from the oracle or the tests.
- No committed source reads the git-ignored working folder (`_work/`).
- Without the built library the binding raises instead of computing anything.
"""
import ast
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2412_20884_amd")
ORACLE = os.path.join(ROOT, "oracle")


def _py_files(top):
    for d, _, files in os.walk(top):
        if "__pycache__" in d:
            continue
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(d, f)


def _imported_roots(path):
    tree = ast.parse(open(path).read(), filename=path)
    roots = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            roots.update(a.name.split(".")[0] for a in node.names)
        elif isinstance(node, ast.ImportFrom) and node.level == 0 and node.module:
            roots.add(node.module.split(".")[0])
        elif isinstance(node, ast.Call) and getattr(node.func, "attr", "") == "import_module":
            for a in node.args:
                if isinstance(a, ast.Constant) and isinstance(a.value, str):
                    roots.add(a.value.split(".")[0])
    return roots


def test_package_never_imports_the_oracle():
    for p in _py_files(PKG):
        assert "oracle" not in _imported_roots(p), p


def test_oracle_never_imports_the_package():
    for p in _py_files(ORACLE):
        assert "paper_2412_20884_amd" not in _imported_roots(p), p


def test_input_generators_import_neither_side():
    roots = _imported_roots(os.path.join(PKG, "inputs.py"))
    assert not roots & {"oracle", "paper_2412_20884_amd", "torch"}, roots


def test_hip_sources_include_nothing_from_oracle_or_tests():
    inc = re.compile(r'^\s*#\s*include\s*[<"]([^>"]+)[>"]', re.M)
    for d, _, files in os.walk(os.path.join(PKG, "csrc")):
        for f in files:
            if f.endswith((".hip", ".h", ".inc")):
                for name in inc.findall(open(os.path.join(d, f)).read()):
                    assert "oracle" not in name and "tests" not in name, (f, name)


def test_no_committed_source_reads_the_working_folder():
    targets = [os.path.join(ROOT, "bench.py"), os.path.join(ROOT, "__graft_entry__.py")]
    for top in (PKG, ORACLE, os.path.join(ROOT, "tests"), os.path.join(ROOT, "include")):
        for d, _, files in os.walk(top):
            if "__pycache__" in d:
                continue
            targets += [os.path.join(d, f) for f in files
                        if f.endswith((".py", ".hip", ".h", ".inc", ".sh"))]
    pat = re.compile(r"[\"'/]_work\b")
    here = os.path.abspath(__file__)
    for t in targets:
        if os.path.abspath(t) == here:
            continue
        assert not pat.search(open(t).read()), t


def test_binding_raises_without_the_library(monkeypatch, tmp_path):
    from paper_2412_20884_amd import gpk

    # both attributes are restored when the test ends
    monkeypatch.setattr(gpk, "LIB_PATH", str(tmp_path / "missing_libgpk.so"))
    monkeypatch.setattr(gpk, "_LIB", None)
    with pytest.raises(RuntimeError, match="not built"):
        gpk.lib()
