"""The product path and the oracle stay apart (no GPU needed).

* No module of the package imports the oracle, and no kernel or host source
  of the library includes or names a file under oracle/; the oracle imports
  nothing of the package.
* bench.py touches the oracle only inside its CPU-baseline functions.
* The package's Python modules call no trigonometric or random function: the
  method's arithmetic runs in the library.
* The binding fails loudly (ImportError) when the HIP library is missing:
  there is no CPU fallback to take its place.
"""
import ast
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2411_16952_amd")
ORACLE = os.path.join(ROOT, "oracle")


def _imported_modules(path):
    tree = ast.parse(open(path).read(), filename=path)
    names = []
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            names += [a.name for a in node.names]
        elif isinstance(node, ast.ImportFrom) and node.module:
            names.append(node.module)
    return names


def _py_files(folder):
    return sorted(os.path.join(folder, f) for f in os.listdir(folder) if f.endswith(".py"))


def test_package_never_imports_the_oracle():
    files = _py_files(PKG)
    assert files
    for f in files:
        for m in _imported_modules(f):
            assert m.split(".")[0] != "oracle", f"{f} imports {m}"


def test_library_sources_do_not_reach_the_oracle():
    csrc = os.path.join(PKG, "csrc")
    srcs = [os.path.join(csrc, f) for f in os.listdir(csrc)]
    assert any(s.endswith(".hip") for s in srcs)
    for s in srcs:
        text = open(s).read()
        for inc in re.findall(r'^\s*#\s*include\s*[<"]([^>"]+)[>"]', text, re.M):
            assert "oracle" not in inc, f"{s} includes {inc}"
        assert "tkdv_oracle" not in text, f"{s} names the oracle library"


def test_oracle_never_imports_the_package():
    for f in _py_files(ORACLE):
        for m in _imported_modules(f):
            assert m.split(".")[0] != "paper_2411_16952_amd", f"{f} imports {m}"
    text = open(os.path.join(ORACLE, "tkdv_oracle.c")).read()
    for inc in re.findall(r'^\s*#\s*include\s*[<"]([^>"]+)[>"]', text, re.M):
        assert "tkdv_" not in inc and "csrc" not in inc, f"the C oracle includes {inc}"


def test_package_python_does_no_method_arithmetic():
    """The Python modules of the package marshal arguments and drive the
    library: no trigonometric function (the draws, the synthesis, the xi-shift
    of training rows) and no random-number generator is called there."""
    banned = {"cos", "sin", "tan", "sincos", "arctan2", "atan2", "standard_normal", "normal", "uniform", "random"}
    # workloads.py is the seeded generator of parameter points shared with the tests
    for f in [f for f in _py_files(PKG) if os.path.basename(f) != "workloads.py"]:
        tree = ast.parse(open(f).read(), filename=f)
        for node in ast.walk(tree):
            if isinstance(node, ast.Call):
                fn = node.func
                name = fn.attr if isinstance(fn, ast.Attribute) else getattr(fn, "id", "")
                assert name not in banned, f"{os.path.basename(f)}:{node.lineno} calls {name}"


def test_bench_calls_the_oracle_only_for_the_cpu_baseline():
    path = os.path.join(ROOT, "bench.py")
    tree = ast.parse(open(path).read(), filename=path)
    seen = []

    def visit(node, func):
        if isinstance(node, (ast.FunctionDef, ast.AsyncFunctionDef)):
            func = node.name
        if isinstance(node, ast.Import) and any(a.name.split(".")[0] == "oracle" for a in node.names):
            seen.append(func)
        if isinstance(node, ast.ImportFrom) and node.module and node.module.split(".")[0] == "oracle":
            seen.append(func)
        for child in ast.iter_child_nodes(node):
            visit(child, func)

    visit(tree, None)
    assert seen, "bench.py is expected to time the oracle as its CPU baseline"
    for func in seen:
        assert func is not None and func.startswith("cpu_baseline"), f"oracle imported in {func}"


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    from paper_2411_16952_amd import tkdv as T
    monkeypatch.setattr(T, "LIB_PATH", str(tmp_path / "libtkdv.so"))
    with pytest.raises(ImportError, match="missing"):
        T._load()
