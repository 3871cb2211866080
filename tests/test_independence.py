"""CPU checks of the separation between the product path and the oracle: the package
never imports the oracle, the oracle never includes or imports the package, the input
generators import neither, only the benchmark's CPU-baseline leg touches the oracle, and
the binding raises when the HIP library is missing (no CPU fallback)."""

import ast
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _files(sub, exts):
    d = os.path.join(ROOT, sub)
    return [os.path.join(d, f) for f in sorted(os.listdir(d)) if f.endswith(exts)]


def _py_imports(path):
    tree = ast.parse(open(path).read())
    out = []
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out += [a.name for a in node.names]
        elif isinstance(node, ast.ImportFrom):
            out.append(("." * node.level) + (node.module or ""))
    return out


def test_package_does_not_import_the_oracle():
    pkg = "paper_2406_03726_amd"
    for path in _files(pkg, (".py",)):
        for mod in _py_imports(path):
            assert not mod.split(".")[0] == "oracle", (path, mod)
    for path in _files(os.path.join(pkg, "csrc"), (".hip", ".h")):
        for inc in re.findall(r'#include\s*[<"]([^>"]+)[>"]', open(path).read()):
            assert "oracle" not in inc, (path, inc)


def test_oracle_does_not_use_the_package():
    for path in _files("oracle", (".py",)):
        for mod in _py_imports(path):
            assert mod.split(".")[0] not in ("paper_2406_03726_amd", "gee_workloads"), (path, mod)
    for path in _files("oracle", (".c", ".h")):
        for inc in re.findall(r'#include\s*[<"]([^>"]+)[>"]', open(path).read()):
            assert inc.startswith(("std", "math", "string")) or inc in ("stdint.h", "stddef.h", "stdlib.h"), (path, inc)


def test_generators_import_neither():
    for path in _files("gee_workloads", (".py",)):
        for mod in _py_imports(path):
            assert mod.split(".")[0] not in ("oracle", "paper_2406_03726_amd"), (path, mod)


def test_bench_uses_the_oracle_only_for_the_cpu_baseline():
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    for fn in [n for n in tree.body if isinstance(n, ast.FunctionDef)]:
        for node in ast.walk(fn):
            if isinstance(node, (ast.Import, ast.ImportFrom)):
                names = [a.name for a in node.names] if isinstance(node, ast.Import) else [node.module or ""]
                if any(n.split(".")[0] == "oracle" for n in names):
                    assert fn.name in ("cpu_baseline", "scipy_baseline"), fn.name  # the CPU-baseline leg
    top = [n for n in tree.body if isinstance(n, (ast.Import, ast.ImportFrom))]
    for node in top:
        names = [a.name for a in node.names] if isinstance(node, ast.Import) else [node.module or ""]
        assert not any(n.split(".")[0] == "oracle" for n in names)


def test_binding_raises_without_the_library(monkeypatch):
    from paper_2406_03726_amd import _lib

    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB", os.path.join(ROOT, "no_such_dir", "libgee.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.load()
