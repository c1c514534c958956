"""The oracle and the HIP path share no code, and the product never reaches the oracle.

Checked on the sources' import statements (AST, not text search):
* nothing under oracle/ imports the product package or reads its sources;
* nothing in the product package (binding, build script) imports oracle/ or workloads/;
* the input generators (workloads/) import neither side;
* the product's native sources do not include anything from oracle/.
"""

import ast
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = "paper_1602_00412_amd"


def _py_files(folder):
    for dirpath, _, names in os.walk(os.path.join(ROOT, folder)):
        if "__pycache__" in dirpath:
            continue
        for n in names:
            if n.endswith(".py"):
                yield os.path.join(dirpath, n)


def _imported_modules(path):
    with open(path) as f:
        tree = ast.parse(f.read(), filename=path)
    mods = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            mods.update(a.name.split(".")[0] for a in node.names)
        elif isinstance(node, ast.ImportFrom) and node.level == 0 and node.module:
            mods.add(node.module.split(".")[0])
    return mods


def test_oracle_does_not_use_the_product():
    for p in _py_files("oracle"):
        mods = _imported_modules(p)
        assert PKG not in mods, p
        with open(p) as f:
            assert "libsfd" not in f.read(), p


def test_product_does_not_use_the_oracle_or_the_generators():
    for p in _py_files(PKG):
        mods = _imported_modules(p)
        assert "oracle" not in mods and "workloads" not in mods, p


def test_generators_import_neither_side():
    for p in _py_files("workloads"):
        mods = _imported_modules(p)
        assert "oracle" not in mods and PKG not in mods, p


def test_native_sources_include_nothing_from_the_oracle():
    csrc = os.path.join(ROOT, PKG, "csrc")
    for n in os.listdir(csrc):
        if n.endswith((".hip", ".cpp", ".h")):
            with open(os.path.join(csrc, n)) as f:
                for inc in re.findall(r'#include\s+"([^"]+)"', f.read()):
                    assert "oracle" not in inc, (n, inc)


def test_bench_runs_the_oracle_only_in_its_cpu_baseline_leg():
    # bench.py may run the oracle only to time it (and to check the device path against what it
    # computes): every import of oracle/ sits inside a function named cpu_baseline*
    path = os.path.join(ROOT, "bench.py")
    with open(path) as f:
        tree = ast.parse(f.read(), filename=path)

    def visit(node, owner):
        for child in ast.iter_child_nodes(node):
            name = child.name if isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)) else owner
            if isinstance(child, ast.Import):
                assert all(a.name.split(".")[0] != "oracle" for a in child.names) or \
                    (owner or "").startswith("cpu_baseline"), (owner, child.lineno)
            elif isinstance(child, ast.ImportFrom) and child.module and child.module.split(".")[0] == "oracle":
                assert (owner or "").startswith("cpu_baseline"), (owner, child.lineno)
            visit(child, name)

    visit(tree, None)
