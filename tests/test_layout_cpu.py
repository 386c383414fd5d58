"""Static checks of where the oracle may run: the product package never imports
it, and bench.py runs it only inside its CPU-baseline leg.  Plus the bench's
one-GPU contract.  No GPU needed."""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def oracle_uses(tree):
    """(line, enclosing top-level function or None) of every import of or attribute
    access on the oracle package."""
    uses = []

    def visit(node, func):
        for child in ast.iter_child_nodes(node):
            f = func
            if isinstance(child, (ast.FunctionDef, ast.ClassDef)) and func is None:
                f = child.name
            if isinstance(child, ast.Import) and any(a.name.split(".")[0] == "oracle"
                                                     for a in child.names):
                uses.append((child.lineno, f))
            elif isinstance(child, ast.ImportFrom) and (child.module or "").split(".")[0] == "oracle":
                uses.append((child.lineno, f))
            elif isinstance(child, ast.Name) and child.id == "oracle":
                uses.append((child.lineno, f))
            visit(child, f)

    visit(tree, None)
    return uses


def test_package_never_uses_oracle():
    pkg = os.path.join(ROOT, "paper_2311_11425_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith(".py"):
                path = os.path.join(dirpath, fn)
                assert not oracle_uses(ast.parse(open(path).read())), path


def test_bench_runs_oracle_only_in_cpu_baseline_leg():
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    uses = oracle_uses(tree)
    assert uses, "the CPU baseline leg must use the oracle"
    assert {f for _, f in uses} == {"cpu_baseline_leg"}, uses


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_entry_uses_oracle_only_to_build_and_check():
    tree = ast.parse(open(os.path.join(ROOT, "__graft_entry__.py")).read())
    assert {f for _, f in oracle_uses(tree)} <= {"build", "smoke"}
