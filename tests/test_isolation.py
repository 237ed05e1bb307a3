"""The oracle and the HIP path share no code: the package never imports the
oracle, the oracle never imports the package, the HIP sources include nothing
from the oracle, and the only places outside the tests that call the oracle
are the smoke check and the CPU-baseline legs of the benchmark."""
import ast
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2101_08453_amd")
ORACLE = os.path.join(ROOT, "oracle")


def _py_files(top):
    for d, _, files in os.walk(top):
        for f in files:
            if f.endswith(".py"):
                yield os.path.join(d, f)


def _imported_modules(tree):
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            for a in node.names:
                yield node, a.name
        elif isinstance(node, ast.ImportFrom) and node.module:
            yield node, node.module


def _top(name):
    return name.split(".")[0]


def test_package_never_imports_the_oracle():
    for path in _py_files(PKG):
        tree = ast.parse(open(path).read(), path)
        for _, mod in _imported_modules(tree):
            assert _top(mod) != "oracle", f"{path} imports {mod}"


def test_oracle_never_imports_the_package():
    for path in _py_files(ORACLE):
        tree = ast.parse(open(path).read(), path)
        for _, mod in _imported_modules(tree):
            assert _top(mod) != "paper_2101_08453_amd", f"{path} imports {mod}"


def test_hip_sources_include_nothing_from_the_oracle():
    csrc = os.path.join(PKG, "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f), errors="replace").read()
        for line in text.splitlines():
            if line.lstrip().startswith("#include"):
                assert "oracle" not in line, f"{f}: {line}"


def _functions_calling_the_oracle(path):
    """Names of the top-level functions whose bodies import the oracle; a
    module-level import of it is reported as '<module>'."""
    tree = ast.parse(open(path).read(), path)
    found = set()
    for node in tree.body:
        if isinstance(node, (ast.FunctionDef, ast.AsyncFunctionDef)):
            for _, mod in _imported_modules(node):
                if _top(mod) == "oracle":
                    found.add(node.name)
        else:
            for _, mod in _imported_modules(node):
                if _top(mod) == "oracle":
                    found.add("<module>")
    return found


def test_only_the_smoke_check_and_the_cpu_baseline_legs_call_the_oracle():
    assert _functions_calling_the_oracle(os.path.join(ROOT, "__graft_entry__.py")) <= {"smoke"}
    allowed = {"cpu_baseline", "cpu_baseline_cold_solve", "oracle_window_check"}
    assert _functions_calling_the_oracle(os.path.join(ROOT, "bench.py")) <= allowed
    # the window check runs only from inside the CPU-baseline leg
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    callers = set()
    for node in tree.body:
        if isinstance(node, ast.FunctionDef):
            for sub in ast.walk(node):
                if (isinstance(sub, ast.Call) and isinstance(sub.func, ast.Name)
                        and sub.func.id == "oracle_window_check"):
                    callers.add(node.name)
    assert callers <= {"cpu_baseline"}
