"""The oracle and the HIP path share no code (no GPU needed).

Parsed, not executed:
* nothing in the package imports the oracle, and the oracle imports neither
  the package nor the input generators' neighbours beyond its own modules;
* the input generators (`synth/`) import neither side;
* no C, C++ or HIP source includes anything from `oracle/`;
* `bench.py` and `__graft_entry__.py` import the oracle only inside the
  CPU-baseline leg and the smoke check.
"""
import ast
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _py(folder):
    d = os.path.join(ROOT, folder)
    return [os.path.join(d, f) for f in sorted(os.listdir(d)) if f.endswith(".py")]


def _imports(path):
    """(module, enclosing function or None) for every import in the file."""
    tree = ast.parse(open(path).read(), path)
    out = []

    def visit(node, fn):
        for child in ast.iter_child_nodes(node):
            f = child.name if isinstance(child, (ast.FunctionDef, ast.AsyncFunctionDef)) else fn
            if isinstance(child, ast.Import):
                out.extend((a.name, fn) for a in child.names)
            elif isinstance(child, ast.ImportFrom):
                out.append(("." * child.level + (child.module or ""), fn))
            visit(child, f)
    visit(tree, None)
    return out


def _top(mod):
    return mod.lstrip(".").split(".")[0] if not mod.startswith(".") else "."


def test_package_never_imports_the_oracle():
    for path in _py("paper_2512_08309_amd"):
        for mod, _ in _imports(path):
            assert _top(mod) not in ("oracle",), (path, mod)


def test_oracle_imports_only_itself_and_libraries():
    for path in _py("oracle"):
        for mod, _ in _imports(path):
            assert _top(mod) not in ("paper_2512_08309_amd", "synth", "bench", "__graft_entry__"), (path, mod)


def test_input_generators_import_neither_side():
    for path in _py("synth"):
        for mod, _ in _imports(path):
            assert _top(mod) not in ("oracle", "paper_2512_08309_amd"), (path, mod)


def test_native_sources_include_nothing_from_the_oracle():
    csrc = os.path.join(ROOT, "paper_2512_08309_amd", "csrc")
    srcs = [os.path.join(csrc, f) for f in os.listdir(csrc)] + [os.path.join(ROOT, "include", "td.h")]
    for path in srcs:
        for inc in re.findall(r'#include\s*[<"]([^>"]+)[>"]', open(path).read()):
            assert "oracle" not in inc, (path, inc)


def test_entry_points_use_the_oracle_only_in_their_checker_legs():
    allowed = {"bench.py": {"cpu_baseline"}, "__graft_entry__.py": {"smoke"}}
    for name, fns in allowed.items():
        for mod, fn in _imports(os.path.join(ROOT, name)):
            if _top(mod) == "oracle":
                assert fn in fns, (name, mod, fn)
