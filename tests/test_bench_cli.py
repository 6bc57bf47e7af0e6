"""bench.py on the CPU: every name it uses is bound (a missing constant would
only show on a GPU run), and a request for more than one GPU is refused
before anything touches a device."""
import ast
import builtins
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def _unbound_names(src: str) -> set:
    tree = ast.parse(src)
    bound = set(dir(builtins)) | {"__file__", "__name__"}
    for node in ast.walk(tree):
        if isinstance(node, (ast.FunctionDef, ast.AsyncFunctionDef, ast.ClassDef)):
            bound.add(node.name)
        elif isinstance(node, ast.Name) and isinstance(node.ctx, (ast.Store, ast.Del)):
            bound.add(node.id)
        elif isinstance(node, ast.arg):
            bound.add(node.arg)
        elif isinstance(node, (ast.Import, ast.ImportFrom)):
            for a in node.names:
                bound.add((a.asname or a.name).split(".")[0])
        elif isinstance(node, ast.ExceptHandler) and node.name:
            bound.add(node.name)
    used = {n.id for n in ast.walk(tree) if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load)}
    return used - bound


def test_bench_uses_no_unbound_name():
    with open(BENCH) as fh:
        assert _unbound_names(fh.read()) == set()


def test_unbound_name_check_finds_a_missing_constant():
    assert _unbound_names("def f():\n    return MISSING + 1\n") == {"MISSING"}


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], cwd=ROOT, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profile_hash_ignores_comments_only():
    """A profile stays current when a comment of its sources changes, not when
    their code does (strings keep their slashes)."""
    sys.path.insert(0, ROOT)
    import bench
    a = 'int f(int x) { return x + 1; } // one\n/* two */ const char* s = "a//b";\n'
    b = 'int f(int x)  {\n  return x + 1;  // another comment\n}\nconst char* s = "a//b";'
    c = 'int f(int x) { return x + 2; } // one\n/* two */ const char* s = "a//b";\n'
    d = 'int f(int x) { return x + 1; } // one\n/* two */ const char* s = "a/b";\n'
    assert bench.source_code(a) == bench.source_code(b)
    assert bench.source_code(a) != bench.source_code(c)
    assert bench.source_code(a) != bench.source_code(d)
