"""Host-side checks of bench.py's command-line contract (no GPU needed).

* every workload the command line offers resolves to a function, and so do
  the helpers its records call (a missing name would only show when the
  driver runs the bench);
* a request for more than one GPU exits with a message and status 2.
"""
import ast
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def _tree():
    return ast.parse(open(BENCH).read())


def test_every_name_bench_calls_is_defined():
    tree = _tree()
    defined = {n.name for n in tree.body if isinstance(n, ast.FunctionDef)}
    for want in ("run_c2", "run_c3", "run_c4", "run_c5", "run_fe", "run_hlu", "run_open", "run_kernels_only", "cpu_baseline_dense",
                 "cpu_baseline_transient", "roofline", "measured_traffic", "copy_ceiling_gbps", "base_record"):
        assert want in defined, want
    # every bare-name call to a lower-case module-level name resolves
    called = {n.func.id for n in ast.walk(tree) if isinstance(n, ast.Call) and isinstance(n.func, ast.Name)}
    names = {n.id for n in ast.walk(tree) if isinstance(n, ast.Name)}
    run_refs = {x for x in names if x.startswith("run_") or x.startswith("cpu_baseline")}
    import builtins as _b
    builtins = set(dir(_b))
    local = set()
    for n in ast.walk(tree):
        if isinstance(n, ast.FunctionDef):
            local.add(n.name)
        if isinstance(n, (ast.FunctionDef, ast.Lambda)):
            local |= {a.arg for a in n.args.args}
        elif isinstance(n, ast.Assign):
            for t in n.targets:
                for x in ast.walk(t):
                    if isinstance(x, ast.Name):
                        local.add(x.id)
        elif isinstance(n, (ast.Import, ast.ImportFrom)):
            local |= {(a.asname or a.name).split(".")[0] for a in n.names}
        elif isinstance(n, (ast.For, ast.comprehension)):
            for x in ast.walk(n.target):
                if isinstance(x, ast.Name):
                    local.add(x.id)
    missing = sorted((called | run_refs) - defined - local - builtins)
    assert not missing, missing


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
