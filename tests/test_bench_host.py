"""The benchmark's contract on the CPU: one GPU only (a request for more
exits with a message), and every committed profile summary carries the
machine-readable record bench.py reads its traffic figure from."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_profile_summaries_are_machine_readable():
    sys.path.insert(0, ROOT)
    import bench
    for workload, (path, sources) in bench.PROFILES.items():
        text = open(os.path.join(ROOT, path)).read()
        lines = [l for l in text.splitlines() if l.startswith("machine-readable:")]
        assert len(lines) == 1, path
        rec = json.loads(lines[0].split(":", 1)[1])
        for key in ("kernel", "avg_ms", "traffic_bytes", "fetch_scale", "write_scale",
                    "source_sha"):
            assert key in rec, (path, key)
        assert rec["traffic_bytes"] > 0 and rec["avg_ms"] > 0
        assert "rocprofv3" in text and "--kernel-trace --stats" in text, path
        for f in sources + bench.COMMON_SOURCES:
            assert os.path.exists(os.path.join(ROOT, f)), f
        # the figure bench.py reports is the summary's, or None once the
        # kernel's sources changed since the counters were taken
        got = bench.profile_traffic(workload)
        assert got in (None, rec["traffic_bytes"])


def test_percentile():
    sys.path.insert(0, ROOT)
    import bench
    xs = list(range(1, 101))
    assert bench.percentile(xs, 50) in (50, 50.5, 51)
    assert bench.percentile(xs, 99) >= 99


def test_workload_legs_name_only_what_they_define():
    """Every workload leg reads only names it has: a leg that hands its line
    back as a sub-object takes `sub`, the others print it.  (Run on the GPU
    a leg that names an undefined variable fails only after its work.)"""
    import ast
    import builtins
    tree = ast.parse(open(os.path.join(ROOT, "bench.py")).read())
    module_names = {n.name for n in tree.body if isinstance(n, (ast.FunctionDef, ast.ClassDef))}
    for n in tree.body:
        if isinstance(n, ast.Assign):
            module_names |= {t.id for tg in n.targets for t in ast.walk(tg)
                             if isinstance(t, ast.Name)}
        elif isinstance(n, (ast.Import, ast.ImportFrom)):
            module_names |= {(a.asname or a.name).split(".")[0] for a in n.names}
    for f in tree.body:
        if not (isinstance(f, ast.FunctionDef) and f.name.startswith("run_")):
            continue
        known = set(module_names) | set(dir(builtins))
        for node in ast.walk(f):
            if isinstance(node, (ast.FunctionDef, ast.Lambda)):
                a = node.args
                known |= {x.arg for x in a.args + a.kwonlyargs}
                if a.vararg:
                    known.add(a.vararg.arg)
                if a.kwarg:
                    known.add(a.kwarg.arg)
            if isinstance(node, ast.FunctionDef):
                known.add(node.name)
            elif isinstance(node, ast.Name) and isinstance(node.ctx, ast.Store):
                known.add(node.id)
            elif isinstance(node, (ast.Import, ast.ImportFrom)):
                known |= {(x.asname or x.name).split(".")[0] for x in node.names}
            elif isinstance(node, ast.ExceptHandler) and node.name:
                known.add(node.name)
        used = {n.id for n in ast.walk(f) if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load)}
        assert not used - known, (f.name, sorted(used - known))
