"""Structural guards: the product path never reaches the oracle, and the
oracle shares no code with the HIP path."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1909_09213_amd")


def _files(top, exts):
    for dp, _, fns in os.walk(top):
        if "_build" in dp or "__pycache__" in dp:
            continue
        for fn in fns:
            if fn.endswith(exts):
                yield os.path.join(dp, fn)


def test_package_does_not_import_the_oracle():
    for path in _files(PKG, (".py", ".hip", ".cpp", ".h")):
        text = open(path).read()
        assert not re.search(r"^\s*(import|from)\s+oracle\b", text, re.M), path
        assert "oracle/" not in text and "liboracle" not in text, path


def test_oracle_does_not_include_the_library():
    for path in _files(os.path.join(ROOT, "oracle"), (".py", ".c", ".h")):
        text = open(path).read()
        assert "cubics" not in text and "paper_1909_09213_amd" not in text, path


def test_generators_hold_no_solver():
    text = open(os.path.join(ROOT, "cspgen", "gen.c")).read()
    code = re.sub(r"/\*.*?\*/", "", text, flags=re.S)  # comments may name the method
    for word in ("propagat", "revise", "backtrack", "fixpoint"):
        assert word not in code.lower()


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: the refusal happens before anything touches a device
    import subprocess
    import sys
    for extra, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + extra,
                           capture_output=True, text=True, timeout=120,
                           env=dict(os.environ, **env), cwd=ROOT)
        assert r.returncode == 2, (extra, env, r.returncode, r.stderr[-300:])
        assert "one GPU" in r.stderr and r.stdout == ""
