"""CPU checks of the repository's contracts: bench.py refuses more than one
GPU with a message and exit status 2, and the product package (Python
binding and HIP/C++ sources) never imports or includes the oracle, so no
result of the product can come from it."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("workload", ["qft", "random-mirror", "batch", "qaoa-spill"])
def test_bench_refuses_more_than_one_gpu(workload):
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2", "--workload", workload], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_product_never_uses_the_oracle():
    pkg = os.path.join(ROOT, "paper_2410_14088_amd")
    seen = 0
    for dirpath, _, files in os.walk(pkg):
        if "_build" in dirpath:
            continue
        for f in files:
            path = os.path.join(dirpath, f)
            if f.endswith(".py"):
                txt = open(path).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", txt, re.M), path
                assert "importlib" not in txt or "oracle" not in txt, path
                seen += 1
            elif f.endswith((".hip", ".cpp", ".h")):
                txt = open(path).read()
                assert not re.search(r"#\s*include\s*[<\"].*oracle", txt), path
                assert "liboracle" not in txt, path
                seen += 1
    assert seen >= 5
