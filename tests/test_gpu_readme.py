"""The Python examples of README.md run as written on the GPU and give results
with an OK status (the pseudo-inverse of the intrinsic RW1 x Besag prior with
the rank the example states)."""
import os
import re
import sys

import pytest

pytestmark = pytest.mark.gpu

README = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "README.md")


def test_readme_examples_run():
    blocks = re.findall(r"```python\n(.*?)```", open(README).read(), flags=re.S)
    assert len(blocks) == 2
    ns = {}

    def run(i):
        print(f"[gpu-readme] block {i}", flush=True)
        sys.stdout.flush()
        exec(compile(blocks[i], f"README.md block {i}", "exec"), ns)

    run(0)   # Laplace evaluations and marginal variances of the n = 3000 model
    assert all(r["info"] == 0 for r in ns["res"])
    assert list(ns["info"]) == [0] * len(ns["res"])
    run(1)   # the Moore-Penrose route on an intrinsic prior
    m = ns["m"]
    assert list(ns["info"]) == [0] and list(ns["rank"]) == [m["n"] - 51]   # "intrinsic: rank n - 51"
    assert [r["info"] for r in ns["res"]] == [0]
    assert list(ns["vinfo"]) == [0]
