"""GPU: the Python example of README.md runs as written, and its results
are those of the same calls made here (the sweep, the two norms and the
download)."""

import os
import re

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _example():
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, flags=re.S)
    assert blocks, "README.md has no python example"
    return blocks[0]


def test_readme_example_runs():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    print("CASE test=readme-example", flush=True)
    ns = {}
    exec(compile(_example(), "README.md", "exec"), ns)
    prob, q, norms, l2 = ns["prob"], ns["q"], ns["norms"], ns["l2"]
    assert q.shape == prob.Q0.shape and np.all(np.isfinite(q))
    assert norms.shape == (prob.S, 4) and l2.shape[0] == prob.S
    W = ns["W"]
    sol = W.Solver.from_problem(prob)
    Q = sol.upload(prob.Q0)
    sol.integrate(Q, prob.S, prob.dt, prob.nsteps)
    assert np.array_equal(sol.download(Q, prob.S), q)
    assert np.array_equal(sol.norms(Q, None, prob.S), norms)
    assert np.array_equal(sol.l2_norms(Q, None, prob.S), l2)
