"""The Python example of the README runs as written and gives finite
gradients."""
import os
import re

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_readme_python_example_runs():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    text = open(os.path.join(os.path.dirname(__file__), "..", "README.md")).read()
    block = re.search(r"## Python API in brief\s+```python\n(.*?)```", text, re.S).group(1)
    ns = {}
    exec(compile(block, "README.md", "exec"), ns)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(ns["y0"].grad).all()) and bool(torch.isfinite(ns["theta"].grad).all())
    assert bool((ns["fast"].status == 0).all())
    assert torch.equal(ns["fast"].y_final, ns["sol"].y_final)
