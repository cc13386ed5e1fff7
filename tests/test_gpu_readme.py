"""The Python example in README.md runs as written, and its results are what it says."""
import os
import re

import pytest

from gpu_util import guard_mod, need_gpu

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_readme_example_runs():
    need_gpu()
    g = guard_mod()
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```python\n(.*?)```", text, re.S)
    assert blocks, "README has no python block"
    env = {}
    exec(compile(blocks[0], "README.md", "exec"), env)
    assert env["status"] in (g.AGILE_OK, g.AGILE_EFAULTED)
    assert env["Y"].shape == (1000, 64)
