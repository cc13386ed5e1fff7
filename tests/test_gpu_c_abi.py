"""The C ABI from C: tests/c_abi_caller.c, built by the repository's build step, creates a table,
validates four queries and runs a guarded copy through libagile_guard.so with no Python
involved, and checks every result itself."""
import os
import subprocess

import pytest

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu
EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_build", "c_abi_caller")


def test_c_caller():
    need_gpu()
    if not os.path.exists(EXE):
        pytest.skip("tests/_build/c_abi_caller is not built: __graft_entry__.build() builds it")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("c abi ok"), r.stdout + r.stderr
