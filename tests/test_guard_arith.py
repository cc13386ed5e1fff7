"""CPU check of the HIP guard's allow decisions (no GPU needed): compiles the kernels'
host-compilable guard arithmetic with g++ and runs randomized exact-bounds properties."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_guard_arithmetic_properties(tmp_path):
    exe = tmp_path / "guard_arith_check"
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(HERE, "guard_arith_check.cpp"),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
