"""Host logic of the apertures (CPU only): the address bookkeeping of one aperture, compiled
with g++ and checked against a granule map on random take/give sequences (lowest fit, inside
the aperture, granule-aligned, no overlap, maximal free ranges, everything reclaimed)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_aperture_bookkeeping_against_granule_map(tmp_path):
    exe = tmp_path / "va_check"
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(HERE, "va_check.cpp"),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
