"""Host logic of the serving loop (CPU only): the per-client output ring of the native loop,
compiled with g++ and checked against a brute-force byte map on random alloc/free sequences
(no overlap, inside the ring, 256-byte aligned, an empty ring takes any slice that fits,
everything reclaimed)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_output_ring_against_byte_map(tmp_path):
    exe = tmp_path / "ring_check"
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(HERE, "ring_check.cpp"),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
