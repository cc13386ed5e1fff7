"""Build tests/c_abi_caller.c (a C program that calls libagile_guard.so without Python) into
tests/_build/c_abi_caller. Called by the repository's build step, on the CPU; the GPU test only
runs the result."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "_build", "c_abi_caller")


def build() -> str:
    from paper_2606_06697_amd import _build
    pkg = os.path.dirname(_build.LIB_PATH)
    tlib = _build.torch_lib_dir()
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(HERE, "c_abi_caller.c"), "-o", OUT,
           pkg + "/" + os.path.basename(_build.LIB_PATH), f"-L{tlib}", "-lamdhip64",
           f"-Wl,-rpath,{pkg}", f"-Wl,-rpath,{tlib}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("c_abi_caller build failed:\n" + r.stderr)
    return OUT
