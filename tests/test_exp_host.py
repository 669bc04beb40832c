"""CPU check of the kernels' FP64 exponential (csrc/hrlb_math.h, compiled into the kernels as is): a
small C++ program measures its error against the long-double exponential on a million seeded
samples over [-700, 700], near zero and around the reduction's half-way points, and checks exp(0),
overflow, underflow and NaN."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_exponential_within_one_ulp(tmp_path):
    exe = tmp_path / "exp_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "paper_1810_07803_amd", "csrc"),
                    os.path.join(ROOT, "tests", "exp_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
