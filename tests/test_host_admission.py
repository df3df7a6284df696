"""CPU test of the serving loop's host admission logic (pool allocator and
in-order admission), compiled with the host compiler against the library's
own header; no GPU, no device code."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("sanitize", [False, True], ids=["plain", "asan-ubsan"])
def test_pool_and_admission(sanitize):
    """The second build runs the same checks under the host address and
    undefined-behaviour sanitizers (host code only)."""
    src = os.path.join(ROOT, "tests", "host", "admission_test.cpp")
    inc = os.path.join(ROOT, "paper_2309_10477_amd", "csrc")
    flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"] if sanitize else []
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "admission_test")
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", *flags, "-I", inc,
                               src, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok"
