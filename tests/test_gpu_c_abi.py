"""The C ABI from plain C.

tests/c_abi_cg.c is built with gcc against include/mfe.h and the in-tree
libmfe.so and run as a process of its own: a context on the null stream with
the library's own allocator, the paper's 20^3 problem solved by FP64 CG in
both formats, the true residual recomputed on the host, the sizes against
their closed forms and three refused calls (its header lists the checks).
"""
import os
import subprocess
import tempfile

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_c_program_solves_through_the_c_abi():
    lib = os.path.join(ROOT, "paper_1505_08023_amd")
    if not os.path.exists(os.path.join(lib, "libmfe.so")):
        pytest.fail("libmfe.so is not built")
    src = os.path.join(ROOT, "tests", "c_abi_cg.c")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "c_abi_cg")
        cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", src, "-o",
               exe, f"-L{lib}", "-lmfe", f"-L{ROCM}/lib", "-lamdhip64", "-lm", f"-Wl,-rpath,{lib}",
               f"-Wl,-rpath,{ROCM}/lib"]
        b = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
        assert b.returncode == 0, b.stderr
        print("running the C program", flush=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        print(r.stdout, r.stderr)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "all checks passed" in r.stdout
        assert r.stdout.count("iterations") == 2
