"""The C ABI from plain C: `tests/c/ns_abi_demo.c` includes `include/ns.h`
as C11 with every warning an error and links against `libns.so` (CPU), then
runs a Gaussian problem to termination through the ABI alone and checks its
evidence against the closed form and its per-iteration records and counts
against one another (GPU)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2509_24949_amd")
SRC = os.path.join(ROOT, "tests", "c", "ns_abi_demo.c")


def _build(out_dir):
    cc = shutil.which("cc") or shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    if not os.path.exists(os.path.join(PKG, "libns.so")):
        pytest.fail("libns.so is not built (python -m paper_2509_24949_amd.build)")
    exe = os.path.join(out_dir, "ns_abi_demo")
    subprocess.run([cc, "-std=c11", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
                    SRC, "-L", PKG, "-lns", "-lm", f"-Wl,-rpath,{PKG}", "-o", exe], check=True)
    return exe


def test_header_compiles_as_c_and_links():
    with tempfile.TemporaryDirectory() as d:
        assert os.path.exists(_build(d))


@pytest.mark.gpu
def test_c_caller_runs_a_gaussian_problem():
    with tempfile.TemporaryDirectory() as d:
        exe = _build(d)
        print("running the C caller", flush=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        print(r.stdout, r.stderr, flush=True)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "ok" in r.stdout
