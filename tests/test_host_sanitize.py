"""Host sanitizers on the library's host code: the host passes of the run
API and the server (`ns_api.hip`, `ns_server.hip`) are rebuilt under
AddressSanitizer and UndefinedBehaviorSanitizer (host code only; the device
code objects and the launchers' host objects come from the regular build),
linked into a copy of libns, and `tests/c/ns_host_sanitize.c` calls the
entry points with invalid arguments and ns_load with thousands of malformed
checkpoints.  Every call must be refused with NS_E_ARG before any GPU work,
so this runs on a host without a GPU.  CPU only."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2509_24949_amd")
BUILD = os.path.join(PKG, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
SANITIZED = ("ns_api", "ns_server")
PLAIN = ("ns_kernels", "ns_slice_d1", "ns_slice_d2", "ns_slice_d3", "ns_slice_m1", "ns_slice_m2", "ns_slice_m3",
         "ns_slice_p64", "ns_slice_p128", "ns_walk")


def test_host_code_under_address_and_undefined_behaviour_sanitizers():
    need = [os.path.join(BUILD, f + ".hip.hipfb") for f in SANITIZED] + \
           [os.path.join(BUILD, f + ".hip.o") for f in PLAIN]
    if not all(os.path.exists(f) for f in need) or not os.path.exists(HIPCC) or not os.path.exists(CLANG):
        pytest.skip("the library's build objects or the ROCm compilers are missing")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    with tempfile.TemporaryDirectory() as d:
        objs = []
        for f in SANITIZED:
            obj = os.path.join(d, f + ".o")
            subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-fvisibility=hidden",
                            "-I", os.path.join(ROOT, "include"), "--cuda-host-only", *san, "-Xclang",
                            "-fcuda-include-gpubinary", "-Xclang", os.path.join(BUILD, f + ".hip.hipfb"), "-c", "-o",
                            obj, os.path.join(PKG, "csrc", f + ".hip")], check=True)
            objs.append(obj)
        objs += [os.path.join(BUILD, f + ".hip.o") for f in PLAIN]
        lib = os.path.join(d, "libns.so")
        subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *san, "-o", lib, *objs,
                        "-lrocprofiler-sdk-roctx"], check=True)
        exe = os.path.join(d, "ns_host_sanitize")
        subprocess.run([CLANG, "-std=c11", "-g", "-O1", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "c", "ns_host_sanitize.c"), "-L", d, "-lns", f"-Wl,-rpath,{d}",
                        "-o", exe], check=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1",
                   HIP_VISIBLE_DEVICES="-1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0 and "ns_host_sanitize: ok" in r.stdout, r.stdout + r.stderr[-3000:]
