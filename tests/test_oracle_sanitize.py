"""Host sanitizers on the oracle: `tests/c/orc_sanitize.c` and
`oracle/nsorc.c` built with gcc under AddressSanitizer and
UndefinedBehaviorSanitizer (leak checking on, undefined behaviour fatal)
drive every oracle entry point the tests use on small problems; any
out-of-bounds access, use after free, leak or undefined operation aborts
the program.  CPU only."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "orc_sanitize")
        flags = ["-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                 "-fno-sanitize-recover=undefined", "-fopenmp"]
        build = subprocess.run([gcc, *flags, "-I", os.path.join(ROOT, "oracle"),
                                os.path.join(ROOT, "tests", "c", "orc_sanitize.c"),
                                os.path.join(ROOT, "oracle", "nsorc.c"), "-lm", "-o", exe],
                               capture_output=True, text=True)
        if build.returncode != 0 and "sanitize" in build.stderr:
            pytest.skip("the sanitizer runtimes are not installed: " + build.stderr[-300:])
        assert build.returncode == 0, build.stderr
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0 and "orc_sanitize: ok" in r.stdout, r.stdout + r.stderr
