"""The FP64 oracles under AddressSanitizer and UndefinedBehaviorSanitizer.

Both C sources (the s-step solvers and the network's convolution loops) are
compiled for the host with -fsanitize=address,undefined into temporary
libraries, and the oracle pin files run against those builds in a child
process (the sanitizer runtime preloaded, any report fatal).  An out-of-bounds
access, a use after free, a signed overflow or a misaligned load anywhere the
pins reach fails this test.  CPU only."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_pins.py", "tests/test_ilu0_oracle.py",
             "tests/test_newton_basis_oracle.py", "tests/test_omin_mgs_oracle.py",
             "tests/test_paper_problem.py", "tests/test_cnn_oracle.py"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="no AddressSanitizer runtime")
def test_oracle_pins_pass_under_asan_and_ubsan():
    flags = ["-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
             "-fno-fast-math", "-fPIC", "-shared", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-Wno-unknown-pragmas"]
    with tempfile.TemporaryDirectory() as tmp:
        libs = {}
        for key, src in (("SSTEP_ORACLE_LIB", "sstep_oracle.c"),
                         ("SSTEP_CNN_ORACLE_LIB", "cnn_oracle.c")):
            out = os.path.join(tmp, src.replace(".c", "_asan.so"))
            subprocess.run(["gcc", *flags, "-o", out, os.path.join(ROOT, "oracle", src), "-lm"],
                           check=True)
            libs[key] = out
        env = dict(os.environ, **libs,
                   LD_PRELOAD=_runtime("libasan.so"),
                   # the interpreter itself leaks by design; report everything else
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                            "-m", "not gpu", *PIN_FILES], cwd=ROOT, env=env,
                           capture_output=True, text=True, timeout=1500)
        tail = (r.stdout + r.stderr)[-4000:]
        assert r.returncode == 0, tail
        assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
        assert " passed" in r.stdout, tail
