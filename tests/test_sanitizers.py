"""CPU sanitizer builds: the FP64 oracle (oracle/su3ref.c) and the library's
host-side layout code (paper_0904_1179_amd/csrc/layout.cpp) compiled with
the address and undefined-behaviour sanitizers and run on small lattices by
tests/sanitize/*.  Any report, or a failed check, fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _run(cmd, env=None, timeout=300):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env)
    return r.returncode, r.stdout + r.stderr


@pytest.mark.parametrize("what", ["oracle", "layout"])
def test_sanitizer_build_is_clean(tmp_path, what):
    cc = shutil.which("gcc" if what == "oracle" else "g++")
    if cc is None:
        pytest.skip("no host compiler")
    exe = str(tmp_path / what)
    if what == "oracle":
        cmd = [cc, "-std=c11", "-fopenmp"] + SAN + ["-o", exe, os.path.join(ROOT, "oracle", "su3ref.c"),
                                                    os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"), "-lm"]
    else:
        cmd = [cc, "-std=c++17"] + SAN + ["-I", os.path.join(ROOT, "include"), "-o", exe,
                                          os.path.join(ROOT, "paper_0904_1179_amd", "csrc", "layout.cpp"),
                                          os.path.join(ROOT, "tests", "sanitize", "layout_check.cpp")]
    rc, out = _run(cmd)
    assert rc == 0, out
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    rc, out = _run([exe], env=env)
    assert rc == 0 and "0 failures" in out and "runtime error" not in out and "ERROR:" not in out, out
