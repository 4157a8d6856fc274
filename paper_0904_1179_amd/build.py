"""Build libsu3hb.so: the gfx950 HIP kernels, the C-ABI host runtime and the
job server.

hipcc cross-compiles for gfx950 without a GPU; each source is compiled in its
own process, then linked.  Packed-FP32 instructions are disabled for all
device code (-packed-fp32-ops); FP64 code is unaffected.
"""
import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsu3hb.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "api.hip", "server.hip", "layout.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=on: multiply-adds are fused only within one source expression,
# never by the backend across statements, so the rounding of a computation does
# not depend on the code around it: the one-lane, several-lanes-per-link and
# batched pass kernels round every staple and heat-bath step alike
COMPILE = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-ffp-contract=on",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I" + os.path.join(ROOT, "include")]
# layout.cpp is plain host C++ (no device code)
COMPILE_CXX = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I" + os.path.join(ROOT, "include")]


def _compile_cmd(src, obj):
    flags = COMPILE_CXX if src.endswith(".cpp") else COMPILE
    return [HIPCC] + flags + ["-c", src, "-o", obj]


def _run(cmd, tmpdir=None):
    env = dict(os.environ, TMPDIR=tmpdir) if tmpdir else None
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env)
    out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + out)
    return out


def build() -> str:
    # object files in a scratch folder inside the package (removed afterwards;
    # `_build/` is git-ignored)
    scratch = os.path.join(HERE, "_build")
    os.makedirs(scratch, exist_ok=True)
    with tempfile.TemporaryDirectory(prefix="su3hb_", dir=scratch) as tmp:
        objs = [os.path.join(tmp, os.path.basename(s) + ".o") for s in SOURCES]
        with ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
            list(pool.map(lambda c: _run(c, tmp),
                          [_compile_cmd(src, obj) for src, obj in zip(SOURCES, objs)]))
        out = LIB + ".tmp"
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out] + objs, tmp)
        os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
