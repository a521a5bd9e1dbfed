"""Build libhecnn.so (gfx950) in-tree with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_obj")
LIB = os.path.join(HERE, "libhecnn.so")
ARCH = os.environ.get("HECNN_ARCH", "gfx950")

# Packed FP32 instructions stay off: none of this code needs them.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Wall", "-Wno-unused-function", "-Wno-unused-result"]
# host-only sources: no contraction of floating-point expressions (double-double arithmetic)
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-D__HIP_PLATFORM_AMD__",
             "-I/opt/rocm/include"]

SOURCES = [
    ("hec_kernels.hip", "hip"),
    ("hec_ctx.hip", "hip"),
    ("hec_encode.hip", "hip"),
    ("hec_layers.cpp", "cxx"),
    ("hec_poly.cpp", "cxx"),
    ("hec_block.cpp", "cxx"),
    ("hec_batch.cpp", "cxx"),
    ("hec_server.cpp", "cxx"),
    ("hec_tune.cpp", "cxx"),
    ("hec_host.cpp", "cxx"),
]


def _compile(src, kind):
    os.makedirs(OBJ, exist_ok=True)
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    path = os.path.join(CSRC, src)
    if kind == "hip":
        cmd = ["/opt/rocm/bin/hipcc", "-c", path, "-o", out] + HIP_FLAGS
    else:
        cmd = ["/opt/rocm/bin/hipcc", "-x", "c++", "-c", path, "-o", out] + CXX_FLAGS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return out


def build():
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(lambda s: _compile(*s), SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["/opt/rocm/bin/hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
    sys.exit(0)
