"""Build libkfbi.so (HIP, gfx950) in-tree.

    python -m paper_2309_05965_amd.build

Every source under csrc/ is compiled by hipcc for gfx950 (packed-FP32
instruction selection disabled) and linked into paper_2309_05965_amd/libkfbi.so;
the test-data generator under gen/ into libkfbi_gen.so, which uses only the
C ABI of libkfbi.so.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build", "kfbi")
LIB = os.path.join(HERE, "libkfbi.so")
GEN = os.path.join(HERE, "gen")
GEN_LIB = os.path.join(HERE, "libkfbi_gen.so")
SOURCES = ["geometry.hip", "collocation.hip", "operator.hip", "dst.hip", "mg.hip", "gmres.hip", "learned.hip", "batch.hip", "twodensity.hip", "api.hip"]
ARCH = os.environ.get("KFBI_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-Wno-unused-result"]


def _compile(src, folder=CSRC):
    out = os.path.join(OBJ, src + ".o")
    cmd = [hipcc()] + flags() + ["-c", os.path.join(folder, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return out


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    gobj = _compile("manufactured.hip", GEN)
    tmp = GEN_LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp, gobj, "-L" + HERE, "-lkfbi",
           "-Wl,-rpath,$ORIGIN"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, GEN_LIB)
    if verbose:
        print("built", LIB, "and", GEN_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
