"""Build libshape.so (the HIP kernels and the C ABI) in-tree for gfx950."""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libshape.so")
SOURCES = ["api.hip", "centroid.hip", "moments.hip", "fit.hip", "adjoint.hip", "queue.hip", "stars.hip", "frames.hip", "noalloc.hip"]
ARCH = os.environ.get("SHAPE_OFFLOAD_ARCH", "gfx950")


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    return path


def build(verbose=False, jobs=None, out=None, defines=()):
    objdir = os.path.join(PKG, "_build" if out is None else "_build_" + os.path.basename(out))
    os.makedirs(objdir, exist_ok=True)
    common = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
              "-Wall", "-Wno-unused-function",
              # packed FP32 instructions are not to be generated
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC] + ["-D" + d for d in defines]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = common + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd))
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        text = p.communicate()[0].decode(errors="replace")
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln]
        if lines and (verbose or p.returncode):
            print("\n".join(lines))
        if p.returncode:
            failed.append(src)
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    lib = out or LIB
    tmp = lib + ".tmp"
    link = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(link))
    subprocess.run(link, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
