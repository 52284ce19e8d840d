"""Build libpba.so (HIP, gfx950) in the package directory with hipcc."""
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpba.so")
SOURCES = ["pba_kernels.hip", "pba_solver.hip", "pba_dense.hip", "pba_learned.hip", "pba_frontend.hip", "pba_affine.hip",
           "pba_api.cpp"]
ARCH = "gfx950"
# -packed-fp32-ops keeps the compiler from emitting packed FP32 instructions.
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wno-unused-command-line-argument"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False):
    cc = hipcc()
    tmp = tempfile.mkdtemp(prefix="pba_build_")
    try:
        procs, objs = [], []
        for s in SOURCES:
            obj = os.path.join(tmp, os.path.splitext(s)[0] + ".o")
            cmd = [cc, *FLAGS, "-c", os.path.join(CSRC, s), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
            objs.append(obj)
        errors = []
        for s, p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                errors.append(f"{s}:\n{out}")
            elif verbose and out.strip():
                print(out)
        if errors:
            raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
        tmp_lib = LIB + ".tmp"
        cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp_lib]
        out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if out.returncode != 0:
            raise RuntimeError("link failed:\n" + out.stdout)
        os.replace(tmp_lib, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
