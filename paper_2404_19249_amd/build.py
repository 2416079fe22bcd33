"""Build the HIP library libks.so in-tree for gfx950 with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIBDIR = os.path.join(HERE, "_lib")
SOURCES = ["ks_api.hip", "assemble.hip", "fields.hip", "spmm_cg.hip", "dense.hip", "adjoint.hip", "batch.hip", "multigrid.hip", "nonnested.hip", "eig_noalloc.hip", "probe.hip", "metric.hip", "pulay.hip"]
ARCH = os.environ.get("KS_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


def lib_path():
    return os.path.join(LIBDIR, "libks.so")


def build(verbose=False, jobs=None):
    os.makedirs(LIBDIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(LIBDIR, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([hipcc, "-c", "-x", "hip", os.path.join(CSRC, src), "-o", obj] + FLAGS)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {cmd[3]}:\n{r.stderr[-4000:]}")
        return r.stderr

    with ThreadPoolExecutor(max_workers=jobs or min(8, len(cmds))) as ex:
        for err in ex.map(run, cmds):
            if verbose and err.strip():
                print(err[-2000:])
    tmp = lib_path() + ".tmp"
    link = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-4000:])
    os.replace(tmp, lib_path())
    for o in objs:
        os.remove(o)
    return lib_path()


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
