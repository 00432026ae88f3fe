"""Build libfftc.so (HIP, gfx950) in-tree with hipcc: the translation units compile in
parallel to objects under _build/, then link into one shared library."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
UNITS = ("fftc_dtt64.hip", "fftc_dtt32.hip", "fftc_residual.hip", "fftc_kernels.hip", "fftc_api.hip",
         "fftc_nn.hip")
OUT = os.path.join(HERE, "libfftc.so")
OBJDIR = os.path.join(HERE, "_build")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _compile(src, obj, verbose):
    cmd = ["hipcc"] + FLAGS + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.run(cmd, capture_output=True, text=True)


def _stale(src, obj):
    """True when the object is missing or older than its source or any header of csrc/."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(HERE, "csrc", f) for f in os.listdir(os.path.join(HERE, "csrc"))
                    if f.endswith(".h")] + [os.path.join(HERE, "..", "include", f)
                                           for f in os.listdir(os.path.join(HERE, "..", "include"))]
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose=False, incremental=False):
    """Compile every unit (incremental=True: only units older than their sources) and link."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [os.path.join(HERE, "csrc", f) for f in UNITS if os.path.exists(os.path.join(HERE, "csrc", f))]
    objs = [os.path.join(OBJDIR, os.path.basename(s).replace(".hip", ".o")) for s in srcs]
    todo = [(s, o) for s, o in zip(srcs, objs) if not incremental or _stale(s, o)]
    results = []
    if todo:
        with ThreadPoolExecutor(max_workers=len(todo)) as ex:
            results = list(ex.map(lambda so: _compile(so[0], so[1], verbose), todo))
    for r in results:
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed building libfftc.so")
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libfftc.so")
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True, incremental="-i" in sys.argv))
