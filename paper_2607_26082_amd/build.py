"""Build libfftc.so (HIP, gfx950) in-tree with hipcc: the translation units compile in
parallel to objects under _build/, then link into one shared library.

build_sanitized() builds the same sources into _build/hostsan/libfftc_hostsan.so with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code only (-Xarch_host before each -fsanitize; the
device code is the same as in libfftc.so).  It is loaded in place of libfftc.so when FFTC_LIB
names it, in a process started with the ASan runtime preloaded
(tests/test_host_sanitizers.py)."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
UNITS = ("fftc_dtt64.hip", "fftc_dtt32.hip", "fftc_residual.hip", "fftc_kernels.hip", "fftc_api.hip",
         "fftc_nn.hip")
OUT = os.path.join(HERE, "libfftc.so")
OBJDIR = os.path.join(HERE, "_build")
SAN_OBJDIR = os.path.join(HERE, "_build", "hostsan")
SAN_OUT = os.path.join(SAN_OBJDIR, "libfftc_hostsan.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g1"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _compile(src, obj, verbose, extra=()):
    cmd = ["hipcc"] + FLAGS + list(extra) + ["-c", src, "-o", obj]
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


def _build(out, objdir, extra, verbose, incremental):
    os.makedirs(objdir, exist_ok=True)
    srcs = [os.path.join(HERE, "csrc", f) for f in UNITS if os.path.exists(os.path.join(HERE, "csrc", f))]
    objs = [os.path.join(objdir, os.path.basename(s).replace(".hip", ".o")) for s in srcs]
    todo = [(s, o) for s, o in zip(srcs, objs) if not incremental or _stale(s, o)]
    results = []
    if todo:
        with ThreadPoolExecutor(max_workers=len(todo)) as ex:
            results = list(ex.map(lambda so: _compile(so[0], so[1], verbose, extra), todo))
    for r in results:
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC"] + list(extra) + objs + ["-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed linking {os.path.basename(out)}")
    os.replace(out + ".tmp", out)
    return out


def build(verbose=False, incremental=False):
    """Compile every unit (incremental=True: only units older than their sources) and link."""
    return _build(OUT, OBJDIR, (), verbose, incremental)


def build_sanitized(verbose=False, incremental=False):
    """The host-sanitized variant of the library (see the module docstring)."""
    return _build(SAN_OUT, SAN_OBJDIR, SAN_FLAGS, verbose, incremental)


if __name__ == "__main__":
    if "--hostsan" in sys.argv:
        print(build_sanitized(verbose=True, incremental="-i" in sys.argv))
    else:
        print(build(verbose=True, incremental="-i" in sys.argv))
