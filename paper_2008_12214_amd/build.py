"""Build step: compile the HIP sources into the in-tree shared library.

    python -m paper_2008_12214_amd.build

produces paper_2008_12214_amd/libhologen.so for gfx950 with hipcc.  Packed
FP32 instructions are disabled for all device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhologen.so")
SIZES = (64, 128, 256, 512, 1024, 2048, 4096)
SOURCES = [os.path.join(HERE, "csrc", "hg_api.hip"), os.path.join(HERE, "csrc", "hg_nn.hip"),
           os.path.join(HERE, "csrc", "hg_small.hip"), os.path.join(HERE, "csrc", "hg_search.hip")] + \
          [os.path.join(HERE, "csrc", f"hg_n{n}.hip") for n in SIZES]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-mcode-object-version=5", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]
OBJDIR = os.path.join(HERE, "_build")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    return r.returncode, err


def build(verbose=True, jobs=None):
    """Compile every translation unit (in parallel) and link the library."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    objs = [os.path.join(OBJDIR, os.path.basename(s) + ".o") for s in SOURCES]
    cmds = [[HIPCC] + FLAGS + ["-c", src, "-o", obj] for src, obj in zip(SOURCES, objs)]
    if verbose:
        print(f"[build] hipcc {' '.join(FLAGS)} -c <{len(SOURCES)} sources> ({jobs} jobs)", flush=True)
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_run, cmds))
    for (rc, err), src in zip(results, SOURCES):
        if rc != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    tmp = LIB + ".tmp"
    rc, err = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    if rc != 0:
        raise RuntimeError("link failed:\n" + err)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
