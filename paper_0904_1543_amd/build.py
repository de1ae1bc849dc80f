"""Build libwvl.so (hand-written HIP for gfx950) in-tree.

Steps: regenerate ``csrc/filters_gen.h`` with the library's own filter
derivation, compile every ``csrc/*.hip`` for gfx950 in parallel, link the
shared library next to this file.  Packed-FP32 instructions are disabled for
all device code.
"""

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libwvl.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _headers():
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    inc = os.path.join(ROOT, "include")
    return hs + [os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h")]


def _compile(src, incremental=False):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if all(os.path.getmtime(d) < t for d in [src] + _headers()):
            return obj, ""
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False, incremental=False):
    """Compile every source (``incremental``: only those older than their
    object file or than a header) and link libwvl.so."""
    os.makedirs(BUILD, exist_ok=True)
    gen = os.path.join(CSRC, "filters_gen.h")
    tmp_gen = gen + ".new"
    subprocess.run([sys.executable, os.path.join(CSRC, "gen_filters.py"), tmp_gen], check=True)
    if os.path.exists(gen) and open(gen).read() == open(tmp_gen).read():
        os.remove(tmp_gen)      # unchanged: keep the old time stamp
    else:
        os.replace(tmp_gen, gen)
    srcs = sources()
    workers = max(1, min(16, os.cpu_count() or 1, len(srcs)))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(lambda s: _compile(s, incremental), srcs))
    if verbose:
        for obj, err in results:
            if err.strip():
                print(err)
    objs = [o for o, _ in results]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
