"""Build the gfx950 shared library ``libdwf.so`` in-tree with hipcc.

Every translation unit under ``csrc/`` is compiled as HIP for gfx950 only and
linked into one shared object next to this file.  Packed FP32 instructions are
disabled (``-packed-fp32-ops``): the compiler would otherwise emit
v_pk_{add,mul,fma}_f32 from scalar float code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libdwf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-x", "hip", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    "-Werror=return-type",
    "-I" + os.path.join(ROOT, "include"),
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


# the host pass does not know the packed-FP32 target feature; that note is
# expected and harmless, every other diagnostic is shown
_KNOWN_NOTE = "packed-fp32-ops"


def _diagnostics(text: str) -> str:
    keep = [ln for ln in text.splitlines() if ln.strip() and _KNOWN_NOTE not in ln]
    return "\n".join(keep)


def _compile(src: str) -> tuple[str, str]:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj, _diagnostics(r.stdout + r.stderr)


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every source and link libdwf.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        done = list(ex.map(_compile, srcs))
    objs = [o for o, _ in done]
    for src, (_, diag) in zip(srcs, done):
        if diag:
            print(f"[hipcc] {os.path.basename(src)}:\n{diag}", file=sys.stderr, flush=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
