"""Builds librsaprng.so (HIP kernels for gfx950 + host library) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "librsaprng.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, "-I" + INCLUDE, "-I" + CSRC,
          "-Wall", "-Wno-unused-function"]
# Kernel code: no contraction of separate multiplies and adds into fma (the
# residue arithmetic relies on each operation rounding exactly as written), IEEE
# division, and no packed-fp32 instruction selection.
DEVICE = ["-ffp-contract=off", "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops"]
SOURCES = ["k_mont_gen.hip", "k_crt_gen.hip", "k_mont_con.hip", "k_crt_con.hip", "k_crt_bat.hip", "k_vector.hip",
           "k_misc.hip", "k_primes.hip", "k_probe.hip", "noalloc.hip", "host.cpp", "server.cpp"]


def source_hash() -> str:
    """Hash of every source the library is built from (the autotuner's cache key
    carries it, so a rebuilt library never reuses another build's choice)."""
    import hashlib
    h = hashlib.sha256()
    for d in (CSRC, INCLUDE):
        for f in sorted(os.listdir(d)):
            if f.endswith((".h", ".hip", ".cpp")):
                with open(os.path.join(d, f), "rb") as fh:
                    h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC, *COMMON, *DEVICE, '-DRSAPRNG_SOURCE_HASH="%s"' % source_hash(), "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(jobs: int = 0) -> str:
    """Compile every source (always) and link librsaprng.so."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 8)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else 0))
