"""Compile the HIP library ``libsbf.so`` (gfx950) in the package directory."""

from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsbf.so")
SOURCES = ["sbf_api.hip", "sbf_server.hip", "kernels_rolling.hip", "kernels_wide.hip", "kernels_param.hip",
           "kernels_generic.hip"]
PROBE_LIB = os.path.join(PKG, "libsbf_probe.so")
PROBE_SOURCES = ["probe_random_access.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-pthread",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]

# Per-source flags.  The lane kernels fully unroll their walk of 32, 48 or 64
# k-mers so that every per-k-mer array is indexed by constants and lives in
# registers; the larger instantiations (m = 18, whose van Herk block of 14
# needs four blocks for 48 k-mers; the 64-k-mer insert) exceed the default
# size budget of an unroll pragma, and the walk's arrays then go to scratch
# memory (a few hundred scratch accesses per k-mer step, 5-20x slower).
SOURCE_FLAGS = {"kernels_rolling.hip": ["-mllvm", "-pragma-unroll-threshold=65536"]}


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    path = os.path.join(rocm, "bin", "hipcc")
    return path if os.path.exists(path) else "hipcc"


def _run(cmd, verbose: bool, what: str) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    text = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        sys.stderr.write(text + "\n")
        raise RuntimeError("hipcc failed building %s" % what)
    if verbose and text.strip():
        print(text)


def _compile(out: str, sources, verbose: bool) -> str:
    """Compile each source to an object file (in parallel), then link the
    shared library; every step writes temporary files first."""
    from concurrent.futures import ThreadPoolExecutor

    tag = "%d" % os.getpid()
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    objs = [os.path.join(CSRC, os.path.splitext(src)[0] + ".o.tmp" + tag) for src in sources]
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]

    def one(i):
        _run([hipcc()] + flags + SOURCE_FLAGS.get(sources[i], []) + inc +
             ["-c", "-o", objs[i], os.path.join(CSRC, sources[i])], verbose, os.path.basename(out))

    try:
        workers = max(1, min(len(sources), int(os.environ.get("MAX_JOBS", "0") or 0) or (os.cpu_count() or 1)))
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(one, range(len(sources))))
        tmp = out + ".tmp" + tag
        _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs, verbose,
             os.path.basename(out))
        os.replace(tmp, out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return out


def build(verbose: bool = False) -> str:
    """Build libsbf.so (the filter) and libsbf_probe.so (roofline probes)."""
    _compile(PROBE_LIB, PROBE_SOURCES, verbose)
    return _compile(LIB, SOURCES, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
