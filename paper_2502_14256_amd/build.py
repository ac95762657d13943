"""Build libldk.so (HIP, gfx950) in-tree with hipcc.

Each source compiles to a relocatable-device-code object under
``paper_2502_14256_amd/_build/`` (in parallel), then one hipcc call links
them, device code included, into ``libldk.so``."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libldk.so")
INCLUDE = os.path.join(HERE, "..", "include")
SOURCES = ["core.hip", "points.hip", "kcol.hip", "kgrad.hip", "transform.hip", "realfft.hip",
           "algebra.hip", "mll.hip", "fwht_mfma.hip", "rqmc.hip", "checked.hip", "batch.hip",
           "noalloc.hip", "bpoints.hip"]
HEADERS = ["common.hpp", "pointset.hpp", "transform.hpp", "passkit.hpp", "kfactor.hpp",
           "passbody.hpp", "batch.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ARCH = ["--offload-arch=gfx950"]
# no packed FP32 instructions anywhere in the device code
NO_PACKED = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
CFLAGS = ARCH + ["-O3", "-std=c++17", "-fPIC", "-fgpu-rdc", "-Wall", "-Wno-unused-function"] + NO_PACKED
LDFLAGS = ARCH + ["-fgpu-rdc", "--hip-link", "-shared", "-fPIC"] + NO_PACKED


def sources() -> list[str]:
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def _obj(src: str) -> str:
    return os.path.join(OBJ, os.path.basename(src) + ".o")


def _stale(src: str) -> bool:
    o = _obj(src)
    if not os.path.exists(o):
        return True
    deps = [src, os.path.join(INCLUDE, "ldk.h")] + [os.path.join(CSRC, h) for h in HEADERS
                                                    if os.path.exists(os.path.join(CSRC, h))]
    return os.path.getmtime(o) < max(os.path.getmtime(d) for d in deps)


def _compile(src: str, verbose: bool) -> None:
    cmd = [HIPCC] + CFLAGS + ["-I", INCLUDE, "-c", "-o", _obj(src) + ".tmp", src]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if out:
        print(out, file=sys.stderr, flush=True)
    if r.returncode:
        raise subprocess.CalledProcessError(r.returncode, cmd)
    os.replace(_obj(src) + ".tmp", _obj(src))


def build(verbose: bool = False, force: bool = True, jobs: int = 8) -> str:
    """Compile the HIP sources and link paper_2502_14256_amd/libldk.so.
    force=True (the default) recompiles every source; force=False only the
    ones older than a source or header."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    todo = [s for s in srcs if force or _stale(s)]
    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(todo) or 1))) as ex:
        list(ex.map(lambda s: _compile(s, verbose), todo))
    if todo or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = [HIPCC] + LDFLAGS + ["-o", tmp] + [_obj(s) for s in srcs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, force="-f" in sys.argv)
    print(LIB)
