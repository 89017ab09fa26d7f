"""Build libwilson_eo.so in-tree for gfx950.

HIP sources (``csrc/*.hip``) are compiled by hipcc for gfx950 with packed FP32
instructions disabled; host-only sources (``csrc/*.cpp``) by g++ against the
HIP runtime headers.  Objects go to ``_build/`` at the repository root and the
library to ``paper_2303_08609_amd/libwilson_eo.so``.  Every call recompiles.

    python -m paper_2303_08609_amd.build [--jobs N] [--debug] [--sanitize]
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libwilson_eo.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter",
             "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include"]


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature
    err = "\n".join(l for l in p.stderr.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"command failed ({p.returncode}): {' '.join(cmd)}\n{err}")
    return err


def sources():
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    return hip, cpp


def build(jobs: int | None = None, debug: bool = False, verbose: bool = False,
          defines=(), out: str | None = None) -> str:
    """Compile and link; ``defines`` are extra -D options for the HIP sources
    (launch-shape knobs), ``out`` an alternative library path."""
    os.makedirs(BUILD, exist_ok=True)
    hip, cpp = sources()
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    cmds = []
    objs = []
    tag = ("_" + "_".join(defines)) if defines else ""
    for f in hip:
        o = os.path.join(BUILD, f + tag + ".o")
        objs.append(o)
        cmds.append([hipcc] + HIPCC_FLAGS + (["-g"] if debug else []) +
                    [f"-D{d}" for d in defines] + ["-c", os.path.join(CSRC, f), "-o", o])
    for f in cpp:
        o = os.path.join(BUILD, f + tag + ".o")
        objs.append(o)
        cmds.append(["g++"] + CXX_FLAGS + (["-g"] if debug else []) +
                    ["-c", os.path.join(CSRC, f), "-o", o])
    jobs = jobs or min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(jobs) as ex:
        for err in ex.map(_run, cmds):
            if verbose and err.strip():
                print(err, file=sys.stderr)
    lib = out or LIB
    tmp = lib + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs +
         [f"-L{ROCM}/lib", "-lamdhip64"])
    os.replace(tmp, lib)
    return lib


SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                  "-g", "-O1"]


def build_sanitized(jobs: int | None = None, out: str | None = None) -> str:
    """A CPU-side checking build: the host-only sources (argument checking,
    solver drivers, workspace layout) compiled by g++ with AddressSanitizer
    and UndefinedBehaviorSanitizer, linked with the HIP objects of the last
    regular build (built first if missing; the device code is not
    instrumented).  Load it with libasan and libubsan preloaded."""
    hip, cpp = sources()
    if not all(os.path.exists(os.path.join(BUILD, f + ".o")) for f in hip):
        build(jobs)
    objs = [os.path.join(BUILD, f + ".o") for f in hip]
    cmds = []
    for f in cpp:
        o = os.path.join(BUILD, f + ".san.o")
        objs.append(o)
        cmds.append(["g++"] + CXX_FLAGS + SANITIZE_FLAGS + ["-c", os.path.join(CSRC, f), "-o", o])
    with ThreadPoolExecutor(jobs or min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(_run, cmds))
    lib = out or os.path.join(BUILD, "libwilson_eo_san.so")
    _run(["g++", "-shared", "-fPIC"] + SANITIZE_FLAGS + ["-o", lib] + objs + [f"-L{ROCM}/lib", "-lamdhip64"])
    return lib


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    ap.add_argument("-D", dest="defines", action="append", default=[],
                    help="extra preprocessor definition for the HIP sources, e.g. -D WEO_NT_LINKS=1")
    ap.add_argument("--out", default=None, help="library path (default: in the package)")
    ap.add_argument("--sanitize", action="store_true",
                    help="build _build/libwilson_eo_san.so: host sources under ASan + UBSan (CPU checks)")
    a = ap.parse_args(argv)
    if a.sanitize:
        print(build_sanitized(a.jobs, a.out))
    else:
        print(build(a.jobs, a.debug, a.verbose, tuple(a.defines), a.out))


if __name__ == "__main__":
    main()
