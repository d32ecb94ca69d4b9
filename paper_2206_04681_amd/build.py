"""Compiles libfourier_llf.so for gfx950 with hipcc (in-tree, next to this file).

Usage: ``python -m paper_2206_04681_amd.build`` or ``build()`` from Python.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfourier_llf.so")
ARCH = "gfx950"

SOURCES = ["fllf_host.cpp", "fllf_server.cpp", "fllf_batch.hip", "fllf_static.hip", "fllf_boostmap.hip", "fllf_kernels_f32.hip",
           "fllf_kernels_f16.hip", "fllf_kernels_bf16.hip"]

# Packed FP32 instructions are disabled for all device code on this target.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

# The compiler's per-kernel resource report (registers, scratch, spills,
# occupancy), kept as a table next to the objects: tests check that the kernels
# of the measured passes use no scratch memory.
RESOURCE_TABLE = os.path.join(HERE, "_build", "kernel_resources.tsv")
RESOURCE_KEYS = ["VGPRs", "AGPRs", "ScratchSize [bytes/lane]", "Occupancy [waves/SIMD]", "VGPRs Spill",
                 "LDS Size [bytes/block]"]
_REMARK = re.compile(r"remark:\s+(Function Name|[A-Za-z][A-Za-z /\[\]]*?): (\S+) \[-Rpass-analysis")


def _resources(stderr: str) -> dict:
    """Kernel name -> {key: value} from the kernel-resource-usage remarks."""
    table, cur = {}, None
    for line in stderr.splitlines():
        m = _REMARK.search(line)
        if not m:
            continue
        key, val = m.group(1).strip(), m.group(2)
        if key == "Function Name":
            cur = table.setdefault(val, {})
        elif cur is not None and key in RESOURCE_KEYS:
            cur[key] = val
    return table


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(cc: str, src: str, obj: str, verbose: bool) -> dict:
    cmd = [cc, "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
           "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
           "-Rpass-analysis=kernel-resource-usage",
           "-x", "hip"] + DEVICE_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise subprocess.CalledProcessError(r.returncode, cmd)
    # compiler warnings still reach the terminal (the host pass's note that it
    # does not know the packed-FP32 feature is expected and left out)
    for line in r.stderr.splitlines():
        if "warning:" in line and "packed-fp32-ops" not in line:
            sys.stderr.write(line + "\n")
    return _resources(r.stderr)


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) into the shared library; returns its path."""
    tmpdir = os.path.join(HERE, "_build")
    os.makedirs(tmpdir, exist_ok=True)
    cc = hipcc()
    objs = [os.path.join(tmpdir, s + ".o") for s in SOURCES]
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    table = {}
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_compile, cc, s, o, verbose) for s, o in zip(SOURCES, objs)]:
            table.update(f.result())
    with open(RESOURCE_TABLE, "w") as fh:
        fh.write("\t".join(["kernel"] + RESOURCE_KEYS) + "\n")
        for name in sorted(table):
            fh.write("\t".join([name] + [table[name].get(k, "") for k in RESOURCE_KEYS]) + "\n")
    tmp_lib = LIB + ".tmp"
    link = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp_lib] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp_lib, LIB)
    build_c_client(cc, verbose)
    return LIB


# A host program that calls the library through its C interface only (tests).
C_CLIENT_SRC = os.path.join(ROOT, "tests", "c_client.cpp")
C_CLIENT = os.path.join(ROOT, "tests", "c_client")


def build_c_client(cc: str, verbose: bool = False) -> str:
    tmp = C_CLIENT + ".tmp"
    cmd = [cc, "-std=c++17", "-O2", f"--offload-arch={ARCH}", "-I", INCLUDE] + DEVICE_FLAGS + [
        C_CLIENT_SRC, "-L", HERE, "-lfourier_llf", "-Wl,-rpath,$ORIGIN/../paper_2206_04681_amd", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, C_CLIENT)
    return C_CLIENT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
