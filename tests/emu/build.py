"""Build the host emulation of libdsketch's kernels (CPU only, AddressSanitizer).

The HIP sources under paper_2105_01271_amd/csrc are compiled as host C++
against the shim in tests/emu/hip/hip_runtime.h (every GPU thread a fiber,
wave operations by per-group exchange, dynamic LDS a heap buffer of the
launch's size) and linked with a driver that calls the C ABI on host
buffers.  The build is cached under tests/emu/_build, keyed by a hash of all
inputs.

    python tests/emu/build.py        -> prints the driver's path
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import hashlib
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2105_01271_amd", "csrc")
OUT = os.path.join(HERE, "_build")


def _cxx() -> str | None:
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


def _inputs():
    files = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h")))
    files += [os.path.join(HERE, f) for f in ("hip/hip_runtime.h", "simt_rt.cpp", "driver.cpp", "build.py")]
    files.append(os.path.join(ROOT, "include", "dsketch.h"))
    return files


def build(verbose: bool = False) -> str:
    cxx = _cxx()
    if cxx is None:
        raise RuntimeError("no clang++ for the host emulation build")
    h = hashlib.sha256()
    for f in _inputs():
        h.update(f.encode())
        h.update(open(f, "rb").read())
    key = h.hexdigest()[:16]
    exe = os.path.join(OUT, f"driver_{key}")
    if os.path.exists(exe):
        return exe
    gen = os.path.join(OUT, "gen")
    os.makedirs(gen, exist_ok=True)
    srcs = []
    for p in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        s = open(p).read()
        # dynamic LDS: a heap buffer of exactly the launch's size
        s = re.sub(r"extern __shared__ (\w+) (\w+)\[\];", r"\1 *\2 = (\1 *)simt::dyn_lds();", s)
        # register-class optimisation barriers (empty GPU asm) have no host meaning
        s = re.sub(r'asm volatile\(""\s*:\s*"\+v"\([^;]*\)\);', ";", s)
        # LDS address-space qualifiers: host memory has one address space
        s = s.replace("__attribute__((address_space(3)))", "")
        if os.path.basename(p) in ("cpqr.hip", "rowid_reg.hip"):
            # workgroups of the one-launch factorization run together: one copy of
            # each static LDS variable per resident block
            s = re.sub(r"__shared__ ((?:unsigned )?(?:long long|\w+)) (\w+)((?:\[[^\]]+\])*);",
                       r"static \1 \2__b[64]\3; auto &\2 = \2__b[simt::block_linear()];", s)
        dst = os.path.join(gen, os.path.basename(p).replace(".hip", ".cpp"))
        open(dst, "w").write(f'#line 1 "{p}"\n' + s)
        srcs.append(dst)
    for p in glob.glob(os.path.join(CSRC, "*.h")):
        open(os.path.join(gen, os.path.basename(p)), "w").write(
            open(p).read().replace('"../../include/dsketch.h"', '"dsketch.h"'))
    srcs += [os.path.join(HERE, "simt_rt.cpp"), os.path.join(HERE, "driver.cpp")]
    flags = ["-std=c++17", "-O1", "-g", "-fsanitize=address,alignment", "-fno-sanitize-recover=alignment",
             "-fno-omit-frame-pointer", "-I", HERE, "-I", gen,
             "-I", os.path.join(ROOT, "include"), "-Wno-unused-result", "-Wno-unknown-attributes",
             "-Wno-ignored-attributes", "-w"]

    def comp(src):
        obj = os.path.join(gen, os.path.basename(src).rsplit(".", 1)[0] + ".o")
        r = subprocess.run([cxx, *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(f"host emulation build failed for {src}:\n{r.stderr[-3000:]}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(comp, srcs))
    r = subprocess.run([cxx, "-fsanitize=address,alignment", "-pthread", *objs, "-o", exe], capture_output=True,
                       text=True)
    if r.returncode:
        raise RuntimeError(f"host emulation link failed:\n{r.stderr[-3000:]}")
    for old in glob.glob(os.path.join(OUT, "driver_*")):   # earlier builds of other inputs
        if old != exe:
            os.remove(old)
    if verbose:
        print("built", exe)
    return exe


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
