"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, its struct layouts match the ctypes mirrors, and the
argument checks that precede any device work return the documented codes."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsketch.h")


def _lib():
    from paper_2105_01271_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2105_01271_amd import build
        build.build(verbose=False)
    return _lib


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dsk_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    L = _lib()
    lib = L.load()
    names = _declared()
    assert "dsk_sketch_svd" in names and "dsk_sketch_id" in names and "dsk_power_iter" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(L.EXPORTED) <= set(names)


def test_struct_layouts_match_c(tmp_path):
    L = _lib()
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "dsketch.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(dsk_restriction), sizeof(dsk_opts), sizeof(dsk_info));
  printf("%zu %zu %zu %zu\n", offsetof(dsk_restriction, index), offsetof(dsk_restriction, w2),
         offsetof(dsk_opts, tau), offsetof(dsk_opts, refine));
  printf("%zu %zu\n", offsetof(dsk_info, normA_fro2), offsetof(dsk_info, sigma_tail));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    got = list(map(int, out))
    exp = [ctypes.sizeof(L.Restriction), ctypes.sizeof(L.Opts), ctypes.sizeof(L.Info),
           L.Restriction.index.offset, L.Restriction.w2.offset, L.Opts.tau.offset, L.Opts.refine.offset,
           L.Info.normA_fro2.offset, L.Info.sigma_tail.offset]
    assert got == exp


def test_null_handle_and_status_strings():
    L = _lib()
    lib = L.load()
    assert lib.dsk_create(None, 0, None) == -1
    assert lib.dsk_sketch_svd(None, None, 0, 1, 1, 1, 1, None, 0, None, None, None, None, None) == -1
    assert lib.dsk_sketch_id(None, None, 0, 1, 1, 1, 1, None, 0, None, None, None, None, None) == -1
    assert lib.dsk_power_iter(None, None, 0, 1, 1, 1, None, 1, 0, 1.0, 1, None) == -1
    assert lib.dsk_project(None, None, 0, 1, 1, 1, None, 1, None, 0) == -1
    assert lib.dsk_status_string(0) == b"success"
    assert lib.dsk_status_string(-7) == b"argument 7 invalid"
    o = L.Opts()
    lib.dsk_opts_default(ctypes.byref(o))
    assert (o.p, o.mode, o.tau, o.refine) == (10, 0, 0.0, 0)


def test_single_hip_runtime_in_process():
    L = _lib()
    L.load()
    maps = open("/proc/self/maps").read()
    libs = set(re.findall(r"\S*libamdhip64\S*", maps))
    assert len(libs) <= 1, libs
