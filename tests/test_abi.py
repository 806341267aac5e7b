"""CPU checks of the C-ABI library: it is built for gfx950, loads, exports every
entry point that include/rbmf.h declares, and reports errors without a GPU."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2110_13115_amd import rbmf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "rbmf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:rb_status|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)))


def test_library_exists_and_loads():
    assert os.path.exists(rbmf.LIB_PATH), "run __graft_entry__.build() first"
    rbmf.lib()


def test_exports_every_declared_symbol():
    names = header_functions()
    assert set(names) == set(rbmf.FUNCTIONS), names
    L = C.CDLL(rbmf.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", rbmf.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, flags=re.M), f"{n} not exported as a text symbol"


def test_code_object_targets_gfx950():
    data = open(rbmf.LIB_PATH, "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa--(gfx\w+)", data))
    assert targets == {b"gfx950"}, targets


def test_error_paths_without_gpu():
    L = rbmf.lib()
    assert L.rb_last_error() is not None
    # NULL handles are rejected before any device work
    assert L.rb_ctx_destroy(None) == rbmf.RB_ERR_ARG
    assert L.rb_bank_free(None) == rbmf.RB_ERR_ARG
    assert L.rb_basis_free(None) == rbmf.RB_ERR_ARG
    assert b"NULL" in L.rb_last_error()
    h = C.c_void_p()
    assert L.rb_ctx_create(0, None, None) == rbmf.RB_ERR_ARG
    st = L.rb_ctx_create(0, None, C.byref(h))
    if st == rbmf.RB_OK:          # a GPU is present: nothing more to check here
        L.rb_ctx_destroy(h)
        pytest.skip("GPU present")
    assert st == rbmf.RB_ERR_DEVICE
    assert len(L.rb_last_error()) > 0
    n = C.c_int64()
    assert L.rb_filter(None, None, 0, None, None, None, None, 0, C.byref(n), None, None) == rbmf.RB_ERR_ARG
    assert L.mf_full(None, None, None, 5.0, None, 0, C.byref(n), None, None) == rbmf.RB_ERR_ARG


def test_struct_layouts_match_header(tmp_path):
    """Every field offset and struct size of the ctypes binding equals what a
    C compiler makes of include/rbmf.h."""
    structs = {"rb_trigger": rbmf.Trigger, "rb_peak": rbmf.Peak, "rb_grid": rbmf.Grid,
               "rb_filter_opts": rbmf.FilterOpts, "rb_stats": rbmf.Stats, "rb_batch_item": rbmf.BatchItem}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rbmf.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                          check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[f"{cname} size"]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got[f"{cname} {f}"]) == getattr(py, f).offset, (cname, f)
    assert rbmf.TRIGGER_NP.itemsize == C.sizeof(rbmf.Trigger) and rbmf.PEAK_NP.itemsize == C.sizeof(rbmf.Peak)
