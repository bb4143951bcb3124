"""The C-ABI library loads and exports every symbol include/pdfs.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdfs.h")
LIB = os.path.join(ROOT, "paper_2603_16721_amd", "libpdfs.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdfs_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("pdfs_create", "pdfs_best_combo", "pdfs_wsc_run", "pdfs_destroy",
              "pdfs_strerror", "pdfs_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build first: python __graft_entry__.py"
    L = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (pdfs_\w+)", out))
    assert set(declared()) <= exported


def test_strerror_without_gpu():
    L = ctypes.CDLL(LIB)
    L.pdfs_strerror.restype = ctypes.c_char_p
    assert L.pdfs_strerror(0) == b"ok"
    assert b"invalid" in L.pdfs_strerror(-1)


def test_binding_names_match_abi():
    from paper_2603_16721_amd import pdfs
    for n in declared():
        assert n in pdfs.EXPORTS


def test_binding_layout_matches_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field
    offsets, and every PDFS_* constant the binding defines has the header's
    value (a C program compiled against include/pdfs.h prints them)."""
    import ctypes as ct
    from paper_2603_16721_amd import pdfs
    structs = {n: getattr(pdfs, n) for n in dir(pdfs)
               if isinstance(getattr(pdfs, n), type) and issubclass(getattr(pdfs, n), ct.Structure)
               and n.startswith("pdfs_")}
    assert set(structs) >= {"pdfs_matrix", "pdfs_options", "pdfs_combo", "pdfs_stats"}
    consts = {n: getattr(pdfs, n) for n in dir(pdfs)
              if n.startswith("PDFS_") and isinstance(getattr(pdfs, n), int)}
    consts["PDFS_MAX_H"] = pdfs.MAX_H
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pdfs.h"', "int main(void) {"]
    for n, cls in sorted(structs.items()):
        lines.append(f'  printf("{n} size %zu\\n", sizeof({n}));')
        for f in cls._fields_:
            lines.append(f'  printf("{n}.{f[0]} off %zu\\n", offsetof({n}, {f[0]}));')
    for n in sorted(consts):
        lines.append(f'  printf("{n} val %lld\\n", (long long)({n}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        key, kind, v = line.rsplit(" ", 2)
        got[(key, kind)] = int(v)
    for n, cls in structs.items():
        assert got[(n, "size")] == ct.sizeof(cls), n
        for f in cls._fields_:
            assert got[(f"{n}.{f[0]}", "off")] == getattr(cls, f[0]).offset, (n, f[0])
    for n, v in consts.items():
        assert got[(n, "val")] == v, n


def test_batch_path_flags_exclude_each_other_without_gpu():
    """Asking for both batch paths is rejected before any device call; the
    binding rejects unknown path names."""
    import numpy as np
    import pytest
    from paper_2603_16721_amd import pdfs
    T = np.ones((3, 1), dtype=np.uint64)
    N = np.ones((3, 1), dtype=np.uint64)
    m, keep = pdfs._matrix_arg(T, N, 1, 1)
    arr = (pdfs.pdfs_matrix * 1)(m)
    opt = pdfs.pdfs_options(prune_mode=pdfs.PRUNE_MODES["empty"], device=0, stream=None,
                            flags=pdfs.PDFS_OPT_BATCH_STREAMS | pdfs.PDFS_OPT_BATCH_ONE_LAUNCH)
    out = ctypes.c_void_p()
    rc = pdfs.lib.pdfs_batch_create(arr, 1, ctypes.byref(opt), ctypes.byref(out))
    assert rc == pdfs.PDFS_ERR_INVALID_ARG and not out.value
    assert b"exclude each other" in pdfs.lib.pdfs_batch_last_error(None)
    with pytest.raises(ValueError):
        pdfs.pdfs_batch_create([(T, N, 1, 1)], "empty", path="one-launch")
    del keep
