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
