"""ctypes loader for the plain C oracle (pdfs_oracle.c).  TEST INFRASTRUCTURE ONLY.

Follows Alg. 1 (greedy set cover) and Alg. 2 (P-DFS) of the paper; see the
header of pdfs_oracle.c for the readings adopted.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pdfs_oracle.c")
LIB = os.path.join(HERE, "libpdfs_oracle.so")
MAX_H = 9
MODES = {"none": 0, "empty": 1, "bound": 2}
TN_LITERAL = 0x100   # mode bit: TN = normals carrying none of the genes (literal T-)


def _mode(mode, tn):
    if tn not in ("all", "literal"):
        raise ValueError("tn must be 'all' or 'literal'")
    return MODES[mode] | (TN_LITERAL if tn == "literal" else 0)


def build() -> str:
    """Compile the oracle with gcc (plain C11, -O2, hardware popcount)."""
    cmd = ["gcc", "-O2", "-mpopcnt", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           SRC, "-o", LIB + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def load_library(path):
    """Load an oracle build (the default one, or a test variant) with its signatures."""
    L = ctypes.CDLL(path)
    _declare(L)
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = load_library(LIB)
    return _lib


def _declare(L):
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    L.oracle_order.argtypes = [i32, i32, P, i32, P, P]
    L.oracle_order.restype = None
    L.oracle_best.argtypes = [i32, i32, i32, i32, P, i32, P, P, i32, i64, i64, P, i32,
                              P, P, P, P]
    L.oracle_best.restype = ctypes.c_int
    L.oracle_best_share.argtypes = [i32, i32, i32, i32, P, i32, P, P, i32, i64, i64, P, i32,
                                    i32, i32, P, P, P, P]
    L.oracle_best_share.restype = ctypes.c_int
    L.oracle_wsc.argtypes = [i32, i32, i32, i32, P, i32, P, i32, i64, i64, i32, i32, P,
                             i32, i32, P, P, P, P, P]
    L.oracle_wsc.restype = ctypes.c_int


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _words(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
    if a.ndim != 2:
        raise ValueError("expected a 2-D uint64 array")
    return a


def order(T, N, L=None):
    """Sorted (sparsest-first) position -> caller gene id."""
    T, N = _words(T), _words(N)
    G = T.shape[0]
    perm = np.zeros(G, dtype=np.int32)
    (L or lib()).oracle_order(G, T.shape[1], _ptr(T), N.shape[1], _ptr(N), _ptr(perm))
    return perm


def counters_dict(c):
    c = np.asarray(c).reshape(3, MAX_H + 1)
    return {"visited": c[0].tolist(), "nonempty": c[1].tolist(), "bound_pruned": c[2].tolist()}


@dataclasses.dataclass
class Best:
    found: bool
    sorted_idx: tuple
    genes: tuple
    tp: int
    fp: int
    tn: int
    score: int
    counters: dict


def best(T, N, n_tumor, n_normal, h, p, q, U=None, mode="empty", perm=None, L=None,
         tn="all") -> Best:
    T, N = _words(T), _words(N)
    G, wt = T.shape
    if perm is None:
        perm = order(T, N, L)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    if U is None:
        U = full_mask(n_tumor, wt)
    U = np.ascontiguousarray(U, dtype=np.uint64)
    idx = np.zeros(MAX_H, dtype=np.int32)
    tp = np.zeros(1, dtype=np.int64)
    fp = np.zeros(1, dtype=np.int64)
    cnt = np.zeros(3 * (MAX_H + 1), dtype=np.uint64)
    r = (L or lib()).oracle_best(G, n_tumor, n_normal, wt, _ptr(T), N.shape[1], _ptr(N), _ptr(perm),
                          h, p, q, _ptr(U), _mode(mode, tn), _ptr(idx), _ptr(tp), _ptr(fp),
                          _ptr(cnt))
    if r < 0:
        raise ValueError("oracle_best: invalid arguments")
    if r == 0:
        return Best(False, (), (), 0, 0, 0, 0, counters_dict(cnt))
    si = tuple(int(i) for i in idx[:h])
    t, f = int(tp[0]), int(fp[0])
    return Best(True, si, tuple(int(perm[i]) for i in si), t, f, n_normal - f,
                p * t + q * (n_normal - f), counters_dict(cnt))


def best_share(T, N, n_tumor, n_normal, h, p, q, g1_lo, g1_hi, U=None, mode="empty",
               perm=None, L=None, tn="all") -> Best:
    """One round restricted to first genes in sorted positions [g1_lo, g1_hi)."""
    T, N = _words(T), _words(N)
    G, wt = T.shape
    if perm is None:
        perm = order(T, N, L)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    U = full_mask(n_tumor, wt) if U is None else np.ascontiguousarray(U, dtype=np.uint64)
    idx = np.zeros(MAX_H, dtype=np.int32)
    tp = np.zeros(1, dtype=np.int64)
    fp = np.zeros(1, dtype=np.int64)
    cnt = np.zeros(3 * (MAX_H + 1), dtype=np.uint64)
    r = (L or lib()).oracle_best_share(G, n_tumor, n_normal, wt, _ptr(T), N.shape[1], _ptr(N),
                                       _ptr(perm), h, p, q, _ptr(U), _mode(mode, tn), g1_lo, g1_hi,
                                       _ptr(idx), _ptr(tp), _ptr(fp), _ptr(cnt))
    if r < 0:
        raise ValueError("oracle_best_share: invalid arguments")
    if r == 0:
        return Best(False, (), (), 0, 0, 0, 0, counters_dict(cnt))
    si = tuple(int(i) for i in idx[:h])
    t, f = int(tp[0]), int(fp[0])
    return Best(True, si, tuple(int(perm[i]) for i in si), t, f, n_normal - f,
                p * t + q * (n_normal - f), counters_dict(cnt))


def full_mask(n, words):
    U = np.zeros(words, dtype=np.uint64)
    for s in range(n):
        U[s >> 6] |= np.uint64(1) << np.uint64(s & 63)
    return U


@dataclasses.dataclass
class WscResult:
    rounds: list          # list of dicts per round
    counters: dict
    final_uncovered: np.ndarray


def wsc(T, N, n_tumor, n_normal, h, p=1, q=10, target=0, max_rounds=0, U0=None,
        mode="bound", cap=4096, L=None, tn="all") -> WscResult:
    T, N = _words(T), _words(N)
    G, wt = T.shape
    genes = np.zeros(cap * h, dtype=np.int32)
    sidx = np.zeros(cap * h, dtype=np.int32)
    rec = np.zeros(cap * 6, dtype=np.int64)
    cnt = np.zeros(3 * (MAX_H + 1), dtype=np.uint64)
    Uo = np.zeros(wt, dtype=np.uint64)
    U0a = None if U0 is None else np.ascontiguousarray(U0, dtype=np.uint64)
    r = (L or lib()).oracle_wsc(G, n_tumor, n_normal, wt, _ptr(T), N.shape[1], _ptr(N), h, p, q,
                         target, max_rounds, _ptr(U0a), _mode(mode, tn), cap, _ptr(genes),
                         _ptr(sidx), _ptr(rec), _ptr(cnt), _ptr(Uo))
    if r < 0:
        raise ValueError("oracle_wsc: invalid arguments")
    if r > cap:
        raise ValueError("oracle_wsc: more rounds than cap")
    rounds = []
    for k in range(r):
        tp, fp, tn, num, den, unc = (int(x) for x in rec[6 * k:6 * k + 6])
        rounds.append({"genes": [int(g) for g in genes[k * h:(k + 1) * h]],
                       "sorted_idx": [int(g) for g in sidx[k * h:(k + 1) * h]],
                       "tp": tp, "fp": fp, "tn": tn, "score_num": num, "score_den": den,
                       "uncovered_before": unc})
    return WscResult(rounds, counters_dict(cnt), Uo)
