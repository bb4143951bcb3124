"""ctypes binding of libpdfs (include/pdfs.h): argument marshalling only.

Every function here forwards to the C ABI of the same name.  Inputs may be
numpy arrays (host memory) or torch tensors on the GPU (device memory; the
library copies them).  There is no CPU fallback: if libpdfs.so is missing the
import of this module raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpdfs.so")

PDFS_OK = 0
PDFS_NO_COMBO = 1
PDFS_PENDING = 2
PDFS_ERR_INVALID_ARG = -1
PDFS_ERR_UNSUPPORTED = -2
PDFS_ERR_OUT_OF_MEMORY = -3
PDFS_ERR_DEVICE = -4
PDFS_ERR_TRUNCATED = -5

PDFS_PRUNE_NONE = 0
PDFS_PRUNE_EMPTY = 1
PDFS_PRUNE_BOUND = 2
PRUNE_MODES = {"none": PDFS_PRUNE_NONE, "empty": PDFS_PRUNE_EMPTY, "bound": PDFS_PRUNE_BOUND}
MAX_H = 9


class pdfs_matrix(ctypes.Structure):
    _fields_ = [("G", ctypes.c_int32), ("n_tumor", ctypes.c_int32),
                ("n_normal", ctypes.c_int32), ("on_device", ctypes.c_int32),
                ("tumor", ctypes.c_void_p), ("normal", ctypes.c_void_p),
                ("tumor_stride_words", ctypes.c_int64), ("normal_stride_words", ctypes.c_int64)]


PDFS_OPT_TIME_KERNELS = 1


class pdfs_options(ctypes.Structure):
    _fields_ = [("prune_mode", ctypes.c_int32), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("flags", ctypes.c_int32),
                ("pair_cap", ctypes.c_int32)]


class pdfs_combo(ctypes.Structure):
    _fields_ = [("h", ctypes.c_int32), ("genes", ctypes.c_int32 * MAX_H),
                ("sorted_idx", ctypes.c_int32 * MAX_H), ("tp", ctypes.c_int32),
                ("fp", ctypes.c_int32), ("tn", ctypes.c_int32),
                ("uncovered_before", ctypes.c_int32), ("newly_covered", ctypes.c_int32),
                ("score_num", ctypes.c_int64), ("score_den", ctypes.c_int64)]


class pdfs_stats(ctypes.Structure):
    _fields_ = [("visited", ctypes.c_uint64 * (MAX_H + 1)),
                ("nonempty", ctypes.c_uint64 * (MAX_H + 1)),
                ("bound_pruned", ctypes.c_uint64 * (MAX_H + 1)),
                ("rounds", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("ns_total", ctypes.c_int64),
                ("kernel_ns", ctypes.c_int64 * 3), ("kernel_launches", ctypes.c_int32 * 3),
                ("pair_macs", ctypes.c_uint64), ("dfs_visits", ctypes.c_uint64 * (MAX_H + 1)),
                ("dfs_leaves", ctypes.c_uint64), ("dfs_fp_leaves", ctypes.c_uint64),
                ("dfs_visit_words3", ctypes.c_uint64), ("dfs_visit_words4", ctypes.c_uint64)]


EXPORTS = ["pdfs_create", "pdfs_destroy", "pdfs_set_prune_mode", "pdfs_best_combo",
           "pdfs_wsc_run", "pdfs_strerror", "pdfs_last_error",
           "pdfs_batch_create", "pdfs_batch_run", "pdfs_batch_destroy",
           "pdfs_server_create", "pdfs_server_submit", "pdfs_server_poll", "pdfs_server_drain",
           "pdfs_server_destroy", "pdfs_measure_int_peak", "pdfs_batch_last_error",
           "pdfs_server_last_error", "pdfs_best_combo_noalloc"]
PDFS_NOALLOC_SCRATCH_BYTES = 64 << 20
PDFS_OPT_GRAPHS = 2
PDFS_OPT_AUTOTUNE = 4
PDFS_OPT_TN_LITERAL = 8
PDFS_OPT_BATCH_STREAMS = 16
PDFS_OPT_BATCH_ONE_LAUNCH = 32
BATCH_PATHS = {"auto": 0, "streams": PDFS_OPT_BATCH_STREAMS, "one_launch": PDFS_OPT_BATCH_ONE_LAUNCH}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, u32 = ctypes.c_int32, ctypes.c_uint32
    L.pdfs_create.argtypes = [ctypes.POINTER(pdfs_matrix), ctypes.POINTER(pdfs_options),
                              ctypes.POINTER(P)]
    L.pdfs_create.restype = i32
    L.pdfs_destroy.argtypes = [P]
    L.pdfs_destroy.restype = None
    L.pdfs_set_prune_mode.argtypes = [P, i32]
    L.pdfs_set_prune_mode.restype = i32
    L.pdfs_best_combo.argtypes = [P, i32, u32, u32, P, ctypes.POINTER(pdfs_combo),
                                  ctypes.POINTER(pdfs_stats)]
    L.pdfs_best_combo.restype = i32
    L.pdfs_best_combo_noalloc.argtypes = [P, i32, u32, u32, P, ctypes.POINTER(pdfs_combo),
                                          ctypes.POINTER(pdfs_stats)]
    L.pdfs_best_combo_noalloc.restype = i32
    L.pdfs_wsc_run.argtypes = [P, i32, u32, u32, i32, i32, P, ctypes.POINTER(pdfs_combo), i32,
                               ctypes.POINTER(i32), P, ctypes.POINTER(pdfs_stats)]
    L.pdfs_wsc_run.restype = i32
    L.pdfs_strerror.argtypes = [i32]
    L.pdfs_strerror.restype = ctypes.c_char_p
    L.pdfs_last_error.argtypes = [P]
    L.pdfs_last_error.restype = ctypes.c_char_p
    PC = ctypes.POINTER(pdfs_combo)
    L.pdfs_batch_create.argtypes = [ctypes.POINTER(pdfs_matrix), i32, ctypes.POINTER(pdfs_options),
                                    ctypes.POINTER(P)]
    L.pdfs_batch_create.restype = i32
    L.pdfs_batch_run.argtypes = [P, ctypes.POINTER(i32), u32, u32, ctypes.POINTER(i32),
                                 ctypes.POINTER(PC), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                 ctypes.POINTER(pdfs_stats)]
    L.pdfs_batch_run.restype = i32
    L.pdfs_batch_destroy.argtypes = [P]
    L.pdfs_batch_destroy.restype = None
    L.pdfs_server_create.argtypes = [ctypes.POINTER(pdfs_options), ctypes.c_uint64, i32,
                                     ctypes.POINTER(P)]
    L.pdfs_server_create.restype = i32
    L.pdfs_server_submit.argtypes = [P, ctypes.POINTER(pdfs_matrix), i32, u32, u32, i32,
                                     ctypes.POINTER(ctypes.c_uint64)]
    L.pdfs_server_submit.restype = i32
    L.pdfs_server_poll.argtypes = [P, ctypes.c_uint64, PC, i32, ctypes.POINTER(i32),
                                   ctypes.POINTER(ctypes.c_int64)]
    L.pdfs_server_poll.restype = i32
    L.pdfs_server_drain.argtypes = [P]
    L.pdfs_server_drain.restype = i32
    L.pdfs_server_destroy.argtypes = [P]
    L.pdfs_server_destroy.restype = None
    L.pdfs_batch_last_error.argtypes = [P]
    L.pdfs_batch_last_error.restype = ctypes.c_char_p
    L.pdfs_server_last_error.argtypes = [P]
    L.pdfs_server_last_error.restype = ctypes.c_char_p
    L.pdfs_measure_int_peak.argtypes = [i32, ctypes.POINTER(ctypes.c_double)]
    L.pdfs_measure_int_peak.restype = i32
    return L


lib = _load()


class PdfsError(RuntimeError):
    def __init__(self, code, detail=""):
        self.code = code
        msg = lib.pdfs_strerror(code).decode()
        super().__init__(f"{msg} ({code}){': ' + detail if detail else ''}")


def pdfs_strerror(code: int) -> str:
    return lib.pdfs_strerror(code).decode()


def _matrix_arg(tumor, normal, n_tumor, n_normal):
    """Builds pdfs_matrix from numpy (host) or torch.cuda (device) uint64/int64 arrays."""
    keep = []

    def ptr_of(a):
        if a is None:
            return None, 0, False
        if hasattr(a, "is_cuda") and a.is_cuda:
            if a.dim() != 2 or a.element_size() != 8 or a.stride(1) != 1:
                raise ValueError("device matrix must be 2-D, 8-byte elements, unit column stride")
            keep.append(a)
            return a.data_ptr(), a.stride(0), True
        arr = np.ascontiguousarray(np.asarray(a, dtype=np.uint64))
        if arr.ndim != 2:
            raise ValueError("matrix must be 2-D")
        keep.append(arr)
        return arr.ctypes.data, arr.shape[1], False

    tp, ts, tdev = ptr_of(tumor)
    npp, ns, ndev = ptr_of(normal if n_normal > 0 else None)
    if normal is not None and n_normal > 0 and tdev != ndev:
        raise ValueError("tumor and normal must both be host or both be device arrays")
    G = tumor.shape[0]
    m = pdfs_matrix(G=G, n_tumor=n_tumor, n_normal=n_normal, on_device=int(tdev),
                    tumor=tp, normal=npp, tumor_stride_words=ts, normal_stride_words=ns)
    return m, keep


def pdfs_create(tumor, normal, n_tumor, n_normal, prune_mode="bound", device=0, stream=None,
                flags=0, pair_cap=0):
    """Returns an opaque context handle (int).  Raises PdfsError on failure."""
    m, keep = _matrix_arg(tumor, normal, n_tumor, n_normal)
    mode = PRUNE_MODES[prune_mode] if isinstance(prune_mode, str) else int(prune_mode)
    opt = pdfs_options(prune_mode=mode, device=device, stream=stream, flags=flags,
                       pair_cap=pair_cap)
    out = ctypes.c_void_p()
    rc = lib.pdfs_create(ctypes.byref(m), ctypes.byref(opt), ctypes.byref(out))
    del keep
    if rc != PDFS_OK:
        raise PdfsError(rc, lib.pdfs_last_error(None).decode())
    return out.value


def pdfs_destroy(ctx):
    lib.pdfs_destroy(ctx)


def pdfs_set_prune_mode(ctx, mode):
    mode = PRUNE_MODES[mode] if isinstance(mode, str) else int(mode)
    rc = lib.pdfs_set_prune_mode(ctx, mode)
    if rc != PDFS_OK:
        raise PdfsError(rc, lib.pdfs_last_error(ctx).decode())


def stats_dict(s: pdfs_stats, h: int):
    return {"visited": [int(v) for v in s.visited[:MAX_H + 1]],
            "nonempty": [int(v) for v in s.nonempty[:MAX_H + 1]],
            "bound_pruned": [int(v) for v in s.bound_pruned[:MAX_H + 1]],
            "rounds": int(s.rounds), "ns_total": int(s.ns_total),
            "kernel_ns": [int(v) for v in s.kernel_ns], "kernel_launches": [int(v) for v in s.kernel_launches],
            "pair_macs": int(s.pair_macs), "dfs_visits": [int(v) for v in s.dfs_visits],
            "dfs_leaves": int(s.dfs_leaves), "dfs_fp_leaves": int(s.dfs_fp_leaves),
            "dfs_visit_words3": int(s.dfs_visit_words3), "dfs_visit_words4": int(s.dfs_visit_words4)}


def combo_dict(c: pdfs_combo):
    h = c.h
    return {"genes": [int(g) for g in c.genes[:h]], "sorted_idx": [int(g) for g in c.sorted_idx[:h]],
            "tp": int(c.tp), "fp": int(c.fp), "tn": int(c.tn), "score_num": int(c.score_num),
            "score_den": int(c.score_den), "uncovered_before": int(c.uncovered_before),
            "newly_covered": int(c.newly_covered)}


def pdfs_best_combo(ctx, h, alpha_p, alpha_q, uncovered=None):
    """Returns (combo dict or None, stats dict)."""
    out = pdfs_combo()
    st = pdfs_stats()
    u = None
    if uncovered is not None:
        u = np.ascontiguousarray(np.asarray(uncovered, dtype=np.uint64))
    rc = lib.pdfs_best_combo(ctx, h, alpha_p, alpha_q, None if u is None else u.ctypes.data,
                             ctypes.byref(out), ctypes.byref(st))
    if rc == PDFS_NO_COMBO:
        return None, stats_dict(st, h)
    if rc != PDFS_OK:
        raise PdfsError(rc, lib.pdfs_last_error(ctx).decode())
    return combo_dict(out), stats_dict(st, h)


def pdfs_best_combo_noalloc(ctx, h, alpha_p, alpha_q, uncovered=None):
    """The allocation-free round: returns (combo dict or None, stats dict)."""
    out = pdfs_combo()
    st = pdfs_stats()
    u = None
    if uncovered is not None:
        u = np.ascontiguousarray(np.asarray(uncovered, dtype=np.uint64))
    rc = lib.pdfs_best_combo_noalloc(ctx, h, alpha_p, alpha_q,
                                     None if u is None else u.ctypes.data, ctypes.byref(out),
                                     ctypes.byref(st))
    if rc == PDFS_NO_COMBO:
        return None, stats_dict(st, h)
    if rc != PDFS_OK:
        raise PdfsError(rc, lib.pdfs_last_error(ctx).decode())
    return combo_dict(out), stats_dict(st, h)


def pdfs_wsc_run(ctx, h, alpha_p, alpha_q, target_covered=0, max_rounds=0,
                 initial_uncovered=None, cap=4096, n_tumor=None):
    """Returns (list of combo dicts, stats dict, final uncovered mask or None)."""
    out = (pdfs_combo * max(cap, 1))()
    st = pdfs_stats()
    n_out = ctypes.c_int32(0)
    u = None
    if initial_uncovered is not None:
        u = np.ascontiguousarray(np.asarray(initial_uncovered, dtype=np.uint64))
    final = None
    if n_tumor is not None:
        final = np.zeros(max(1, (n_tumor + 63) // 64), dtype=np.uint64)
    rc = lib.pdfs_wsc_run(ctx, h, alpha_p, alpha_q, target_covered, max_rounds,
                          None if u is None else u.ctypes.data, out, cap, ctypes.byref(n_out),
                          None if final is None else final.ctypes.data, ctypes.byref(st))
    if rc != PDFS_OK:
        raise PdfsError(rc, lib.pdfs_last_error(ctx).decode())
    rounds = [combo_dict(out[i]) for i in range(n_out.value)]
    return rounds, stats_dict(st, h), final


class Solver:
    """Owns one context for a cohort (packed uint64 rows, LSB-first samples)."""

    def __init__(self, tumor, normal, n_tumor, n_normal, prune_mode="bound", device=0,
                 stream=None, time_kernels=False, tn_literal=False, pair_cap=0):
        self.n_tumor = n_tumor
        self.n_normal = n_normal
        self.ctx = None
        flags = (PDFS_OPT_TIME_KERNELS if time_kernels else 0) | \
            (PDFS_OPT_TN_LITERAL if tn_literal else 0)
        self.ctx = pdfs_create(tumor, normal, n_tumor, n_normal, prune_mode, device, stream, flags,
                               pair_cap)

    def close(self):
        if self.ctx:
            pdfs_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_prune_mode(self, mode):
        pdfs_set_prune_mode(self.ctx, mode)

    def best(self, h, p=1, q=10, uncovered=None):
        return pdfs_best_combo(self.ctx, h, p, q, uncovered)

    def best_noalloc(self, h, p=1, q=10, uncovered=None):
        return pdfs_best_combo_noalloc(self.ctx, h, p, q, uncovered)

    def wsc(self, h, p=1, q=10, target=0, max_rounds=0, initial_uncovered=None, cap=4096):
        return pdfs_wsc_run(self.ctx, h, p, q, target, max_rounds, initial_uncovered, cap,
                            n_tumor=self.n_tumor)


def pdfs_batch_create(instances, prune_mode="bound", device=0, autotune=False,
                      path="auto", pair_cap=0):
    """instances: list of (tumor, normal, n_tumor, n_normal) host arrays.  Returns a handle.
    path: "auto" (the faster way for the mode: one launch per round step over all
    instances under bound pruning, each instance's own launches on the batch's
    streams otherwise), "streams" or "one_launch" (PDFS_OPT_BATCH_STREAMS /
    PDFS_OPT_BATCH_ONE_LAUNCH).  pair_cap: every instance's initial pair-list
    capacity (pdfs_options.pair_cap)."""
    if path not in BATCH_PATHS:
        raise ValueError(f"path must be one of {sorted(BATCH_PATHS)}")
    mats, keep = [], []
    for (T, N, nt, nn) in instances:
        m, k = _matrix_arg(T, N, nt, nn)
        mats.append(m)
        keep.append(k)
    arr = (pdfs_matrix * len(mats))(*mats)
    mode = PRUNE_MODES[prune_mode] if isinstance(prune_mode, str) else int(prune_mode)
    opt = pdfs_options(prune_mode=mode, device=device, stream=None,
                       flags=(PDFS_OPT_AUTOTUNE if autotune else 0) | BATCH_PATHS[path],
                       pair_cap=pair_cap)
    out = ctypes.c_void_p()
    rc = lib.pdfs_batch_create(arr, len(mats), ctypes.byref(opt), ctypes.byref(out))
    del keep
    if rc != PDFS_OK:
        raise PdfsError(rc, lib.pdfs_batch_last_error(None).decode())
    return out.value


def pdfs_batch_run(batch, hs, alpha_p, alpha_q, targets=None, caps=None, n_tumors=None):
    """Returns (list of per-instance round lists, aggregate stats dict)."""
    n = len(hs)
    if caps is None:
        caps = [(nt + 1) if n_tumors else 4096 for nt in (n_tumors or [0] * n)]
    bufs = [(pdfs_combo * max(1, c))() for c in caps]
    outs = (ctypes.POINTER(pdfs_combo) * n)(*[ctypes.cast(b, ctypes.POINTER(pdfs_combo))
                                               for b in bufs])
    h_arr = (ctypes.c_int32 * n)(*hs)
    t_arr = (ctypes.c_int32 * n)(*(targets or [0] * n))
    c_arr = (ctypes.c_int32 * n)(*caps)
    n_out = (ctypes.c_int32 * n)()
    st = pdfs_stats()
    rc = lib.pdfs_batch_run(batch, h_arr, alpha_p, alpha_q, t_arr, outs, c_arr, n_out,
                            ctypes.byref(st))
    if rc != PDFS_OK:
        raise PdfsError(rc, lib.pdfs_batch_last_error(batch).decode())
    res = [[combo_dict(bufs[i][k]) for k in range(n_out[i])] for i in range(n)]
    return res, stats_dict(st, max(hs))


def pdfs_batch_destroy(batch):
    lib.pdfs_batch_destroy(batch)


def pdfs_server_create(prune_mode="bound", device=0, hbm_budget_bytes=0, max_active=8):
    mode = PRUNE_MODES[prune_mode] if isinstance(prune_mode, str) else int(prune_mode)
    opt = pdfs_options(prune_mode=mode, device=device, stream=None, flags=0)
    out = ctypes.c_void_p()
    rc = lib.pdfs_server_create(ctypes.byref(opt), hbm_budget_bytes, max_active,
                                ctypes.byref(out))
    if rc != PDFS_OK:
        raise PdfsError(rc, lib.pdfs_server_last_error(None).decode())
    return out.value


def pdfs_server_submit(server, tumor, normal, n_tumor, n_normal, h, alpha_p, alpha_q, target=0):
    m, keep = _matrix_arg(tumor, normal, n_tumor, n_normal)
    ticket = ctypes.c_uint64(0)
    rc = lib.pdfs_server_submit(server, ctypes.byref(m), h, alpha_p, alpha_q, target,
                                ctypes.byref(ticket))
    del keep
    if rc != PDFS_OK:
        raise PdfsError(rc, lib.pdfs_server_last_error(server).decode())
    return ticket.value


def pdfs_server_poll(server, ticket, cap=4096):
    """Returns None while pending, else (rounds list, latency seconds)."""
    buf = (pdfs_combo * max(1, cap))()
    n_out = ctypes.c_int32(0)
    lat = ctypes.c_int64(0)
    rc = lib.pdfs_server_poll(server, ticket, buf, cap, ctypes.byref(n_out), ctypes.byref(lat))
    if rc == PDFS_PENDING:
        return None
    if rc != PDFS_OK:
        raise PdfsError(rc, lib.pdfs_server_last_error(server).decode())
    return [combo_dict(buf[k]) for k in range(n_out.value)], lat.value * 1e-9


def pdfs_server_drain(server):
    rc = lib.pdfs_server_drain(server)
    if rc != PDFS_OK:
        raise PdfsError(rc)


def pdfs_server_destroy(server):
    lib.pdfs_server_destroy(server)


def pdfs_measure_int_peak(device=0):
    """Measured integer VALU rate (lane-ops/s) for the and + popcount pair."""
    v = ctypes.c_double(0.0)
    rc = lib.pdfs_measure_int_peak(device, ctypes.byref(v))
    if rc != PDFS_OK:
        raise PdfsError(rc, "probe failed")
    return v.value
