"""Shared test helpers (no method arithmetic beyond plain recounts)."""
import numpy as np


def bits_of_mask(U, n):
    U = np.asarray(U, dtype=np.uint64)
    out = np.zeros(n, dtype=bool)
    for s in range(n):
        out[s] = (int(U[s >> 6]) >> (s & 63)) & 1
    return out


def mask_of_bits(b):
    b = np.asarray(b, dtype=bool)
    W = max(1, (b.size + 63) // 64)
    U = np.zeros(W, dtype=np.uint64)
    for s in np.flatnonzero(b):
        U[s >> 6] |= np.uint64(1) << np.uint64(s & 63)
    return U


def recount(tumor, normal, genes, uncovered):
    """TP/FP straight from the unpacked 0/1 matrices (the coverage re-check
    of the paper's artifact)."""
    cov_t = np.all(tumor[list(genes)], axis=0)
    cov_n = np.all(normal[list(genes)], axis=0) if normal.shape[1] else np.zeros(0, bool)
    return int((cov_t & uncovered).sum()), int(cov_n.sum()), cov_t
