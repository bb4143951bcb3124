"""Brute-force definition of one greedy round.  TEST INFRASTRUCTURE ONLY.

The plain definition P-DFS reaches exactly (Sec. II-B, Eq. 1; score of
Sec. II-C; maximum search of Alg. 2): among all h-subsets gamma of genes whose
cover C(gamma) contains at least one still-uncovered tumour sample, take the
one with the largest S = p*TP + q*TN, ties to the lexicographically smallest
tuple of sorted (sparsest-first) indices.  Written on unpacked 0/1 numpy
matrices, enumerating every subset with itertools -- independent of the C
oracle's bit-vector walk.  Only for tiny inputs.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def sparse_first_order(tumor: np.ndarray, normal: np.ndarray) -> np.ndarray:
    """Genes sorted by ascending combined mutation count, ties by gene id."""
    counts = tumor.sum(axis=1).astype(np.int64) + normal.sum(axis=1).astype(np.int64)
    return np.lexsort((np.arange(tumor.shape[0]), counts)).astype(np.int32)


def best(tumor, normal, h, p, q, uncovered, tn="all"):
    """Returns (sorted_idx tuple, tp, fp, score) or None; tumor/normal are bool.
    tn = "all": a normal counts as a false positive when it carries every gene
    of the subset; "literal": when it carries any of them (TN = normals with
    none of the genes)."""
    tumor = np.asarray(tumor, dtype=bool)
    normal = np.asarray(normal, dtype=bool)
    order = sparse_first_order(tumor, normal)
    Tu = tumor[order][:, np.asarray(uncovered, dtype=bool)]
    Ns = normal[order]
    n_normal = normal.shape[1]
    best_key = None
    for combo in itertools.combinations(range(tumor.shape[0]), h):
        c = list(combo)
        tp = int(np.all(Tu[c], axis=0).sum())
        if tp == 0:
            continue
        hitn = np.any(Ns[c], axis=0) if tn == "literal" else np.all(Ns[c], axis=0)
        fp = int(hitn.sum()) if n_normal else 0
        s = p * tp + q * (n_normal - fp)
        if best_key is None or s > best_key[3]:
            best_key = (combo, tp, fp, s)
    return best_key


def wsc(tumor, normal, h, p, q, target=0, max_rounds=0, tn="all"):
    """Greedy loop (Alg. 1) on top of brute-force rounds."""
    tumor = np.asarray(tumor, dtype=bool)
    n_tumor = tumor.shape[1]
    order = sparse_first_order(tumor, normal)
    unc = np.ones(n_tumor, dtype=bool)
    K = target if target > 0 else n_tumor
    out = []
    while (n_tumor - unc.sum()) < K and (max_rounds <= 0 or len(out) < max_rounds):
        b = best(tumor, normal, h, p, q, unc, tn)
        if b is None:
            break
        combo, tp, fp, s = b
        genes = [int(order[i]) for i in combo]
        out.append({"genes": genes, "sorted_idx": list(combo), "tp": tp, "fp": fp, "score_num": s,
                    "uncovered_before": int(unc.sum())})
        unc &= ~np.all(tumor[genes], axis=0)
    return out


def counts(tumor, normal, h, uncovered):
    """Per-depth node counts of the empty-intersection walk, by direct enumeration.

    A depth-l node is an l-tuple i1<...<il of sorted indices with
    i_j <= G-h+j-1 (the loop bounds of Alg. 2, 0-based).  It is visited when its
    (l-1)-prefix has a non-empty cover (every depth-1 node is visited) and it is
    non-empty when its own cover of uncovered tumour samples is non-empty.
    """
    tumor = np.asarray(tumor, dtype=bool)
    order = sparse_first_order(tumor, normal)
    Tu = tumor[order][:, np.asarray(uncovered, dtype=bool)]
    G = tumor.shape[0]
    visited = [0] * (h + 1)
    nonempty = [0] * (h + 1)
    for l in range(1, h + 1):
        for combo in itertools.combinations(range(G), l):
            if any(combo[j] > G - h + j for j in range(l)):
                continue
            pre = list(combo[:-1])
            if pre and not np.any(np.all(Tu[pre], axis=0)):
                continue
            visited[l] += 1
            if np.any(np.all(Tu[list(combo)], axis=0)):
                nonempty[l] += 1
    return visited, nonempty


def n_choose_k(n, k):
    return math.comb(n, k)
