"""Held-out coverage of learned combinations (the accuracy protocol of Sec. IV).

A cohort's tumour and normal samples are split at random, 75 % / 25 %; the
greedy weighted set cover (Alg. 1, run on the GPU through `pdfs.Solver`)
learns its h-hit combinations on the training split only; the frozen
combinations are then scored on both splits.  A sample is *covered* when it
carries every gene of at least one learned combination.  Reported per split:
tumours covered TC of TT, normals covered NC of NT, sensitivity TC/TT and
specificity 1 - NC/NT (the quantities of Tables III and IV).

This module is reporting code around the library: the split, the packing and
the coverage count are plain numpy on the host; every combination it scores
comes from the GPU path.
"""
from __future__ import annotations

import numpy as np

from . import synth


def split_samples(n: int, test_frac: float, rng: np.random.Generator):
    """Random disjoint (train, test) index arrays over n samples, each sorted;
    the test part has round(test_frac * n) samples."""
    perm = rng.permutation(n)
    n_test = int(round(test_frac * n))
    return np.sort(perm[n_test:]), np.sort(perm[:n_test])


def split_cohort(inst: synth.Instance, test_frac: float = 0.25, seed: int = 0) -> dict:
    """Tumour and normal columns of `inst` split independently (same seed
    stream).  Returns bool matrices [G, n] for each part."""
    rng = np.random.default_rng(seed)
    t_tr, t_te = split_samples(inst.n_tumor, test_frac, rng)
    n_tr, n_te = split_samples(inst.n_normal, test_frac, rng)
    return {
        "train": (inst.tumor[:, t_tr], inst.normal[:, n_tr]),
        "test": (inst.tumor[:, t_te], inst.normal[:, n_te]),
    }


def covered(combos, bits: np.ndarray) -> np.ndarray:
    """bool [n]: samples (columns of bits [G, n]) carrying every gene of at
    least one combination (combos: iterables of gene ids)."""
    hit = np.zeros(bits.shape[1], dtype=bool)
    for genes in combos:
        hit |= np.logical_and.reduce(bits[list(genes)], axis=0)
    return hit


def coverage_report(combos, tumor: np.ndarray, normal: np.ndarray) -> dict:
    """TC, TT, NC, NT, sensitivity and specificity of `combos` on one split."""
    tc = int(covered(combos, tumor).sum())
    nc = int(covered(combos, normal).sum())
    tt, nt = tumor.shape[1], normal.shape[1]
    return {"TC": tc, "TT": tt, "NC": nc, "NT": nt,
            "sensitivity": tc / tt if tt else None,
            "specificity": 1.0 - nc / nt if nt else None}


def learn_and_evaluate(pdfs, inst: synth.Instance, test_frac: float = 0.25, seed: int = 0,
                       prune_mode: str = "bound", tn_literal: bool = False) -> dict:
    """Split, learn the cover on the training split with the GPU path
    (`pdfs` is the binding module), report both splits.  tn_literal: learn
    with the literal reading of T- (TN = normals carrying none of the genes)."""
    parts = split_cohort(inst, test_frac, seed)
    t_tr, n_tr = parts["train"]
    T, N = synth.pack_rows(t_tr), synth.pack_rows(n_tr)
    # a coverage-target stop rule keeps its fraction of the tumours
    target = 0
    if inst.target_covered:
        target = int(np.ceil(inst.target_covered * t_tr.shape[1] / inst.n_tumor))
    with pdfs.Solver(T, N if n_tr.shape[1] else None, t_tr.shape[1], n_tr.shape[1],
                     prune_mode, tn_literal=tn_literal) as sv:
        rounds, _, _ = sv.wsc(inst.h, inst.alpha_p, inst.alpha_q, target=target)
    combos = [r["genes"] for r in rounds]
    return {"combinations": len(combos), "h": inst.h, "split_seed": seed, "target": target,
            "tn": "literal" if tn_literal else "all",
            "train_tp_sum": sum(r["tp"] for r in rounds),
            "train": coverage_report(combos, *parts["train"]),
            "test": coverage_report(combos, *parts["test"]),
            "combos": combos}
