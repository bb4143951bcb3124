"""The oracle's pins are strong enough to catch plausible mistakes.

Each case copies the oracle source, plants one mistake (a dropped term, a
wrong sign, an off-by-one loop bound, a flipped tie-break, an unsafe bound,
a reversed sort, a wrong cover update, OR in place of AND), builds it with
gcc on the CPU, and checks that the pins used by test_oracle_pins reject it.
"""
import os
import subprocess

import numpy as np
import pytest

from oracle import bruteforce as bf
from oracle import cpu
from paper_2603_16721_amd import synth
from tests.helpers import mask_of_bits

MUTANTS = {
    "drop_tn_term": ("int64_t s = st->p * tp + st->q * tn;", "int64_t s = st->p * tp;"),
    "tn_sign": ("int64_t tn = st->n_normal - fp;", "int64_t tn = st->n_normal + fp;"),
    "loop_bound_off_by_one": ("int32_t hi = st->G - st->h + l - 1;",
                              "int32_t hi = st->G - st->h + l - 2;"),
    "tie_keeps_last": ("if (!st->found || s > st->best_s) {", "if (!st->found || s >= st->best_s) {"),
    "unsafe_bound": ("st->p * c + st->q * (int64_t)st->n_normal <= st->best_s",
                     "st->p * c + st->q * (int64_t)st->n_normal <= st->best_s + st->q"),
    "sort_dense_first": ("if (x->key != y->key) return x->key < y->key ? -1 : 1;",
                         "if (x->key != y->key) return x->key > y->key ? -1 : 1;"),
    "delcols_keeps_covered": ("for (int w = 0; w < wt; w++) U[w] &= ~cov[w];",
                              "for (int w = 0; w < wt; w++) U[w] &= cov[w];"),
    "normals_or": ("for (int w = 0; w < st->wn; w++) st->z[w] &= nl[w];",
                   "for (int w = 0; w < st->wn; w++) st->z[w] |= nl[w];"),
    "tp_ignores_uncovered": ("memcpy(st.y, U, sizeof(uint64_t) * (size_t)wt);",
                             "memset(st.y, 0xff, sizeof(uint64_t) * (size_t)wt);"),
}


def _build(tmp_path, name):
    src = open(cpu.SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", str(path), "-o", str(so)],
                   check=True)
    return cpu.load_library(str(so))


def _pins_pass(L):
    """A compact run of the pins: brute-force rounds on tiny inputs (all
    modes) and full greedy loops; returns False at the first disagreement."""
    cases = [(1, 12, 70, 30, 0.30, 3, (1, 10)), (3, 10, 130, 65, 0.40, 4, (1, 10)),
             (5, 9, 100, 64, 0.50, 4, (3, 7)), (7, 11, 65, 128, 0.45, 3, (1, 10)),
             (21, 12, 80, 60, 0.45, 2, (1, 10))]
    for seed, G, nt, nn, d, h, a in cases:
        I = synth.random_tiny(seed, G, nt, nn, d, h, alpha=a)
        T, N = I.packed()
        rng = np.random.default_rng(seed)
        for trial in range(3):
            unc = np.ones(nt, bool) if trial == 0 else rng.random(nt) < 0.6
            ref = bf.best(I.tumor, I.normal, h, a[0], a[1], unc)
            for mode in ("none", "empty", "bound"):
                b = cpu.best(T, N, nt, nn, h, a[0], a[1], U=mask_of_bits(unc), mode=mode, L=L)
                got = (b.sorted_idx, b.tp, b.fp, b.score) if b.found else None
                if got != ref:
                    return False
        refw = bf.wsc(I.tumor, I.normal, h, a[0], a[1])
        w = cpu.wsc(T, N, nt, nn, h, a[0], a[1], mode="bound", L=L, max_rounds=len(refw) + 1)
        if [(r["genes"], r["tp"], r["fp"]) for r in w.rounds] != \
                [(r["genes"], r["tp"], r["fp"]) for r in refw]:
            return False
    return True


def test_unmodified_oracle_passes(tmp_path):
    assert _pins_pass(cpu.lib())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    assert not _pins_pass(_build(tmp_path, name)), f"mutant {name} survived the pins"
