"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bit-exact on every field: the same chosen combinations in the same order,
with the same TP / FP / TN / score, in both GPU pruning modes (empty-only,
the paper's Alg. 2, and exact bound pruning); per-depth counters of the
empty-only mode equal the oracle's.  Sizes span several 32x32 MFMA tiles, 64-
pair batches, row widths from 1 to 20 words and ragged sample counts.
"""
import json
import os

import numpy as np
import pytest

from oracle import cpu
from paper_2603_16721_amd import synth
from tests.helpers import mask_of_bits

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
KEYS = ("genes", "sorted_idx", "tp", "fp", "tn", "score_num", "score_den", "uncovered_before")


@pytest.fixture(scope="module")
def pdfs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_16721_amd import pdfs as binding
    return binding


def _same_rounds(got, exp):
    assert len(got) == len(exp), (len(got), len(exp))
    for k, (g, e) in enumerate(zip(got, exp)):
        for key in KEYS:
            assert g[key] == e[key], (k, key, g, e)
        if "newly_covered" in g:
            # the round adds its tp samples to the cover, and the next round
            # starts from what is left
            assert g["newly_covered"] == e["tp"], (k, g)
            if k + 1 < len(got):
                assert got[k + 1]["uncovered_before"] == g["uncovered_before"] - g["newly_covered"]


def _counters_equal(gpu_stats, oracle_counters, h):
    for l in range(1, h + 1):
        assert gpu_stats["visited"][l] == oracle_counters["visited"][l], ("visited", l)
        assert gpu_stats["nonempty"][l] == oracle_counters["nonempty"][l], ("nonempty", l)


TINY = [
    # seed, G, n_tumor, n_normal, density, h, alpha
    (101, 5, 1, 0, 0.9, 2, (1, 10)),
    (102, 40, 63, 17, 0.25, 3, (1, 10)),
    (103, 70, 64, 64, 0.2, 4, (1, 10)),
    (104, 90, 65, 1, 0.15, 3, (3, 7)),
    (105, 33, 130, 100, 0.3, 2, (1, 1)),
    (106, 120, 200, 128, 0.12, 4, (1, 10)),
    (107, 64, 129, 300, 0.2, 3, (0, 1)),
    (108, 200, 300, 50, 0.06, 4, (2, 5)),
    (109, 50, 700, 512, 0.1, 3, (1, 10)),
    (110, 16, 1280, 200, 0.5, 4, (1, 10)),
    (111, 300, 90, 30, 0.05, 2, (1, 10)),
    (112, 45, 150, 40, 0.2, 1, (1, 10)),
    (113, 4, 100, 10, 0.8, 4, (1, 10)),
    (114, 60, 100, 40, 0.2, 4, (0, 1)),
    (115, 80, 150, 60, 0.15, 4, (7, 2)),
]


@pytest.mark.parametrize("case", TINY, ids=[f"s{c[0]}_G{c[1]}_nt{c[2]}_h{c[5]}" for c in TINY])
@pytest.mark.parametrize("mode", ["empty", "bound"])
def test_wsc_tiny(pdfs, case, mode):
    seed, G, nt, nn, d, h, (p, q) = case
    I = synth.random_tiny(seed, G, nt, nn, d, h, alpha=(p, q))
    T, N = I.packed()
    exp = cpu.wsc(T, N, nt, nn, h, p, q, mode="empty")
    with pdfs.Solver(T, N, nt, nn, mode) as s:
        got, stats, final = s.wsc(h, p, q)
    _same_rounds(got, exp.rounds)
    assert np.array_equal(final, exp.final_uncovered)
    if mode == "empty":
        _counters_equal(stats, exp.counters, h)


# With p = 0 every leaf without false positives scores the same, so the argmax
# is decided by the tuple order alone and almost every comparison of two
# candidates (per lane, wave, block and round, at every h) is a tie on S: the
# winner's TP, FP and indices must still come from one leaf.
# Which block holds which leaf varies from run to run, so each case runs
# several times.
TIES = [
    # seed, G, n_tumor, n_normal, density, h, alpha
    (107, 64, 129, 300, 0.2, 3, (0, 1)),
    (114, 60, 100, 40, 0.2, 4, (0, 1)),
    (121, 90, 200, 0, 0.15, 3, (0, 1)),
    (122, 70, 64, 20, 0.25, 2, (0, 3)),
    (123, 45, 150, 40, 0.2, 1, (0, 1)),
    (124, 40, 100, 30, 0.25, 5, (0, 2)),
    (206, 36, 130, 0, 0.3, 6, (0, 1)),
]


@pytest.mark.parametrize("case", TIES, ids=[f"s{c[0]}_G{c[1]}_h{c[5]}" for c in TIES])
@pytest.mark.parametrize("mode", ["empty", "bound"])
def test_wsc_score_ties(pdfs, case, mode):
    seed, G, nt, nn, d, h, (p, q) = case
    I = synth.random_tiny(seed, G, nt, nn, d, h, alpha=(p, q))
    T, N = I.packed()
    exp = cpu.wsc(T, N, nt, nn, h, p, q, mode="empty")
    for _ in range(4):
        with pdfs.Solver(T, N, nt, nn, mode) as s:
            got, stats, final = s.wsc(h, p, q)
        _same_rounds(got, exp.rounds)
        assert np.array_equal(final, exp.final_uncovered)


# h = 5..9: the ring walk below the pair level (every mode; BOUND runs the same walk)
DEEP = [
    # seed, G, n_tumor, n_normal, density, h, alpha
    (201, 40, 100, 30, 0.25, 5, (1, 10)),
    (202, 30, 150, 50, 0.35, 6, (1, 10)),
    (203, 24, 80, 20, 0.45, 7, (2, 5)),
    (204, 20, 64, 64, 0.5, 8, (1, 10)),
    (205, 60, 200, 40, 0.15, 5, (3, 7)),
    (206, 36, 130, 0, 0.3, 6, (0, 1)),
    (207, 18, 96, 40, 0.6, 9, (1, 10)),
    (208, 22, 70, 20, 0.55, 9, (2, 5)),
    (209, 9, 64, 10, 0.9, 9, (1, 10)),    # h = G: one subset
]


@pytest.mark.parametrize("case", DEEP, ids=[f"s{c[0]}_G{c[1]}_h{c[5]}" for c in DEEP])
@pytest.mark.parametrize("mode", ["empty", "none", "bound"])
def test_wsc_deep(pdfs, case, mode):
    seed, G, nt, nn, d, h, (p, q) = case
    I = synth.random_tiny(seed, G, nt, nn, d, h, alpha=(p, q))
    T, N = I.packed()
    exp = cpu.wsc(T, N, nt, nn, h, p, q, mode="empty" if mode == "bound" else mode)
    with pdfs.Solver(T, N, nt, nn, mode) as s:
        got, stats, final = s.wsc(h, p, q)
    _same_rounds(got, exp.rounds)
    assert np.array_equal(final, exp.final_uncovered)
    if mode != "bound":
        _counters_equal(stats, exp.counters, h)


# The literal reading of T- (TN = normals carrying none of the genes): every
# leaf path (h = 1 .. 6, and 9) in every mode, against the oracle.
LITERAL = [c for c in TINY if c[0] in (102, 103, 104, 105, 106, 107, 109, 112, 113, 114, 115)] + \
    [c for c in DEEP if c[0] in (201, 202, 207)] + [(117, 90, 120, 300, 0.12, 2, (1, 10))]


@pytest.mark.parametrize("case", LITERAL, ids=[f"s{c[0]}_h{c[5]}" for c in LITERAL])
@pytest.mark.parametrize("mode", ["empty", "bound", "none"])
def test_wsc_tn_literal(pdfs, case, mode):
    seed, G, nt, nn, d, h, (p, q) = case
    I = synth.random_tiny(seed, G, nt, nn, d, h, alpha=(p, q))
    T, N = I.packed()
    exp = cpu.wsc(T, N, nt, nn, h, p, q, mode="none" if mode == "none" else "empty", tn="literal")
    with pdfs.Solver(T, N, nt, nn, mode, tn_literal=True) as s:
        got, stats, final = s.wsc(h, p, q)
    _same_rounds(got, exp.rounds)
    assert np.array_equal(final, exp.final_uncovered)
    if mode != "bound":
        _counters_equal(stats, exp.counters, h)


# Exhaustive mode: every prefix is extended, empty or not.  The oracle's
# exhaustive walk of seed 108 (G = 200, h = 4) takes minutes; the rest take
# seconds.
TINY_ALL = [c for c in TINY if c[0] != 108]


@pytest.mark.parametrize("case", TINY_ALL, ids=[f"s{c[0]}_G{c[1]}_h{c[5]}" for c in TINY_ALL])
def test_wsc_tiny_exhaustive(pdfs, case):
    seed, G, nt, nn, d, h, (p, q) = case
    I = synth.random_tiny(seed, G, nt, nn, d, h, alpha=(p, q))
    T, N = I.packed()
    exp = cpu.wsc(T, N, nt, nn, h, p, q, mode="none")
    with pdfs.Solver(T, N, nt, nn, "none") as s:
        got, stats, final = s.wsc(h, p, q)
    _same_rounds(got, exp.rounds)
    assert np.array_equal(final, exp.final_uncovered)
    _counters_equal(stats, exp.counters, h)


def test_exhaustive_mode_switches(pdfs):
    # one context: empty-prefix walk, then exhaustive (every gene becomes a row
    # of the round, buffers regrown), then empty again
    I = synth.random_tiny(116, 150, 120, 40, 0.08, 4, alpha=(1, 10))
    T, N = I.packed()
    with pdfs.Solver(T, N, 120, 40, "empty") as s:
        for mode in ("empty", "none", "empty", "bound", "none"):
            s.set_prune_mode(mode)
            exp = cpu.wsc(T, N, 120, 40, 4, 1, 10, max_rounds=3,
                          mode="bound" if mode == "bound" else mode)
            got, stats, _ = s.wsc(4, 1, 10, max_rounds=3)
            _same_rounds(got, exp.rounds)
            if mode != "bound":
                _counters_equal(stats, exp.counters, 4)
            if mode == "none":
                # every depth-2 prefix within the loop bounds is extended
                assert stats["visited"][3] > exp.counters["nonempty"][2]


@pytest.mark.parametrize("case", TINY[1:9], ids=[f"s{c[0]}" for c in TINY[1:9]])
def test_best_combo_random_masks(pdfs, case):
    seed, G, nt, nn, d, h, (p, q) = case
    I = synth.random_tiny(seed, G, nt, nn, d, h, alpha=(p, q))
    T, N = I.packed()
    rng = np.random.default_rng(seed)
    with pdfs.Solver(T, N, nt, nn, "empty") as s:
        for trial in range(4):
            unc = rng.random(nt) < (0.3 + 0.2 * trial)
            U = mask_of_bits(unc)
            e = cpu.best(T, N, nt, nn, h, p, q, U=U, mode="empty")
            g, st = s.best(h, p, q, U)
            if not e.found:
                assert g is None
                continue
            assert g["sorted_idx"] == list(e.sorted_idx)
            assert (g["tp"], g["fp"], g["score_num"]) == (e.tp, e.fp, e.score)
            _counters_equal(st, e.counters, h)


@pytest.mark.parametrize("mode", ["empty", "bound"])
def test_workload_h2_G500(pdfs, mode):
    I = synth.workload_small_h2()
    T, N = I.packed()
    exp = cpu.wsc(T, N, I.n_tumor, I.n_normal, 2, 1, 10, mode="empty")
    with pdfs.Solver(T, N, I.n_tumor, I.n_normal, mode) as s:
        got, stats, _ = s.wsc(2, 1, 10)
    _same_rounds(got, exp.rounds)
    if mode == "empty":
        _counters_equal(stats, exp.counters, 2)


def _golden(key):
    with open(os.path.join(HERE, "golden", "oracle_counters.json")) as f:
        return json.load(f)["cases"][key]


@pytest.mark.parametrize("mode", ["empty", "bound"])
def test_workload_h3_G5000(pdfs, mode):
    I = synth.workload_h3_g5000()
    T, N = I.packed()
    exp = cpu.wsc(T, N, I.n_tumor, I.n_normal, 3, 1, 10, target=I.target_covered, mode="bound")
    with pdfs.Solver(T, N, I.n_tumor, I.n_normal, mode) as s:
        got, stats, _ = s.wsc(3, 1, 10, target=I.target_covered)
    _same_rounds(got, exp.rounds)
    if mode == "empty":
        g = _golden("h3_G5000_empty_all_rounds")
        _same_rounds(got, g["rounds"])
        _counters_equal(stats, g, 3)


def test_workload_h4_G20000_bound_all_rounds(pdfs):
    """Full size (G=20000, h=4): every round of the greedy loop."""
    I = synth.workload_h4_g20000()
    T, N = I.packed()
    exp = cpu.wsc(T, N, I.n_tumor, I.n_normal, 4, 1, 10, mode="bound")
    with pdfs.Solver(T, N, I.n_tumor, I.n_normal, "bound") as s:
        got, _, final = s.wsc(4, 1, 10)
    _same_rounds(got, exp.rounds)
    assert np.array_equal(final, exp.final_uncovered)


def test_workload_h4_G20000_empty_round1_counters(pdfs):
    """Full size, the paper's empty-only walk: round 1 and its exact counts."""
    I = synth.workload_h4_g20000()
    T, N = I.packed()
    g = _golden("h4_G20000_empty_round1")
    with pdfs.Solver(T, N, I.n_tumor, I.n_normal, "empty") as s:
        got, stats, _ = s.wsc(4, 1, 10, max_rounds=1)
    _same_rounds(got, g["rounds"])
    _counters_equal(stats, g, 4)


def test_workload_h4_G20000_empty_all_rounds(pdfs):
    """Full size, the paper's empty-only walk, the whole greedy solve (the
    benchmark's step): all 133 rounds and the per-depth counts summed over
    them equal the oracle's (stored; each round's empty-mode walk run on the
    oracle in first-gene shares).  Then every round again on its own, from
    the uncovered mask the oracle's sequence gives it, with that round's own
    per-depth counts."""
    I = synth.workload_h4_g20000()
    T, N = I.packed()
    g = _golden("h4_G20000_empty_all_rounds")
    with pdfs.Solver(T, N, I.n_tumor, I.n_normal, "empty") as s:
        got, stats, _ = s.wsc(4, 1, 10)
        _same_rounds(got, g["rounds"])
        _counters_equal(stats, g, 4)
        U = cpu.full_mask(I.n_tumor, T.shape[1])
        for r, rd in enumerate(g["rounds"]):
            b, st = s.best(4, 1, 10, U)
            _same_rounds([b], [rd])
            for l in range(1, 5):
                assert st["visited"][l] == g["per_round_visited"][r][l], (r, l)
                assert st["nonempty"][l] == g["per_round_nonempty"][r][l], (r, l)
            cov = U.copy()
            for gene in rd["genes"]:
                cov &= T[gene]
            U = U & ~cov


@pytest.mark.parametrize("key", ["h5_G5000_empty_round1", "h6_G5000_empty_round1"])
@pytest.mark.parametrize("mode", ["empty", "bound"])
def test_workload_h3_G5000_deeper_round1(pdfs, key, mode):
    """Full-size cohort (G=5000, 1000 / 400 samples) at h = 5 and 6: the
    first greedy round of the deep walk, and in EMPTY mode its exact
    per-depth counts (bound pruning changes the counts, not the answer)."""
    I = synth.workload_h3_g5000()
    T, N = I.packed()
    g = _golden(key)
    with pdfs.Solver(T, N, I.n_tumor, I.n_normal, mode) as s:
        got, stats, _ = s.wsc(g["h"], 1, 10, max_rounds=1)
    _same_rounds(got, g["rounds"])
    if mode == "empty":
        _counters_equal(stats, g, g["h"])


def test_two_phase_depth4_medium(pdfs):
    """h = 4, empty-only walk with more active genes than the long-stream
    threshold (384 candidates): the round lists long-stream depth-3
    prefixes for the sorted tile kernel and expands the rest in the main
    kernel.  Every round and every counter equals the oracle's, plain and
    with the rounds replayed from captured graphs on a caller stream; a
    second run on the same context reuses the sized lists."""
    import torch
    I = synth.random_tiny(121, 1200, 150, 40, 0.02, 4)
    T, N = I.packed()
    exp = cpu.wsc(T, N, I.n_tumor, I.n_normal, 4, 1, 10, max_rounds=3, mode="empty")
    with pdfs.Solver(T, N, I.n_tumor, I.n_normal, "empty") as s:
        for _ in range(2):
            got, stats, _ = s.wsc(4, 1, 10, max_rounds=3)
            _same_rounds(got, exp.rounds)
            _counters_equal(stats, exp.counters, 4)
    st = torch.cuda.Stream()
    ctx = pdfs.pdfs_create(T, N, I.n_tumor, I.n_normal, "empty", 0, st.cuda_stream,
                           pdfs.PDFS_OPT_GRAPHS)
    try:
        for _ in range(2):
            got, stats, _ = pdfs.pdfs_wsc_run(ctx, 4, 1, 10, 0, 3, n_tumor=I.n_tumor)
            _same_rounds(got, exp.rounds)
            _counters_equal(stats, exp.counters, 4)
    finally:
        pdfs.pdfs_destroy(ctx)


@pytest.mark.parametrize("mode", ["empty", "bound"])
def test_pair_list_regrowth(pdfs, mode):
    """A pair list far too small for the cohort (64 pairs): each round that
    emits more pairs grows it and runs again from the same uncovered set, so
    the whole cover -- and in empty mode every counter -- equals the
    oracle's.  The grown list serves a second run on the same context, and a
    run whose starting mask already meets the target returns no round."""
    I = synth.workload_h3_g5000()
    T, N = I.packed()
    g = _golden("h3_G5000_empty_all_rounds")
    with pdfs.Solver(T, N, I.n_tumor, I.n_normal, mode, pair_cap=64) as s:
        for _ in range(2):
            got, stats, final = s.wsc(3, 1, 10, target=I.target_covered)
            _same_rounds(got, g["rounds"])
            if mode == "empty":
                _counters_equal(stats, g, 3)
        again, _, final2 = s.wsc(3, 1, 10, target=I.target_covered, initial_uncovered=final)
    assert again == []
    assert np.array_equal(final2, final)


def test_pair_list_regrowth_two_phase_graphs(pdfs):
    """h = 4 two-phase walk with a 64-pair list: the sizing pass and the run
    grow it; plain and replayed from captured graphs on a caller stream."""
    import torch
    I = synth.random_tiny(121, 1200, 150, 40, 0.02, 4)
    T, N = I.packed()
    exp = cpu.wsc(T, N, I.n_tumor, I.n_normal, 4, 1, 10, max_rounds=3, mode="empty")
    with pdfs.Solver(T, N, I.n_tumor, I.n_normal, "empty", pair_cap=64) as s:
        got, stats, _ = s.wsc(4, 1, 10, max_rounds=3)
        _same_rounds(got, exp.rounds)
        _counters_equal(stats, exp.counters, 4)
    st = torch.cuda.Stream()
    ctx = pdfs.pdfs_create(T, N, I.n_tumor, I.n_normal, "empty", 0, st.cuda_stream,
                           pdfs.PDFS_OPT_GRAPHS, pair_cap=64)
    try:
        for _ in range(2):
            got, stats, _ = pdfs.pdfs_wsc_run(ctx, 4, 1, 10, 0, 3, n_tumor=I.n_tumor)
            _same_rounds(got, exp.rounds)
            _counters_equal(stats, exp.counters, 4)
    finally:
        pdfs.pdfs_destroy(ctx)


def test_device_inputs_and_stream(pdfs):
    import torch
    I = synth.random_tiny(55, 80, 190, 70, 0.15, 3)
    T, N = I.packed()
    exp = cpu.wsc(T, N, I.n_tumor, I.n_normal, 3, 1, 10, mode="empty")
    Td = torch.from_numpy(T.view(np.int64)).cuda()
    Nd = torch.from_numpy(N.view(np.int64)).cuda()
    s = torch.cuda.Stream()
    with pdfs.Solver(Td, Nd, I.n_tumor, I.n_normal, "bound", 0, s.cuda_stream) as sv:
        got, _, _ = sv.wsc(3, 1, 10)
    _same_rounds(got, exp.rounds)


def test_resume_equals_straight_run(pdfs):
    I = synth.workload_small_h2()
    T, N = I.packed()
    with pdfs.Solver(T, N, I.n_tumor, I.n_normal, "bound") as s:
        full, _, ffinal = s.wsc(2, 1, 10)
        part, _, pfinal = s.wsc(2, 1, 10, max_rounds=9)
        rest, _, rfinal = s.wsc(2, 1, 10, initial_uncovered=pfinal)
    _same_rounds(part + rest, full)
    assert np.array_equal(rfinal, ffinal)


def test_edge_cases(pdfs):
    # no tumour mutation at all -> no combination
    T = np.zeros((10, 2), np.uint64)
    N = np.zeros((10, 1), np.uint64)
    with pdfs.Solver(T, N, 100, 30, "bound") as s:
        g, _ = s.best(2)
        assert g is None
        rounds, _, _ = s.wsc(3)
        assert rounds == []
    # h = G, duplicate rows (ties broken by the lexicographic rule)
    I = synth.random_tiny(77, 6, 80, 20, 0.7, 3)
    Td = np.repeat(I.tumor[:3], 2, axis=0)
    Nd = np.repeat(I.normal[:3], 2, axis=0)
    T, N = synth.pack_rows(Td), synth.pack_rows(Nd)
    for h in (1, 2, 3, 4, 6):
        exp = cpu.wsc(T, N, 80, 20, h, 1, 10, mode="empty")
        with pdfs.Solver(T, N, 80, 20, "bound") as s:
            got, _, _ = s.wsc(h)
        _same_rounds(got, exp.rounds)
    # no normals at all
    I = synth.random_tiny(78, 30, 100, 0, 0.3, 3)
    T, N = I.packed()
    exp = cpu.wsc(T, N, 100, 0, 3, 1, 10, mode="empty")
    with pdfs.Solver(T, None, 100, 0, "bound") as s:
        got, _, _ = s.wsc(3)
    _same_rounds(got, exp.rounds)


def test_invalid_arguments(pdfs):
    I = synth.random_tiny(79, 20, 70, 20, 0.3, 2)
    T, N = I.packed()
    bad = T.copy()
    bad[3, 1] |= np.uint64(1) << np.uint64(63)   # sample 127 > n_tumor
    with pytest.raises(pdfs.PdfsError) as e:
        pdfs.Solver(bad, N, 70, 20)
    assert e.value.code == pdfs.PDFS_ERR_INVALID_ARG
    with pdfs.Solver(T, N, 70, 20) as s:
        with pytest.raises(pdfs.PdfsError) as e:
            s.wsc(0)
        assert e.value.code == pdfs.PDFS_ERR_INVALID_ARG
        with pytest.raises(pdfs.PdfsError) as e:
            s.best(2, 1, 0)
        assert e.value.code == pdfs.PDFS_ERR_INVALID_ARG
        with pytest.raises(pdfs.PdfsError) as e:
            s.wsc(3, cap=1)
        assert e.value.code == pdfs.PDFS_ERR_TRUNCATED
