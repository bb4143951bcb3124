"""The allocation-free round (pdfs_best_combo_noalloc) against pdfs_best_combo
on the same context and against the oracle: every result field, the per-depth
counters of the empty-intersection walk, two calls in a row with the second on
a smaller cohort, and the size limits.  Calls go through the C ABI."""
import numpy as np
import pytest

from oracle import cpu
from paper_2603_16721_amd import synth
from tests.helpers import mask_of_bits

pytestmark = pytest.mark.gpu

KEYS = ("genes", "sorted_idx", "tp", "fp", "tn", "score_num", "score_den", "uncovered_before")

COHORTS = [
    # seed, G, n_tumor, n_normal, density, h  (the second is the smaller one)
    (901, 1000, 300, 120, 0.025, 4),
    (902, 400, 100, 50, 0.08, 3),
    (903, 90, 70, 20, 0.2, 2),
    (904, 60, 64, 0, 0.3, 1),
]


@pytest.fixture(scope="module")
def pdfs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_16721_amd import pdfs as binding
    return binding


def _masks(I, seed):
    rng = np.random.default_rng(seed)
    return [None, mask_of_bits(rng.random(I.n_tumor) < 0.55)]


def _check(pdfs, I, mode, seed):
    T, N = I.packed()
    perm = cpu.order(T, N)
    with pdfs.Solver(T, N, I.n_tumor, I.n_normal, mode) as s:
        for U in _masks(I, seed):
            ref, ref_st = s.best(I.h, I.alpha_p, I.alpha_q, U)
            got, got_st = s.best_noalloc(I.h, I.alpha_p, I.alpha_q, U)
            exp = cpu.best(T, N, I.n_tumor, I.n_normal, I.h, I.alpha_p, I.alpha_q, U=U,
                           mode="empty", perm=perm)
            assert (got is None) == (ref is None) == (not exp.found)
            if got is None:
                continue
            for k in KEYS:
                assert got[k] == ref[k], (k, got, ref)
            assert tuple(got["sorted_idx"]) == exp.sorted_idx
            assert (got["tp"], got["fp"]) == (exp.tp, exp.fp)
            if mode == "empty":
                for l in range(1, I.h + 1):
                    assert got_st["visited"][l] == ref_st["visited"][l] == exp.counters["visited"][l]
                    assert got_st["nonempty"][l] == ref_st["nonempty"][l] == \
                        exp.counters["nonempty"][l]


@pytest.mark.parametrize("mode", ["empty", "bound"])
def test_noalloc_matches_best_combo(pdfs, mode):
    """Calls in a row on cohorts of decreasing size (each later call smaller
    than the one before) share the static array and must each equal the
    allocating round and the oracle."""
    for k, case in enumerate(COHORTS):
        seed, G, nt, nn, d, h = case
        I = synth.random_tiny(seed, G, nt, nn, d, h)
        _check(pdfs, I, mode, seed + 7 * k)


def test_noalloc_repeat_after_larger(pdfs):
    """The smaller cohort again after the larger one on the same context pair:
    nothing of the earlier call's contents leaks into the later one."""
    big = synth.random_tiny(*COHORTS[0][:5], COHORTS[0][5])
    small = synth.random_tiny(*COHORTS[1][:5], COHORTS[1][5])
    Tb, Nb = big.packed()
    Ts, Ns = small.packed()
    with pdfs.Solver(Tb, Nb, big.n_tumor, big.n_normal, "empty") as sb, \
            pdfs.Solver(Ts, Ns, small.n_tumor, small.n_normal, "empty") as ss:
        first, _ = ss.best_noalloc(small.h, 1, 10)
        sb.best_noalloc(big.h, 1, 10)
        again, _ = ss.best_noalloc(small.h, 1, 10)
        ref, _ = ss.best(small.h, 1, 10)
        assert first == again == ref


def test_noalloc_limits(pdfs):
    """h above 4 and a workspace larger than the static array are refused
    with a clear error before any work."""
    I = synth.random_tiny(905, 30, 40, 10, 0.3, 5)
    T, N = I.packed()
    with pdfs.Solver(T, N, I.n_tumor, I.n_normal, "empty") as s:
        with pytest.raises(pdfs.PdfsError) as e:
            s.best_noalloc(5, 1, 10)
        assert e.value.code == pdfs.PDFS_ERR_UNSUPPORTED
    # 60000 genes with one tumour mutation each at 1280 tumour samples: the
    # unpacked rows alone (60000 x 1280 bytes) exceed the array
    G, nt = 60000, 1280
    T = np.zeros((G, nt // 64), dtype=np.uint64)
    smp = np.arange(G) % nt
    T[np.arange(G), smp // 64] = np.uint64(1) << (smp % 64).astype(np.uint64)
    N = np.zeros((G, 1), dtype=np.uint64)
    with pdfs.Solver(T, N, nt, 1, "empty") as s:
        with pytest.raises(pdfs.PdfsError) as e:
            s.best_noalloc(2, 1, 10)
        assert e.value.code == pdfs.PDFS_ERR_UNSUPPORTED
        assert "exceeds" in str(e.value)
