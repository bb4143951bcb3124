"""Held-out coverage report (accuracy protocol of Sec. IV): split, coverage
count and the learned-on-train / scored-on-test flow."""
import numpy as np
import pytest

from oracle import cpu
from paper_2603_16721_amd import heldout, synth


def test_split_is_a_partition():
    rng = np.random.default_rng(3)
    tr, te = heldout.split_samples(101, 0.25, rng)
    assert len(te) == 25 and len(tr) == 76
    assert np.array_equal(np.sort(np.concatenate([tr, te])), np.arange(101))
    assert len(np.intersect1d(tr, te)) == 0


def test_coverage_hand_example():
    # genes x samples; sample 0 has genes 0,1; sample 1 gene 2; sample 2 none;
    # sample 3 genes 0,2
    bits = np.array([[1, 0, 0, 1],
                     [1, 0, 0, 0],
                     [0, 1, 0, 1]], dtype=bool)
    assert heldout.covered([(0, 1)], bits).tolist() == [True, False, False, False]
    assert heldout.covered([(0, 1), (2,)], bits).tolist() == [True, True, False, True]
    assert heldout.covered([(0, 2)], bits).tolist() == [False, False, False, True]
    assert heldout.covered([], bits).tolist() == [False] * 4
    rep = heldout.coverage_report([(0, 1), (2,)], bits, bits[:, :2])
    assert (rep["TC"], rep["TT"], rep["NC"], rep["NT"]) == (3, 4, 2, 2)
    assert rep["sensitivity"] == 0.75 and rep["specificity"] == 0.0


@pytest.mark.parametrize("seed,h", [(31, 2), (32, 3), (33, 4)])
def test_train_coverage_equals_greedy_tp(seed, h):
    # the greedy counts only uncovered tumours each round, so the learned
    # combinations cover exactly sum(TP) training tumours
    I = synth.random_tiny(seed, 60, 120, 40, 0.12, h)
    parts = heldout.split_cohort(I, 0.25, seed)
    t_tr, n_tr = parts["train"]
    T, N = synth.pack_rows(t_tr), synth.pack_rows(n_tr)
    res = cpu.wsc(T, N, t_tr.shape[1], n_tr.shape[1], h, 1, 10, mode="bound")
    combos = [r["genes"] for r in res.rounds]
    rep = heldout.coverage_report(combos, t_tr, n_tr)
    assert rep["TC"] == sum(r["tp"] for r in res.rounds)
    # each combination's FP on the training normals is its normal coverage
    for r in res.rounds:
        assert int(heldout.covered([r["genes"]], n_tr).sum()) == r["fp"]


@pytest.mark.gpu
@pytest.mark.parametrize("name", ["tiny3", "tiny4"])
def test_learn_on_gpu_matches_oracle(name):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_16721_amd import pdfs
    h = 3 if name == "tiny3" else 4
    I = synth.random_tiny(40 + h, 90, 160, 60, 0.1, h)
    out = heldout.learn_and_evaluate(pdfs, I, 0.25, seed=7)
    parts = heldout.split_cohort(I, 0.25, 7)
    t_tr, n_tr = parts["train"]
    exp = cpu.wsc(synth.pack_rows(t_tr), synth.pack_rows(n_tr), t_tr.shape[1], n_tr.shape[1],
                  h, 1, 10, mode="empty")
    assert out["combos"] == [r["genes"] for r in exp.rounds]
    assert out["train"]["TC"] == out["train_tp_sum"]
    assert out["train"]["TT"] + out["test"]["TT"] == 160
    assert out["train"]["NT"] + out["test"]["NT"] == 60


@pytest.mark.gpu
def test_learn_literal_tn_on_gpu_matches_oracle():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_16721_amd import pdfs
    I = synth.random_tiny(45, 80, 160, 60, 0.1, 3)
    out = heldout.learn_and_evaluate(pdfs, I, 0.25, seed=9, tn_literal=True)
    t_tr, n_tr = heldout.split_cohort(I, 0.25, 9)["train"]
    exp = cpu.wsc(synth.pack_rows(t_tr), synth.pack_rows(n_tr), t_tr.shape[1], n_tr.shape[1],
                  3, 1, 10, mode="empty", tn="literal")
    assert out["combos"] == [r["genes"] for r in exp.rounds]
    # under the literal reading a combination's FP is the normals carrying any gene
    for r in exp.rounds:
        carried = np.zeros(n_tr.shape[1], dtype=bool)
        for g in r["genes"]:
            carried |= n_tr[g]
        assert int(carried.sum()) == r["fp"]
