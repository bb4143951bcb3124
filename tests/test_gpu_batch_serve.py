"""Batched and served front ends: every result equals the oracle's (and the
plain path's), alone or in a mix; admission by device memory; repeated graph
replays give the same results."""
import json
import os
import time

import pytest

from paper_2603_16721_amd import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def pdfs():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_16721_amd import pdfs as binding
    return binding


def _golden(kind):
    with open(os.path.join(HERE, "golden", f"{kind}_oracle.json")) as f:
        return json.load(f)["instances"]


def _compact(rounds):
    return [[*r["genes"], r["tp"], r["fp"], r["score_num"]] for r in rounds]


def _batch(pdfs, idx, autotune=False, mode="bound", path="one_launch", pair_cap=0):
    insts = [synth.batched_instance(i) for i in idx]
    packed = [(I.packed(), I) for I in insts]
    b = pdfs.pdfs_batch_create([(T, N, I.n_tumor, I.n_normal) for (T, N), I in packed], mode,
                               autotune=autotune, path=path, pair_cap=pair_cap)
    return b, insts


def test_batched_all_instances_match_oracle(pdfs):
    gold = _golden("batched")
    b, insts = _batch(pdfs, range(32))
    try:
        res, st = pdfs.pdfs_batch_run(b, [I.h for I in insts], 1, 10,
                                      n_tumors=[I.n_tumor for I in insts])
        for i, I in enumerate(insts):
            assert _compact(res[i]) == gold[str(i)]["rounds"], i
        # the same batch again: replays of the captured rounds
        res2, _ = pdfs.pdfs_batch_run(b, [I.h for I in insts], 1, 10,
                                      n_tumors=[I.n_tumor for I in insts])
        assert [_compact(r) for r in res2] == [_compact(r) for r in res]
    finally:
        pdfs.pdfs_batch_destroy(b)
    assert st["rounds"] == sum(len(gold[str(i)]["rounds"]) for i in range(32))


def test_batched_autotune_and_empty_mode_same_results(pdfs, tmp_path, monkeypatch):
    """Tuned (work-item shape, seed size, split depth) and untuned batches give
    the oracle's results; the tuner's choices land in its JSON cache."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("PDFS_TUNE_CACHE", str(cache))
    gold = _golden("batched")
    idx = [0, 5, 7, 10, 12, 16, 20, 24, 28]   # small instances: quick in empty mode too
    for mode, tune in (("bound", True), ("empty", True), ("empty", False)):
        b, insts = _batch(pdfs, idx, autotune=tune, mode=mode)
        try:
            res, _ = pdfs.pdfs_batch_run(b, [I.h for I in insts], 1, 10,
                                         n_tumors=[I.n_tumor for I in insts])
        finally:
            pdfs.pdfs_batch_destroy(b)
        for k, i in enumerate(idx):
            assert _compact(res[k]) == gold[str(i)]["rounds"], (mode, i)
    entries = json.loads(cache.read_text())
    assert entries and all(e["split"] in (2, 3) and e["chunk"] > 0 for e in entries)
    assert {e["mode"] for e in entries} == {1, 2}


@pytest.mark.parametrize("path", ["streams", "auto"])
@pytest.mark.parametrize("mode", ["bound", "empty"])
def test_batched_streams_path_matches_oracle(pdfs, mode, path):
    """The stream-parallel batched runs (each instance's own launches), and the
    path a batch takes by default for its mode, give the oracle's results."""
    gold = _golden("batched")
    idx = [2, 5, 12, 20]
    b, insts = _batch(pdfs, idx, mode=mode, path=path)
    try:
        res, _ = pdfs.pdfs_batch_run(b, [I.h for I in insts], 1, 10,
                                     n_tumors=[I.n_tumor for I in insts])
    finally:
        pdfs.pdfs_batch_destroy(b)
    for k, i in enumerate(idx):
        assert _compact(res[k]) == gold[str(i)]["rounds"], (mode, i)


@pytest.mark.parametrize("path", ["one_launch", "streams"])
@pytest.mark.parametrize("mode", ["bound", "empty"])
def test_batched_pair_list_regrowth(pdfs, mode, path):
    """Every instance starts with a 64-pair list: the rounds that emit more
    grow their instance's list and run again (one launch per round step over
    all instances, or each instance on the batch's streams); the results are
    the oracle's."""
    gold = _golden("batched")
    idx = [0, 3, 5, 12, 16, 21]
    b, insts = _batch(pdfs, idx, mode=mode, path=path, pair_cap=64)
    try:
        res, _ = pdfs.pdfs_batch_run(b, [I.h for I in insts], 1, 10,
                                     n_tumors=[I.n_tumor for I in insts])
    finally:
        pdfs.pdfs_batch_destroy(b)
    for k, i in enumerate(idx):
        assert _compact(res[k]) == gold[str(i)]["rounds"], (mode, i)


def test_batched_empty_counters_equal_plain(pdfs):
    """One launch per round step over several instances, empty-intersection
    walk (two-phase depth 4 for the h = 4 ones): the summed per-depth counts
    equal the plain path's on each instance alone, so every instance's walk
    is complete and nothing is counted twice."""
    idx = [0, 5, 10, 12, 16, 20]   # h = 3 and h = 4 (10, 16) cohorts
    b, insts = _batch(pdfs, idx, mode="empty")
    try:
        res, st = pdfs.pdfs_batch_run(b, [I.h for I in insts], 1, 10,
                                      n_tumors=[I.n_tumor for I in insts])
    finally:
        pdfs.pdfs_batch_destroy(b)
    vis = [0] * 10
    ne = [0] * 10
    for k, I in enumerate(insts):
        T, N = I.packed()
        with pdfs.Solver(T, N, I.n_tumor, I.n_normal, "empty") as s:
            plain, pst, _ = s.wsc(I.h, 1, 10)
        assert _compact(res[k]) == _compact(plain), idx[k]
        vis = [a + b for a, b in zip(vis, pst["visited"])]
        ne = [a + b for a, b in zip(ne, pst["nonempty"])]
    assert st["visited"] == vis and st["nonempty"] == ne


def test_batched_equals_plain_path(pdfs):
    for i in (1, 9, 30):
        I = synth.batched_instance(i)
        T, N = I.packed()
        with pdfs.Solver(T, N, I.n_tumor, I.n_normal, "bound") as s:
            plain, _, _ = s.wsc(I.h, 1, 10)
        b, insts = _batch(pdfs, [i])
        try:
            res, _ = pdfs.pdfs_batch_run(b, [I.h], 1, 10, n_tumors=[I.n_tumor])
        finally:
            pdfs.pdfs_batch_destroy(b)
        assert _compact(res[0]) == _compact(plain)


def _serve(pdfs, js, max_active=8, one_at_a_time=False, budget=0):
    srv = pdfs.pdfs_server_create("bound", 0, budget, max_active)
    out = {}
    try:
        reqs = {j: synth.served_request(j) for j in js}
        tickets = {}
        for j in js:
            I = reqs[j]
            T, N = I.packed()
            tickets[j] = pdfs.pdfs_server_submit(srv, T, N, I.n_tumor, I.n_normal, I.h, 1, 10)
            if one_at_a_time:
                while True:
                    r = pdfs.pdfs_server_poll(srv, tickets[j], cap=I.n_tumor + 1)
                    if r is not None:
                        out[j] = r
                        break
                    time.sleep(0.001)
        deadline = time.time() + 300
        while len(out) < len(js):
            for j in js:
                if j in out:
                    continue
                r = pdfs.pdfs_server_poll(srv, tickets[j], cap=reqs[j].n_tumor + 1)
                if r is not None:
                    out[j] = r
            assert time.time() < deadline, "served requests did not finish"
            time.sleep(0.002)
    finally:
        pdfs.pdfs_server_destroy(srv)
    return out


def test_served_sample_matches_oracle(pdfs):
    gold = _golden("served")
    js = [int(j) for j in gold]
    out = _serve(pdfs, js)
    for j in js:
        rounds, lat = out[j]
        assert _compact(rounds) == gold[str(j)]["rounds"], j
        assert lat > 0


def test_served_alone_equals_mix(pdfs):
    js = [3, 11, 42, 77, 105, 160, 199]
    alone = _serve(pdfs, js, max_active=1, one_at_a_time=True)
    mix = _serve(pdfs, js, max_active=8)
    for j in js:
        assert _compact(alone[j][0]) == _compact(mix[j][0]), j


def test_server_admission_by_memory(pdfs):
    I = synth.served_request(0)
    T, N = I.packed()
    srv = pdfs.pdfs_server_create("bound", 0, 1 << 20, 4)   # 1 MiB budget: too small
    try:
        with pytest.raises(pdfs.PdfsError) as e:
            pdfs.pdfs_server_submit(srv, T, N, I.n_tumor, I.n_normal, I.h, 1, 10)
        assert e.value.code == pdfs.PDFS_ERR_OUT_OF_MEMORY
    finally:
        pdfs.pdfs_server_destroy(srv)
    # a budget that holds one or two of these requests: the rest queue, all finish
    js = [1, 2, 4]
    out = _serve(pdfs, js, max_active=4, budget=1 << 30)
    assert sorted(out) == js
    with pytest.raises(pdfs.PdfsError):
        srv = pdfs.pdfs_server_create("bound", 0, 0, 2)
        try:
            pdfs.pdfs_server_poll(srv, 12345)
        finally:
            pdfs.pdfs_server_destroy(srv)


# Deeper combinations through the front ends: one batch (and one server)
# mixing h = 3, 5 and 6 cohorts; every result equals the oracle's.
DEEP_MIX = [
    # seed, G, n_tumor, n_normal, density, h
    (301, 40, 100, 30, 0.25, 5),
    (302, 30, 150, 50, 0.35, 6),
    (303, 60, 120, 40, 0.2, 3),
]
ROUND_KEYS = ("sorted_idx", "tp", "fp", "score_num")


def _deep_mix():
    from oracle import cpu
    insts = [synth.random_tiny(s, G, nt, nn, d, h) for s, G, nt, nn, d, h in DEEP_MIX]
    exp = []
    for I in insts:
        T, N = I.packed()
        exp.append(cpu.wsc(T, N, I.n_tumor, I.n_normal, I.h, 1, 10, mode="empty").rounds)
    return insts, exp


def _same(got, exp):
    assert len(got) == len(exp)
    for g, e in zip(got, exp):
        assert all(g[k] == e[k] for k in ROUND_KEYS), (g, e)


@pytest.mark.parametrize("mode", ["bound", "empty"])
def test_batched_deep_mix_matches_oracle(pdfs, mode):
    insts, exp = _deep_mix()
    b = pdfs.pdfs_batch_create([(*I.packed(), I.n_tumor, I.n_normal) for I in insts], mode)
    try:
        for _ in range(2):   # the second run replays captured rounds
            res, _ = pdfs.pdfs_batch_run(b, [I.h for I in insts], 1, 10,
                                         n_tumors=[I.n_tumor for I in insts])
            for r, e in zip(res, exp):
                _same(r, e)
    finally:
        pdfs.pdfs_batch_destroy(b)


def test_served_deep_mix_matches_oracle(pdfs):
    insts, exp = _deep_mix()
    srv = pdfs.pdfs_server_create("bound", 0, 0, 4)
    try:
        tickets = [pdfs.pdfs_server_submit(srv, *I.packed(), I.n_tumor, I.n_normal, I.h, 1, 10)
                   for I in insts]
        out = [None] * len(insts)
        deadline = time.time() + 120
        while any(o is None for o in out):
            for k, t in enumerate(tickets):
                if out[k] is None:
                    r = pdfs.pdfs_server_poll(srv, t, cap=insts[k].n_tumor + 1)
                    if r is not None:
                        out[k] = r[0]
            assert time.time() < deadline, "served requests did not finish"
            time.sleep(0.002)
    finally:
        pdfs.pdfs_server_destroy(srv)
    for r, e in zip(out, exp):
        _same(r, e)
