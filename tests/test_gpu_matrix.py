"""GPU parity of the matrix-core filter (FPM_UNIT_MATRIX): the filter test
F_D <= t of Eq. 1 computed as an 8-bit integer contraction on the matrix
cores.  Match sets equal the oracle's exact ones; survivor counts equal the
oracle's count of pairs with F_D <= t (t = 2k; 4k for bigrams) and the
vector-ALU path's, for occurrence, occurrence-halved, 16-bit count and
bigram fingerprints (16- and 32-bit keys), Hamming and Levenshtein,
k = 1..3, both schedules, tiles whose query and word counts are not
multiples of the pass, all pairs surviving, and full-size workloads in the
benchmark's launch configuration."""
import numpy as np
import pytest

import oracle
from paper_1711_08475_amd import datagen

pytestmark = pytest.mark.gpu

VARIANTS = {"occ": oracle.OCC, "occh": oracle.OCCH, "qgram": oracle.QGRAM, "count": oracle.COUNT}
NOMAP = np.full(256, oracle.NONE, dtype=np.uint8)


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def fpm(gpu):
    from paper_1711_08475_amd import fpm as f

    f.lib()
    return f


@pytest.fixture(scope="module")
def small():
    return datagen.workload("english_10k_q1k")


_cache = {}


def ref_match(key, d, q, metric, k):
    if (key, metric, k) not in _cache:
        _cache[(key, metric, k)] = oracle.match(d, q, metric, k)
    return _cache[(key, metric, k)]


def oracle_survivors(d, q, variant, mp, metric, k, bits=16):
    _, surv, _ = oracle.filter_stats(d, q, VARIANTS[variant], bits, NOMAP if variant == "qgram" else mp, metric, k)
    return surv


CASES = [
    ("occ", 16, oracle.HAM, 1), ("occ", 16, oracle.LEV, 1), ("occ", 16, oracle.LEV, 2), ("occ", 16, oracle.LEV, 3),
    ("occ", 16, oracle.HAM, 3), ("occh", 16, oracle.HAM, 1), ("occh", 16, oracle.HAM, 2),
    ("qgram", 16, oracle.LEV, 1), ("qgram", 16, oracle.HAM, 2), ("qgram", 16, oracle.LEV, 3),
    ("occ", 32, oracle.LEV, 1), ("occ", 32, oracle.HAM, 1), ("occ", 32, oracle.LEV, 2), ("occ", 32, oracle.LEV, 3),
    ("occh", 32, oracle.HAM, 2), ("count", 16, oracle.LEV, 1), ("count", 16, oracle.HAM, 2),
    ("qgram", 32, oracle.LEV, 1), ("qgram", 32, oracle.LEV, 2),
]


@pytest.mark.parametrize("variant,bits,metric,k", CASES)
@pytest.mark.parametrize("schedule", [0, 1])
def test_matrix_match_equals_oracle(fpm, small, variant, bits, metric, k, schedule):
    d, q = small
    say("matrix", variant, bits, metric, k, "schedule", schedule)
    ix = fpm.fpm_build_fingerprints(d, variant, bits, "common")
    got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=schedule, filter_unit="matrix"), with_stats=True)
    assert st["filter_unit"] == fpm.FPM_UNIT_MATRIX
    assert np.array_equal(got, ref_match("small", d, q, metric, k))
    surv = oracle_survivors(d, q, variant, fpm.fpm_get_map(ix), metric, k, bits)
    assert st["survivors"] == surv
    got_v, st_v = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=schedule, filter_unit="valu"),
                                with_stats=True)
    assert st_v["filter_unit"] == fpm.FPM_UNIT_VALU
    assert np.array_equal(got_v, got)
    assert (st_v["pairs_examined"], st_v["survivors"]) == (st["pairs_examined"], st["survivors"])


@pytest.mark.parametrize("qt,slab,tail", [(16, 64, 0), (48, 128, 0), (64, 64, 0), (80, 192, 0), (112, 4096, 50),
                                          (1024, 1 << 20, 0)])
@pytest.mark.parametrize("bits", [16, 32])
def test_matrix_ragged_tiles(fpm, small, qt, slab, tail, bits):
    """Tiles of 16..1024 queries and 64..1M words: passes with fewer than 64
    queries (the lane halves see 0..32 of them) and fewer than 64 (16-bit
    keys) or 32 (32-bit keys) words."""
    d, q = small
    ix = fpm.fpm_build_fingerprints(d, "occ", bits, "common")
    surv = oracle_survivors(d, q, "occ", fpm.fpm_get_map(ix), oracle.LEV, 1, bits)
    for sched in (0, 1):
        say("matrix ragged", bits, qt, slab, tail, sched)
        got, st = fpm.fpm_match(ix, q, oracle.LEV, 1, fpm.options(schedule=sched, queries_per_item=qt, slab=slab,
                                                                  tail_split=tail, filter_unit="matrix"),
                                with_stats=True)
        assert np.array_equal(got, ref_match("small", d, q, oracle.LEV, 1))
        assert st["survivors"] == surv


def test_matrix_every_pair_survives(fpm):
    """No symbol in the map: every key is 0, F_D = 0 for every pair, so every
    examined pair survives (the queue's overflow path: 2,048 survivors per
    lane mask and pass)."""
    rng = np.random.default_rng(12)
    words = [bytes(rng.integers(97, 100, size=int(rng.integers(1, 7)))) for _ in range(3001)]
    queries = [bytes(rng.integers(97, 100, size=int(rng.integers(1, 7)))) for _ in range(150)]
    d, q = datagen.to_csr(words), datagen.to_csr(queries)
    for bits in (16, 32):
        ix = fpm.fpm_build_fingerprints(d, "occ", bits, custom_map=NOMAP)
        for metric, k in [(oracle.LEV, 1), (oracle.LEV, 2), (oracle.HAM, 1)]:
            for qt, slab in [(64, 4096), (128, 64), (1024, 1 << 20)]:
                say("matrix all survive", bits, metric, k, qt, slab)
                got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=1, queries_per_item=qt, slab=slab,
                                                                      filter_unit="matrix"), with_stats=True)
                assert np.array_equal(got, oracle.match(d, q, metric, k))
                assert st["survivors"] == st["pairs_examined"]


def test_matrix_key_bits_one_at_a_time(fpm):
    """Sixteen letters, each its own field: a query and a word that differ in
    one symbol set differ in one or two key bits.  Every key position of the
    contraction (both lane halves, both nibbles of each) decides some pair,
    and the survivor count equals the oracle's."""
    rng = np.random.default_rng(5)
    letters = np.frombuffer(b"abcdefghijklmnop", np.uint8)
    words = [bytes(rng.choice(letters, int(rng.integers(1, 12)))) for _ in range(4003)]
    queries = []
    for i in range(203):
        w = bytearray(words[int(rng.integers(len(words)))])
        if w and i % 3:
            w[int(rng.integers(len(w)))] = int(rng.choice(letters))
        queries.append(bytes(w))
    d, q = datagen.to_csr(words), datagen.to_csr(queries)
    mp = np.full(256, 255, dtype=np.uint8)
    mp[letters] = np.arange(16)
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, custom_map=mp)
    for metric, k in [(oracle.LEV, 1), (oracle.HAM, 1), (oracle.LEV, 2)]:
        say("matrix sixteen letters", metric, k)
        got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=1, queries_per_item=64, slab=128,
                                                              filter_unit="matrix"), with_stats=True)
        assert np.array_equal(got, oracle.match(d, q, metric, k))
        _, surv, _ = oracle.filter_stats(d, q, oracle.OCC, 16, mp, metric, k)
        assert st["survivors"] == surv


def test_matrix_filter_pairs_equal_valu(fpm, small):
    d, q = small
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    say("matrix filter pairs")
    pairs = fpm.fpm_filter_pairs(ix, q, "lev", 1)
    fq = oracle.fingerprints(q, oracle.OCC, 16, fpm.fpm_get_map(ix))
    fw = oracle.fingerprints(d, oracle.OCC, 16, fpm.fpm_get_map(ix))
    assert np.all(oracle.fd(fq[pairs[:, 0]], fw[pairs[:, 1]], oracle.OCC, 16) <= 2)
    assert pairs.shape[0] == oracle_survivors(d, q, "occ", fpm.fpm_get_map(ix), oracle.LEV, 1)


def test_matrix_unit_errors(fpm, small):
    d, q = small
    say("matrix errors")
    for variant, bits in [("count", 32), ("pos", 16), ("pos", 32), ("combo", 32)]:
        ix = fpm.fpm_build_fingerprints(d, variant, bits, "common")
        with pytest.raises(fpm.FpmError) as e:
            fpm.fpm_match(ix, q, "ham", 1, fpm.options(filter_unit="matrix"))
        assert e.value.status == fpm.FPM_EUNSUPPORTED
        # auto falls back to the vector ALUs
        assert np.array_equal(fpm.fpm_match(ix, q, "ham", 1), ref_match("small", d, q, oracle.HAM, 1))
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_match(ix, q, "lev", 1, fpm.options(filter_unit="matrix", bound="asym"))
    assert e.value.status == fpm.FPM_EUNSUPPORTED
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_match(ix, q, "lev", 1, fpm.options(filter_unit=3))
    assert e.value.status == fpm.FPM_EINVAL
    # empty query list, a single empty query, one word
    assert fpm.fpm_match(ix, datagen.to_csr([]), "lev", 1, fpm.options(filter_unit="matrix")).shape[0] == 0
    one = datagen.to_csr([b""])
    assert np.array_equal(fpm.fpm_match(ix, one, "lev", 1, fpm.options(filter_unit="matrix")),
                          oracle.match(d, one, oracle.LEV, 1))
    ix1 = fpm.fpm_build_fingerprints(datagen.to_csr([b"abc"]), "occ", 16, "common")
    qs = datagen.to_csr([b"abc", b"abd", b"ab", b"abcd", b"xyz", b"ab", b"bca"])
    assert np.array_equal(fpm.fpm_match(ix1, qs, "lev", 1, fpm.options(filter_unit="matrix")),
                          oracle.match(datagen.to_csr([b"abc"]), qs, oracle.LEV, 1))


def test_matrix_full_size_sampled_parity(fpm):
    """english_1m_q10k with the learned grouping (occ16, Lev k = 1) in the
    benchmark's launch configuration (batched, persistent, hipGraph, the
    tiles of the tuning table's headline entry): the matrix and vector paths
    return the same match list and survivor count, and sampled query rows
    equal the oracle's."""
    import json
    import os

    import torch

    from paper_1711_08475_amd import learn

    table = json.load(open(os.path.join(os.path.dirname(learn.__file__), "tuned.json")))
    entry = dict(table["english_1m_q10k|occ16|lev1|learned|matrix"])
    entry.pop("inflight", None)

    d, q = datagen.workload("english_1m_q10k")
    nq = q[1].size - 1
    mp, _ = learn.load_map("english_1m_q10k_occ16_k1")
    say("matrix full size")
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, custom_map=mp)
    qb = torch.from_numpy(q[0].copy()).cuda()
    qo = torch.from_numpy(q[1].view(np.int64).copy()).cuda()
    torch.cuda.synchronize()
    res = {}
    for unit in ("matrix", "valu"):
        plan = fpm.fpm_plan_create(ix, nq, int(q[1][-1]), oracle.LEV, 1, fpm.options(**entry, filter_unit=unit))
        fpm.fpm_plan_run(plan, qb.data_ptr(), qo.data_ptr(), nq)
        res[unit] = (fpm.fpm_plan_copy_matches(plan), fpm.fpm_plan_result(plan)[2])
        del plan
    assert np.array_equal(res["matrix"][0], res["valu"][0])
    assert res["matrix"][1]["survivors"] == res["valu"][1]["survivors"]
    sample = np.random.default_rng(17).choice(nq, 48, replace=False)
    sample.sort()
    ref = oracle.match(d, datagen.take_csr(q, sample), oracle.LEV, 1, length_pruned=True)
    ref[:, 0] = sample[ref[:, 0]]
    got = res["matrix"][0]
    assert np.array_equal(got[np.isin(got[:, 0], sample)], ref)


def test_matrix_thirty_two_letters(fpm):
    """Thirty-two letters, each its own field of a 32-bit key: pairs that
    differ in one symbol exercise every key position of both chained
    products (bits 0..15 with the threshold, bits 16..31)."""
    rng = np.random.default_rng(8)
    letters = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz012345", np.uint8)
    words = [bytes(rng.choice(letters, int(rng.integers(1, 12)))) for _ in range(4007)]
    queries = []
    for i in range(211):
        w = bytearray(words[int(rng.integers(len(words)))])
        if w and i % 3:
            w[int(rng.integers(len(w)))] = int(rng.choice(letters))
        queries.append(bytes(w))
    d, q = datagen.to_csr(words), datagen.to_csr(queries)
    mp = np.full(256, 255, dtype=np.uint8)
    mp[letters] = np.arange(32)
    ix = fpm.fpm_build_fingerprints(d, "occ", 32, custom_map=mp)
    for metric, k in [(oracle.LEV, 1), (oracle.HAM, 1), (oracle.LEV, 2)]:
        say("matrix thirty-two letters", metric, k)
        got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=1, queries_per_item=64, slab=128,
                                                              filter_unit="matrix"), with_stats=True)
        assert np.array_equal(got, oracle.match(d, q, metric, k))
        _, surv, _ = oracle.filter_stats(d, q, oracle.OCC, 32, mp, metric, k)
        assert st["survivors"] == surv


def test_matrix_url_full_size_sampled_parity(fpm):
    """url_1m_q10k with its learned grouping (occ32, Lev k = 2) in the
    batched launch configuration: matrix and vector paths agree on the match
    list and survivor count, and sampled query rows equal the oracle's."""
    import torch

    from paper_1711_08475_amd import learn

    d, q = datagen.workload("url_1m_q10k")
    nq = q[1].size - 1
    mp, _ = learn.load_map("url_1m_q10k_occ32_k2")
    say("matrix url full size")
    ix = fpm.fpm_build_fingerprints(d, "occ", 32, custom_map=mp)
    qb = torch.from_numpy(q[0].copy()).cuda()
    qo = torch.from_numpy(q[1].view(np.int64).copy()).cuda()
    torch.cuda.synchronize()
    res = {}
    for unit in ("matrix", "valu"):
        plan = fpm.fpm_plan_create(ix, nq, int(q[1][-1]), oracle.LEV, 2,
                                   fpm.options(schedule=1, queries_per_item=128, slab=1024, filter_unit=unit))
        fpm.fpm_plan_run(plan, qb.data_ptr(), qo.data_ptr(), nq)
        res[unit] = (fpm.fpm_plan_copy_matches(plan), fpm.fpm_plan_result(plan)[2])
        del plan
    assert np.array_equal(res["matrix"][0], res["valu"][0])
    assert res["matrix"][1]["survivors"] == res["valu"][1]["survivors"]
    sample = np.random.default_rng(19).choice(nq, 24, replace=False)
    sample.sort()
    ref = oracle.match(d, datagen.take_csr(q, sample), oracle.LEV, 2, length_pruned=True)
    ref[:, 0] = sample[ref[:, 0]]
    got = res["matrix"][0]
    assert np.array_equal(got[np.isin(got[:, 0], sample)], ref)


def test_matrix_plan_graph_replays_and_batches_in_flight(fpm, small):
    """One batched plan (hipGraph on) replayed several times on two query
    batches (the graph is re-captured when the batch changes and replayed
    otherwise), with eager device work and synchronisations between the
    replays; then two plans on their own streams taking alternate batches
    without waiting for each other.  Every result equals the oracle's."""
    import torch

    d, q = small
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    half = datagen.take_csr(q, np.arange(0, q[1].size - 1, 2))
    batches = []
    for qq in (q, half):
        qb = torch.from_numpy(qq[0].copy()).cuda()
        qo = torch.from_numpy(qq[1].view(np.int64).copy()).cuda()
        batches.append((qq, qb, qo, qq[1].size - 1, oracle.match(d, qq, oracle.LEV, 1)))
    torch.cuda.synchronize()
    nq_max, bytes_max = q[1].size - 1, int(q[1][-1])
    opts = fpm.options(schedule=1, filter_unit="matrix", queries_per_item=64, slab=512)
    plan = fpm.fpm_plan_create(ix, nq_max, bytes_max, oracle.LEV, 1, opts)
    x = torch.ones(512, 512, device="cuda")
    for i, b in enumerate([0, 0, 0, 1, 1, 0, 1, 0]):
        say("matrix graph replay", i, "batch", b)
        _, qb, qo, nq, ref = batches[b]
        fpm.fpm_plan_run(plan, qb.data_ptr(), qo.data_ptr(), nq)
        x = (x @ x).clamp_(max=1.0)  # eager work on the default stream between replays
        torch.cuda.synchronize()
        got = fpm.fpm_plan_copy_matches(plan)
        assert np.array_equal(got, ref)
        assert fpm.fpm_plan_result(plan)[2]["filter_unit"] == fpm.FPM_UNIT_MATRIX
    del plan
    plans = [fpm.fpm_plan_create(ix, nq_max, bytes_max, oracle.LEV, 1, opts) for _ in range(2)]
    for rnd in range(3):
        say("matrix plans in flight", rnd)
        for j, p in enumerate(plans):
            _, qb, qo, nq, _ = batches[(j + rnd) % 2]
            fpm.fpm_plan_run(p, qb.data_ptr(), qo.data_ptr(), nq)
        for j, p in enumerate(plans):
            assert np.array_equal(fpm.fpm_plan_copy_matches(p), batches[(j + rnd) % 2][4])


@pytest.mark.parametrize("which", ["url", "mixed"])
@pytest.mark.parametrize("variant,metric,k", [("occ", oracle.LEV, 1), ("occ", oracle.LEV, 2), ("occ", oracle.HAM, 1),
                                              ("occh", oracle.HAM, 2), ("qgram", oracle.LEV, 1)])
def test_matrix_long_strings(fpm, which, variant, metric, k):
    """URL-like strings (lengths 20-120, shared host and path vocabulary) and
    a mixed English / URL set through the matrix filter with 16-bit keys:
    match sets and survivor counts equal the oracle's."""
    d, q = datagen.url_workload(4000, 300, 5, 0.3, (1, 2)) if which == "url" else \
        datagen.mixed_workload(2000, 2000, 300, 9)
    say("matrix long strings", which, variant, metric, k)
    ix = fpm.fpm_build_fingerprints(d, variant, 16, "mixed" if which == "url" else "common")
    for sched in (0, 1):
        got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=sched, filter_unit="matrix"),
                                with_stats=True)
        assert np.array_equal(got, ref_match(which, d, q, metric, k))
        assert st["survivors"] == oracle_survivors(d, q, variant, fpm.fpm_get_map(ix), metric, k)


def test_matrix_autotune_keeps_the_unit(fpm, small):
    """fpm_autotune searches tiles around a base whose filter unit is the
    matrix cores: the returned options keep the unit, and a plan built from
    them runs on the matrix cores and matches the oracle."""
    import torch

    d, q = small
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    qb = torch.from_numpy(q[0].copy()).cuda()
    qo = torch.from_numpy(q[1].view(np.int64).copy()).cuda()
    torch.cuda.synchronize()
    nq = q[1].size - 1
    say("matrix autotune")
    best, rows = fpm.fpm_autotune(ix, qb.data_ptr(), qo.data_ptr(), nq, int(q[1][-1]), "lev", 1, 1,
                                  base=fpm.options(filter_unit="matrix"))
    assert rows and best.filter_unit == fpm.FPM_UNIT_MATRIX
    plan = fpm.fpm_plan_create(ix, nq, int(q[1][-1]), "lev", 1, best)
    fpm.fpm_plan_run(plan, qb.data_ptr(), qo.data_ptr(), nq)
    assert fpm.fpm_plan_result(plan)[2]["filter_unit"] == fpm.FPM_UNIT_MATRIX
    assert np.array_equal(fpm.fpm_plan_copy_matches(plan), ref_match("small", d, q, oracle.LEV, 1))
