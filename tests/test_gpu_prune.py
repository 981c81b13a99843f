"""GPU parity of popcount pruning (fpm_options.pop_prune = FPM_PRUNE_ON):
the paper's rule over popcount-ordered blocks skips groups of pairs whose
key popcounts lie more than the threshold apart (F_D >= |pq - pw|).  Match
sets equal the oracle's, survivor and examined-pair counts equal the
oracle's F_D <= t counts (pruning removes only pairs the filter would
reject), for every key family it is offered for, with small and ragged
tiles, graph replays and two plans in flight; errors where it does not
apply."""
import numpy as np
import pytest

import oracle
from paper_1711_08475_amd import datagen

pytestmark = pytest.mark.gpu

NAMES = {oracle.OCC: "occ", oracle.COUNT: "count", oracle.OCCH: "occh", oracle.QGRAM: "qgram"}


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def fpm(gpu):
    from paper_1711_08475_amd import fpm as f

    f.lib()
    return f


_cache = {}


def ref_match(key, d, q, metric, k):
    if (key, metric, k) not in _cache:
        _cache[(key, metric, k)] = oracle.match(d, q, metric, k)
    return _cache[(key, metric, k)]


CASES = [
    (oracle.OCC, 16, oracle.HAM, 1), (oracle.OCC, 16, oracle.LEV, 1), (oracle.OCC, 16, oracle.LEV, 2),
    (oracle.OCC, 32, oracle.LEV, 1), (oracle.OCC, 32, oracle.LEV, 3), (oracle.OCCH, 16, oracle.HAM, 1),
    (oracle.COUNT, 16, oracle.LEV, 1), (oracle.COUNT, 32, oracle.LEV, 1), (oracle.COUNT, 32, oracle.HAM, 2),
    (oracle.QGRAM, 16, oracle.LEV, 1), (oracle.QGRAM, 32, oracle.LEV, 2),
]


MATRIX_OK = {(oracle.OCC, 16), (oracle.OCC, 32), (oracle.OCCH, 16), (oracle.COUNT, 16), (oracle.QGRAM, 16),
             (oracle.QGRAM, 32)}


@pytest.mark.parametrize("variant,bits,metric,k", CASES)
@pytest.mark.parametrize("which", ["english", "mixed"])
@pytest.mark.parametrize("unit", ["valu", "matrix"])
def test_pruned_match_equals_oracle(fpm, variant, bits, metric, k, which, unit):
    if unit == "matrix" and (variant, bits) not in MATRIX_OK:
        pytest.skip("the matrix cores take 16- and 32-bit keys whose F_D is the popcount of their XOR")
    d, q = datagen.workload("english_10k_q1k") if which == "english" else \
        datagen.mixed_workload(3000, 3000, 400, 17)
    say("prune", unit, which, NAMES[variant], bits, metric, k)
    ix = fpm.fpm_build_fingerprints(d, variant, bits, "common")
    got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=1, queries_per_item=64, slab=512,
                                                          pop_prune="on", filter_unit=unit), with_stats=True)
    assert st["filter_unit"] == fpm.UNITS[unit]
    assert np.array_equal(got, ref_match(which, d, q, metric, k))
    ex, surv, _ = oracle.filter_stats(d, q, variant, bits, fpm.fpm_get_map(ix), metric, k)
    assert (st["pairs_examined"], st["survivors"]) == (ex, surv)
    assert st["pairs_filtered"] <= st["pairs_examined"]
    _, st_off = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=1, queries_per_item=64, slab=512),
                              with_stats=True)
    assert st_off["survivors"] == surv and st_off["pairs_filtered"] == st_off["pairs_examined"] == ex


def spread_workload(seed):
    """Words over 16 letters, each its own field, lengths 1..16: occurrence
    popcounts run from 1 to 16 inside every length block; ragged buckets."""
    rng = np.random.default_rng(seed)
    letters = np.frombuffer(b"abcdefghijklmnop", np.uint8)
    words = []
    for _ in range(5003):
        n = int(rng.integers(1, 17))
        pool = rng.choice(letters, int(rng.integers(1, min(n, 16) + 1)), replace=False)
        words.append(bytes(rng.choice(pool, n)))
    queries = []
    for i in range(301):
        w = bytearray(words[int(rng.integers(len(words)))])
        if i % 2 and w:
            w[int(rng.integers(len(w)))] = int(rng.choice(letters))
        queries.append(bytes(w))
    mp = np.full(256, 255, dtype=np.uint8)
    mp[letters] = np.arange(16)
    return datagen.to_csr(words), datagen.to_csr(queries), mp


@pytest.mark.parametrize("variant,bits,unit", [(oracle.OCC, 16, "valu"), (oracle.OCC, 32, "valu"),
                                               (oracle.COUNT, 32, "valu"), (oracle.OCC, 16, "matrix"),
                                               (oracle.OCC, 32, "matrix")])
def test_pruning_skips_tiles_and_passes(fpm, variant, bits, unit):
    """Popcounts spread over 1..16 in each length block: with tiles from
    16 x 64 to 1024 x 1M, whole items and 32 x 128 passes are skipped (with
    the narrow tiles, fewer pairs are filtered than examined) and nothing
    that survives is lost."""
    d, q, mp = spread_workload(41)
    if variant == oracle.COUNT:
        mp = mp.copy()
        mp[mp != 255] = mp[mp != 255] % oracle.num_fields(variant, bits)
    ix = fpm.fpm_build_fingerprints(d, variant, bits, custom_map=mp)
    for metric, k in [(oracle.LEV, 1), (oracle.LEV, 2), (oracle.HAM, 1)]:
        ref = oracle.match(d, q, metric, k)
        ex, surv, _ = oracle.filter_stats(d, q, variant, bits, mp, metric, k)
        for qt, slab, tail in [(16, 64, 0), (32, 128, 50), (64, 4096, 0), (1024, 1 << 20, 0), (48, 192, 25)]:
            say("prune spread", unit, NAMES[variant], bits, metric, k, qt, slab, tail)
            got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=1, queries_per_item=qt, slab=slab,
                                                                  tail_split=tail, pop_prune="on",
                                                                  filter_unit=unit), with_stats=True)
            assert np.array_equal(got, ref)
            assert (st["pairs_examined"], st["survivors"]) == (ex, surv)
            assert st["pairs_filtered"] <= st["pairs_examined"]
            if qt <= 32 and variant == oracle.OCC:
                # tiles narrower than a length block's popcount spread (count
                # keys: popcount ~ length, nothing to prune inside a block)
                assert st["pairs_filtered"] < st["pairs_examined"]


def test_pruning_when_everything_survives(fpm):
    """No symbol in the map: every key and popcount is 0, nothing is pruned
    and every examined pair survives."""
    rng = np.random.default_rng(13)
    words = [bytes(rng.integers(97, 100, size=int(rng.integers(1, 7)))) for _ in range(3001)]
    queries = [bytes(rng.integers(97, 100, size=int(rng.integers(1, 7)))) for _ in range(77)]
    d, q = datagen.to_csr(words), datagen.to_csr(queries)
    none = np.full(256, 255, dtype=np.uint8)
    for variant, bits in [("occ", 16), ("count", 32), ("occ", 32)]:
        ix = fpm.fpm_build_fingerprints(d, variant, bits, custom_map=none)
        for metric, k in [(oracle.LEV, 1), (oracle.HAM, 1)]:
            say("prune all survive", variant, bits, metric, k)
            got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=1, queries_per_item=16, slab=64,
                                                                  pop_prune="on"), with_stats=True)
            assert np.array_equal(got, oracle.match(d, q, metric, k))
            assert st["survivors"] == st["pairs_examined"] == st["pairs_filtered"]


@pytest.mark.parametrize("unit", ["valu", "matrix"])
def test_pruned_plan_replays_and_two_in_flight(fpm, unit):
    """Device-scheduled plans with pruning, replayed through their graphs and
    run two at a time on their own streams, with a smaller second batch: every
    run returns the oracle's list."""
    import torch

    d, q = datagen.mixed_workload(3000, 3000, 500, 23)
    ix = fpm.fpm_build_fingerprints(d, "occ", 32, "common")
    ref = oracle.match(d, q, oracle.LEV, 1)
    nq = q[1].size - 1
    qb = torch.from_numpy(q[0].copy()).cuda()
    qo = torch.from_numpy(q[1].view(np.int64).copy()).cuda()
    torch.cuda.synchronize()
    opts = fpm.options(schedule=1, queries_per_item=128, slab=1024, pop_prune="on", filter_unit=unit)
    plans = [fpm.fpm_plan_create(ix, nq, int(q[1][-1]), "lev", 1, opts) for _ in range(2)]
    for r in range(3):
        say("prune replay", unit, r)
        for p in plans:
            fpm.fpm_plan_run(p, qb.data_ptr(), qo.data_ptr(), nq)
        for p in plans:
            assert np.array_equal(fpm.fpm_plan_copy_matches(p), ref)
    half = nq // 2
    sub = (q[0][: int(q[1][half])], q[1][: half + 1])
    say("prune smaller batch")
    fpm.fpm_plan_run(plans[0], qb.data_ptr(), qo.data_ptr(), half)
    assert np.array_equal(fpm.fpm_plan_copy_matches(plans[0]), oracle.match(d, sub, oracle.LEV, 1))


def test_pruning_errors(fpm):
    d, q = datagen.workload("english_10k_q1k")
    say("prune errors")
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    ix_pos = fpm.fpm_build_fingerprints(d, "pos", 16, "common")
    for o, index in [(fpm.options(schedule=1, pop_prune="on"), ix_pos),
                     (fpm.options(schedule=0, pop_prune="on"), ix),
                     (fpm.options(schedule=2, pop_prune="on"), ix),
                     (fpm.options(schedule=1, pop_prune="on", bound="asym"), ix)]:
        with pytest.raises(fpm.FpmError) as e:
            fpm.fpm_match(index, q, "ham", 1, o)
        assert e.value.status == fpm.FPM_EUNSUPPORTED
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_match(ix, q, "lev", 1, fpm.options(pop_prune=2))
    assert e.value.status == fpm.FPM_EINVAL
    # empty query list and a single empty query
    assert fpm.fpm_match(ix, datagen.to_csr([]), "lev", 1, fpm.options(schedule=1, pop_prune="on")).shape[0] == 0
    one = datagen.to_csr([b""])
    got = fpm.fpm_match(ix, one, "lev", 1, fpm.options(schedule=1, pop_prune="on"))
    assert np.array_equal(got, oracle.match(d, one, oracle.LEV, 1))
