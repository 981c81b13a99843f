"""GPU parity of the asymmetric bound (FPM_BOUND_ASYM): match sets equal the
oracle's exact ones, and the filter's survivor counts equal the oracle's
count of pairs with max(excess(q, w), excess(w, q)) <= k, for every key
family (thermometer-extended 16-bit keys, 32-bit and 64-bit keys) and both
schedules; popcount-range skipping is exercised with small tiles and spread
popcounts."""
import numpy as np
import pytest

import oracle
from paper_1711_08475_amd import datagen

pytestmark = pytest.mark.gpu

VARIANT_NAMES = {oracle.OCC: "occ", oracle.COUNT: "count", oracle.POS: "pos", oracle.OCCH: "occh"}


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


ASYM_CASES = [
    # 16-bit occ / occh: thermometer-extended keys
    (oracle.OCC, 16, oracle.HAM, 1), (oracle.OCC, 16, oracle.LEV, 1), (oracle.OCC, 16, oracle.LEV, 2),
    (oracle.OCCH, 16, oracle.HAM, 1), (oracle.OCCH, 16, oracle.HAM, 2),
    # 32-bit keys
    (oracle.OCC, 32, oracle.LEV, 1), (oracle.OCC, 32, oracle.HAM, 2), (oracle.COUNT, 16, oracle.LEV, 1),
    (oracle.COUNT, 16, oracle.HAM, 1), (oracle.OCCH, 32, oracle.HAM, 2),
    # 64-bit keys
    (oracle.COUNT, 32, oracle.LEV, 1), (oracle.COUNT, 32, oracle.LEV, 2),
    # k = 3
    (oracle.OCC, 16, oracle.LEV, 3), (oracle.OCC, 32, oracle.LEV, 3), (oracle.COUNT, 32, oracle.HAM, 3),
]


@pytest.mark.parametrize("variant,bits,metric,k", ASYM_CASES)
@pytest.mark.parametrize("schedule", [0, 1])
def test_asym_match_equals_oracle(fpm, small, variant, bits, metric, k, schedule):
    d, q = small
    say("asym", VARIANT_NAMES[variant], bits, metric, k, "schedule", schedule)
    ix = fpm.fpm_build_fingerprints(d, variant, bits, "common")
    got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=schedule, bound="asym"), with_stats=True)
    ref = ref_match("small", d, q, metric, k)
    assert np.array_equal(got, ref)
    mp = fpm.fpm_get_map(ix)
    ex, surv = oracle.filter_stats_asym(d, q, variant, bits, mp, metric, k)
    ex_fd, surv_fd, _ = oracle.filter_stats(d, q, variant, bits, mp, metric, k)
    assert st["pairs_examined"] == ex == ex_fd
    assert st["survivors"] == surv
    assert surv <= surv_fd
    # the paper's rule on the same index is unchanged
    _, st_fd = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=schedule), with_stats=True)
    assert st_fd["survivors"] == surv_fd


@pytest.mark.parametrize("variant,bits,metric,k", [
    (oracle.OCC, 32, oracle.LEV, 1), (oracle.OCC, 32, oracle.LEV, 2), (oracle.COUNT, 32, oracle.LEV, 1),
    (oracle.OCC, 16, oracle.LEV, 2), (oracle.COUNT, 32, oracle.HAM, 1),
])
@pytest.mark.parametrize("which", ["url", "mixed"])
def test_asym_long_strings(fpm, variant, bits, metric, k, which):
    d, q = datagen.url_workload(4000, 300, 5, 0.3, (1, 2)) if which == "url" else \
        datagen.mixed_workload(2000, 2000, 300, 9)
    say("asym", which, VARIANT_NAMES[variant], bits, metric, k)
    ix = fpm.fpm_build_fingerprints(d, variant, bits, "mixed" if which == "url" else "common")
    got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=1, bound="asym"), with_stats=True)
    assert np.array_equal(got, ref_match(which, d, q, metric, k))
    ex, surv = oracle.filter_stats_asym(d, q, variant, bits, fpm.fpm_get_map(ix), metric, k)
    assert (st["pairs_examined"], st["survivors"]) == (ex, surv)


def spread_workload(seed):
    """Words over 16 letters, each its own field, lengths 1..16: occurrence
    popcounts run from 1 to 16 inside every length block, so tiles of one
    length bucket cover many popcounts; bucket sizes are ragged."""
    rng = np.random.default_rng(seed)
    letters = np.frombuffer(b"abcdefghijklmnop", np.uint8)
    words = []
    for _ in range(5003):
        n = int(rng.integers(1, 17))
        distinct = int(rng.integers(1, min(n, 16) + 1))
        pool = rng.choice(letters, distinct, replace=False)
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


@pytest.mark.parametrize("variant,bits", [(oracle.OCC, 16), (oracle.OCC, 32), (oracle.COUNT, 32)])
def test_asym_popcount_skips_small_tiles(fpm, variant, bits):
    """Tiles of 16 queries x 64 words and ragged buckets, with popcounts spread
    over 1..16 in each length block: whole tiles and 32 x 128 passes are
    skipped by popcount range, and nothing that matches is lost."""
    d, q, mp = spread_workload(31)
    if variant == oracle.COUNT:
        mp = mp.copy()
        mp[mp != 255] = mp[mp != 255] % oracle.num_fields(variant, bits)
    for metric, k in [(oracle.LEV, 1), (oracle.LEV, 2), (oracle.HAM, 1)]:
        ref = oracle.match(d, q, metric, k)
        ex, surv = oracle.filter_stats_asym(d, q, variant, bits, mp, metric, k)
        ix = fpm.fpm_build_fingerprints(d, variant, bits, custom_map=mp)
        for sched, qt, slab, tail in [(0, 16, 64, 0), (1, 16, 64, 0), (1, 32, 128, 50), (1, 64, 4096, 0),
                                      (1, 1024, 1 << 20, 0)]:
            say("asym spread", VARIANT_NAMES[variant], bits, metric, k, sched, qt, slab, tail)
            got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=sched, queries_per_item=qt, slab=slab,
                                                                  tail_split=tail, bound="asym"), with_stats=True)
            assert np.array_equal(got, ref)
            assert (st["pairs_examined"], st["survivors"]) == (ex, surv)


def test_asym_everything_survives(fpm):
    """No symbol in the map: every fingerprint and popcount is 0, nothing is
    skipped and every examined pair survives."""
    rng = np.random.default_rng(12)
    words = [bytes(rng.integers(97, 100, size=int(rng.integers(1, 7)))) for _ in range(3001)]
    queries = [bytes(rng.integers(97, 100, size=int(rng.integers(1, 7)))) for _ in range(77)]
    d, q = datagen.to_csr(words), datagen.to_csr(queries)
    none = np.full(256, 255, dtype=np.uint8)
    for variant, bits in [("occ", 16), ("count", 32), ("occ", 32)]:
        ix = fpm.fpm_build_fingerprints(d, variant, bits, custom_map=none)
        for metric, k in [(oracle.LEV, 1), (oracle.LEV, 2), (oracle.HAM, 1)]:
            say("asym all survive", variant, bits, metric, k)
            got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=1, queries_per_item=16, slab=64,
                                                                  bound="asym"), with_stats=True)
            assert np.array_equal(got, oracle.match(d, q, metric, k))
            assert st["survivors"] == st["pairs_examined"]


def test_asym_edges_and_errors(fpm, small):
    d, q = small
    say("asym errors")
    ix_pos = fpm.fpm_build_fingerprints(d, "pos", 16, "common")
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_match(ix_pos, q, "ham", 1, fpm.options(bound="asym"))
    assert e.value.status == fpm.FPM_EUNSUPPORTED
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_match(ix, q, "lev", 1, fpm.options(bound=2))
    assert e.value.status == fpm.FPM_EINVAL
    # brute force has no filter: the bound is ignored
    got = fpm.fpm_match(ix, q, "lev", 1, fpm.options(schedule=fpm.FPM_SCHED_BRUTE, bound="asym"))
    assert np.array_equal(got, ref_match("small", d, q, oracle.LEV, 1))
    # empty query list, a single empty query, a single word
    assert fpm.fpm_match(ix, datagen.to_csr([]), "lev", 1, fpm.options(bound="asym")).shape[0] == 0
    one = datagen.to_csr([b""])
    got = fpm.fpm_match(ix, one, "lev", 1, fpm.options(bound="asym"))
    assert np.array_equal(got, oracle.match(d, one, oracle.LEV, 1))
    ix1 = fpm.fpm_build_fingerprints(datagen.to_csr([b"abc"]), "occ", 16, "common")
    qs = datagen.to_csr([b"abc", b"abd", b"ab", b"abcd", b"xyz", b"ab", b"bca"])
    got = fpm.fpm_match(ix1, qs, "lev", 1, fpm.options(bound="asym"))
    assert np.array_equal(got, oracle.match(datagen.to_csr([b"abc"]), qs, oracle.LEV, 1))


@pytest.mark.parametrize("name,variant,bits,metric,k", [
    ("english_1m_q10k", "occ", 16, oracle.LEV, 1), ("url_1m_q10k", "occ", 32, oracle.LEV, 2),
    ("mixed_2m_q64k", "occ", 32, oracle.LEV, 2),
])
def test_asym_full_size_sampled_parity(fpm, name, variant, bits, metric, k):
    """Full size in the benchmark's launch configuration (batched, persistent,
    hipGraph) under the asymmetric bound: equal to the GPU brute force on
    every query, and sampled rows equal to the oracle's."""
    import torch

    d, q = datagen.workload(name)
    nq = q[1].size - 1
    say("asym full size", name, variant, bits, metric, k)
    ix = fpm.fpm_build_fingerprints(d, variant, bits, "common")
    qb = torch.from_numpy(q[0].copy()).cuda()
    qo = torch.from_numpy(q[1].view(np.int64).copy()).cuda()
    torch.cuda.synchronize()
    res = {}
    for sched in (fpm.FPM_SCHED_BATCHED, fpm.FPM_SCHED_BRUTE):
        plan = fpm.fpm_plan_create(ix, nq, int(q[1][-1]), metric, k, fpm.options(schedule=sched, bound="asym"))
        fpm.fpm_plan_run(plan, qb.data_ptr(), qo.data_ptr(), nq)
        res[sched] = fpm.fpm_plan_copy_matches(plan)
        del plan
    assert np.array_equal(res[fpm.FPM_SCHED_BATCHED], res[fpm.FPM_SCHED_BRUTE])
    sample = np.random.default_rng(13).choice(nq, 48, replace=False)
    sample.sort()
    ref = oracle.match(d, datagen.take_csr(q, sample), metric, k, length_pruned=True)
    ref[:, 0] = sample[ref[:, 0]]
    got = res[fpm.FPM_SCHED_BATCHED]
    assert np.array_equal(got[np.isin(got[:, 0], sample)], ref)
