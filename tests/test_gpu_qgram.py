"""GPU parity of the bigram (q = 2) fingerprints: fingerprints equal the
oracle's, match sets equal the oracle's exact ones and survivor counts equal
the oracle's count of pairs with F_D <= 4k, for Hamming and Levenshtein,
k = 1..3, both schedules, English-like, URL-like and ragged inputs."""
import numpy as np
import pytest

import oracle
from paper_1711_08475_amd import datagen

pytestmark = pytest.mark.gpu

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


@pytest.fixture(scope="module")
def url_small():
    return datagen.url_workload(4000, 300, 5, 0.3, (1, 2))


@pytest.mark.parametrize("bits", [16, 32])
def test_bigram_fingerprints_equal_oracle(fpm, small, url_small, bits):
    for name, (d, q) in (("english", small), ("url", url_small)):
        say("bigram fingerprints", name, bits)
        ix = fpm.fpm_build_fingerprints(d, "qgram", bits, "common")
        assert np.array_equal(fpm.fpm_get_fingerprints(ix), oracle.fingerprints(d, oracle.QGRAM, bits, NOMAP))
        assert np.array_equal(fpm.fpm_fingerprints(ix, q), oracle.fingerprints(q, oracle.QGRAM, bits, NOMAP))


_cache = {}


def ref(key, d, q, metric, k):
    if (key, metric, k) not in _cache:
        _cache[(key, metric, k)] = oracle.match(d, q, metric, k)
    return _cache[(key, metric, k)]


@pytest.mark.parametrize("bits,metric,k", [(16, oracle.LEV, 1), (32, oracle.LEV, 1), (32, oracle.HAM, 1),
                                           (32, oracle.LEV, 2), (16, oracle.HAM, 2), (32, oracle.LEV, 3)])
@pytest.mark.parametrize("schedule", [0, 1])
def test_bigram_match_equals_oracle(fpm, small, bits, metric, k, schedule):
    d, q = small
    say("bigram match", bits, metric, k, schedule)
    ix = fpm.fpm_build_fingerprints(d, "qgram", bits, "common")
    got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=schedule), with_stats=True)
    assert np.array_equal(got, ref("small", d, q, metric, k))
    ex, surv, _ = oracle.filter_stats(d, q, oracle.QGRAM, bits, NOMAP, metric, k)
    assert (st["pairs_examined"], st["survivors"]) == (ex, surv)


@pytest.mark.parametrize("metric,k", [(oracle.LEV, 1), (oracle.LEV, 2)])
def test_bigram_long_strings(fpm, url_small, metric, k):
    d, q = url_small
    say("bigram url", metric, k)
    ix = fpm.fpm_build_fingerprints(d, "qgram", 32, "common")
    got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=1), with_stats=True)
    assert np.array_equal(got, ref("url", d, q, metric, k))
    ex, surv, _ = oracle.filter_stats(d, q, oracle.QGRAM, 32, NOMAP, metric, k)
    assert (st["pairs_examined"], st["survivors"]) == (ex, surv)


def test_bigram_ragged_tiles_and_errors(fpm):
    rng = np.random.default_rng(17)
    words = [bytes(rng.integers(97, 101, size=int(rng.integers(0, 9)))) for _ in range(2999)]
    queries = [bytes(rng.integers(97, 101, size=int(rng.integers(0, 9)))) for _ in range(93)]
    d, q = datagen.to_csr(words), datagen.to_csr(queries)
    ix = fpm.fpm_build_fingerprints(d, "qgram", 16, "common")
    for metric, k in [(oracle.LEV, 1), (oracle.HAM, 2), (oracle.LEV, 3)]:
        r = oracle.match(d, q, metric, k)
        for sched, qt, slab in [(0, 16, 64), (1, 32, 128), (1, 1024, 1 << 20)]:
            say("bigram ragged", metric, k, sched, qt, slab)
            got = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=sched, queries_per_item=qt, slab=slab))
            assert np.array_equal(got, r)
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_match(ix, q, "lev", 1, fpm.options(bound="asym"))
    assert e.value.status == fpm.FPM_EUNSUPPORTED
