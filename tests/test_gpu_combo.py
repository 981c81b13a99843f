"""GPU parity of the combined occurrence + count fingerprint: fingerprints
equal the oracle's, match sets equal the oracle's exact ones and survivor
counts equal the oracle's count of pairs whose larger part F_D is <= 2k, for
Hamming and Levenshtein, k = 1..3, both schedules, English-like, URL-like and
ragged inputs."""
import numpy as np
import pytest

import oracle
from paper_1711_08475_amd import datagen

pytestmark = pytest.mark.gpu


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


def ref(key, d, q, metric, k):
    if (key, metric, k) not in _cache:
        _cache[(key, metric, k)] = oracle.match(d, q, metric, k)
    return _cache[(key, metric, k)]


@pytest.mark.parametrize("bits", [16, 32])
@pytest.mark.parametrize("symset", ["common", "mixed"])
def test_combined_fingerprints_equal_oracle(fpm, small, bits, symset):
    d, q = small
    say("combined fingerprints", bits, symset)
    ix = fpm.fpm_build_fingerprints(d, "combo", bits, symset)
    mp = fpm.fpm_get_map(ix)
    assert np.array_equal(mp, oracle.select_symbols(oracle.histogram(d), oracle.COMBO, bits,
                                                    oracle.COMMON if symset == "common" else oracle.MIXED))
    assert np.array_equal(fpm.fpm_get_fingerprints(ix), oracle.fingerprints(d, oracle.COMBO, bits, mp))
    assert np.array_equal(fpm.fpm_fingerprints(ix, q), oracle.fingerprints(q, oracle.COMBO, bits, mp))


@pytest.mark.parametrize("bits,metric,k", [(16, oracle.LEV, 1), (32, oracle.LEV, 1), (32, oracle.HAM, 1),
                                           (32, oracle.LEV, 2), (16, oracle.HAM, 2), (32, oracle.LEV, 3)])
@pytest.mark.parametrize("schedule", [0, 1])
def test_combined_match_equals_oracle(fpm, small, bits, metric, k, schedule):
    d, q = small
    say("combined match", bits, metric, k, schedule)
    ix = fpm.fpm_build_fingerprints(d, "combo", bits, "common")
    got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=schedule), with_stats=True)
    assert np.array_equal(got, ref("small", d, q, metric, k))
    ex, surv, _ = oracle.filter_stats(d, q, oracle.COMBO, bits, fpm.fpm_get_map(ix), metric, k)
    assert (st["pairs_examined"], st["survivors"]) == (ex, surv)


def test_combined_long_strings_ragged_and_errors(fpm):
    d, q = datagen.url_workload(4000, 300, 5, 0.3, (1, 2))
    say("combined url")
    ix = fpm.fpm_build_fingerprints(d, "combo", 32, "mixed")
    for metric, k in [(oracle.LEV, 1), (oracle.LEV, 2)]:
        got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=1), with_stats=True)
        assert np.array_equal(got, oracle.match(d, q, metric, k))
        ex, surv, _ = oracle.filter_stats(d, q, oracle.COMBO, 32, fpm.fpm_get_map(ix), metric, k)
        assert (st["pairs_examined"], st["survivors"]) == (ex, surv)
    rng = np.random.default_rng(23)
    words = [bytes(rng.integers(97, 103, size=int(rng.integers(0, 9)))) for _ in range(2999)]
    queries = [bytes(rng.integers(97, 103, size=int(rng.integers(0, 9)))) for _ in range(93)]
    d, q = datagen.to_csr(words), datagen.to_csr(queries)
    ix = fpm.fpm_build_fingerprints(d, "combo", 16, "common")
    for metric, k in [(oracle.LEV, 1), (oracle.HAM, 2), (oracle.LEV, 3)]:
        r = oracle.match(d, q, metric, k)
        for sched, qt, slab in [(0, 16, 64), (1, 32, 128), (1, 1024, 1 << 20)]:
            say("combined ragged", metric, k, sched, qt, slab)
            got = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=sched, queries_per_item=qt, slab=slab))
            assert np.array_equal(got, r)
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_match(ix, q, "lev", 1, fpm.options(bound="asym"))
    assert e.value.status == fpm.FPM_EUNSUPPORTED
