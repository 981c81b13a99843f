"""GPU parity: the HIP path against the CPU oracle, element by element, on the
same seeded inputs.  Every comparison is exact (integer work)."""
import numpy as np
import pytest

import oracle
from paper_1711_08475_amd import datagen

pytestmark = pytest.mark.gpu

VARIANT_NAMES = {oracle.OCC: "occ", oracle.COUNT: "count", oracle.POS: "pos", oracle.OCCH: "occh", oracle.QGRAM: "qgram",
                 oracle.COMBO: "combo"}


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def fpm(gpu):
    from paper_1711_08475_amd import fpm as f

    f.lib()
    return f


@pytest.fixture(scope="module")
def small():
    """10,000 English-like words (lengths 3-15) x 1,000 queries, half near-matches."""
    return datagen.workload("english_10k_q1k")


_oracle_cache = {}


def oracle_match(key, d, q, metric, k):
    if (key, metric, k) not in _oracle_cache:
        _oracle_cache[(key, metric, k)] = oracle.match(d, q, metric, k)
    return _oracle_cache[(key, metric, k)]


# ---------------------------------------------------------------- symbols, fps

@pytest.mark.parametrize("variant", [oracle.OCC, oracle.COUNT, oracle.POS, oracle.OCCH])
@pytest.mark.parametrize("bits", [16, 32])
@pytest.mark.parametrize("symset", [oracle.COMMON, oracle.RARE, oracle.MIXED])
def test_symbol_map_and_fingerprints(fpm, small, variant, bits, symset):
    d, q = small
    say("fingerprints", VARIANT_NAMES[variant], bits, symset)
    ref_map = oracle.select_symbols(oracle.histogram(d), variant, bits, symset)
    assert np.array_equal(fpm.fpm_select_symbols(d, variant, bits, symset), ref_map)
    ix = fpm.fpm_build_fingerprints(d, variant, bits, symset)
    assert np.array_equal(fpm.fpm_get_map(ix), ref_map)
    assert np.array_equal(fpm.fpm_get_fingerprints(ix), oracle.fingerprints(d, variant, bits, ref_map))
    assert np.array_equal(fpm.fpm_fingerprints(ix, q), oracle.fingerprints(q, variant, bits, ref_map))


@pytest.mark.parametrize("extra,lead", [(0, 0), (1, 0), (7, 3), (15, 0), (16, 13), (17, 1), (33, 16)])
def test_symbol_selection_counts_every_byte(fpm, extra, lead):
    """Symbol counts 1..48 differ by one between neighbours, so one byte
    missed or counted twice -- in the unaligned head or tail of the byte range
    or in its 16-byte groups -- changes the rare, common or mixed map.  The
    total length runs through several residues mod 16, and `lead` bytes
    before offsets[0] (outside every string) must not be counted."""
    rng = np.random.default_rng(300 + extra)
    counts = np.arange(1, 49)
    pool = np.repeat(np.arange(65, 65 + 48, dtype=np.uint8), counts)
    pool = np.concatenate([pool, np.full(100 + extra, ord("z"), dtype=np.uint8)])
    pool = rng.permutation(pool)
    cuts = [0]
    while cuts[-1] < pool.size:
        cuts.append(min(pool.size, cuts[-1] + int(rng.integers(1, 21))))
    junk = np.full(lead, 66, dtype=np.uint8)  # a counted symbol, so counting it would show
    d = (np.concatenate([junk, pool]), np.array(cuts, dtype=np.uint64) + np.uint64(lead))
    hist = oracle.histogram(d)
    assert hist[66] == 2 and hist[ord("z")] == 100 + extra
    say("byte histogram", extra, lead)
    for variant, bits in [(oracle.OCC, 32), (oracle.OCC, 16), (oracle.COUNT, 32)]:
        for symset in (oracle.COMMON, oracle.RARE, oracle.MIXED):
            ref = oracle.select_symbols(hist, variant, bits, symset)
            assert np.array_equal(fpm.fpm_select_symbols(d, variant, bits, symset), ref), (variant, bits, symset)


def test_url_alphabet_fingerprints(fpm):
    d, q = datagen.url_workload(3000, 100, 5)
    for variant, bits in [(oracle.OCC, 32), (oracle.COUNT, 32), (oracle.POS, 32), (oracle.OCC, 16)]:
        say("url fingerprints", VARIANT_NAMES[variant], bits)
        ix = fpm.fpm_build_fingerprints(d, variant, bits, "mixed")
        m = oracle.select_symbols(oracle.histogram(d), variant, bits, oracle.MIXED)
        assert np.array_equal(fpm.fpm_get_fingerprints(ix), oracle.fingerprints(d, variant, bits, m))


def test_custom_many_to_one_map(fpm, small):
    d, q = small
    rng = np.random.default_rng(4)
    m = np.full(256, 255, dtype=np.uint8)
    m[97:123] = rng.integers(0, 16, size=26)
    m[ord("q")] = 255
    say("custom map")
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, custom_map=m)
    assert np.array_equal(fpm.fpm_get_fingerprints(ix), oracle.fingerprints(d, oracle.OCC, 16, m))
    got = fpm.fpm_match(ix, q, "lev", 1)
    assert np.array_equal(got, oracle_match("small", d, q, oracle.LEV, 1))


# ------------------------------------------------------------------ matching

CASES = [
    # (variant, bits, metric, k)
    (oracle.OCC, 16, oracle.HAM, 1), (oracle.OCC, 16, oracle.LEV, 1), (oracle.OCC, 16, oracle.LEV, 2),
    (oracle.OCC, 32, oracle.LEV, 1), (oracle.OCC, 32, oracle.HAM, 2),
    (oracle.COUNT, 16, oracle.LEV, 1), (oracle.COUNT, 16, oracle.HAM, 1), (oracle.COUNT, 32, oracle.LEV, 1),
    (oracle.COUNT, 32, oracle.LEV, 2),
    (oracle.POS, 16, oracle.HAM, 1), (oracle.POS, 32, oracle.HAM, 1), (oracle.POS, 16, oracle.HAM, 2),
    (oracle.OCCH, 16, oracle.HAM, 1), (oracle.OCCH, 32, oracle.HAM, 2),
    # k = 3 (larger k, Section 5)
    (oracle.OCC, 16, oracle.LEV, 3), (oracle.OCC, 32, oracle.HAM, 3), (oracle.COUNT, 32, oracle.LEV, 3),
    (oracle.POS, 16, oracle.HAM, 3), (oracle.OCCH, 32, oracle.HAM, 3),
]


@pytest.mark.parametrize("variant,bits,metric,k", CASES)
@pytest.mark.parametrize("schedule", [0, 1])
def test_match_equals_oracle(fpm, small, variant, bits, metric, k, schedule):
    d, q = small
    say("match", VARIANT_NAMES[variant], bits, "ham" if metric == 0 else "lev", k, "schedule", schedule)
    ix = fpm.fpm_build_fingerprints(d, variant, bits, "common")
    got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=schedule), with_stats=True)
    ref = oracle_match("small", d, q, metric, k)
    assert np.array_equal(got, ref)
    # filter counters against the oracle's F_D counts
    m = fpm.fpm_get_map(ix)
    ex, surv, _ = oracle.filter_stats(d, q, variant, bits, m, metric, k)
    assert st["pairs_examined"] == ex
    assert st["survivors"] == surv
    assert st["matches"] == ref.shape[0]
    assert st["pairs_logical"] == (d[1].size - 1) * (q[1].size - 1)


@pytest.mark.parametrize("metric,k", [(oracle.HAM, 1), (oracle.LEV, 1), (oracle.LEV, 2), (oracle.HAM, 2),
                                      (oracle.LEV, 3), (oracle.HAM, 3)])
def test_bruteforce_equals_oracle(fpm, small, metric, k):
    d, q = small
    say("brute force", metric, k)
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=fpm.FPM_SCHED_BRUTE), with_stats=True)
    assert np.array_equal(got, oracle_match("small", d, q, metric, k))
    assert st["survivors"] == st["pairs_examined"]


@pytest.mark.parametrize("variant,bits,metric,k", [(oracle.OCC, 16, oracle.LEV, 1), (oracle.COUNT, 32, oracle.LEV, 2),
                                                   (oracle.POS, 16, oracle.HAM, 1), (oracle.QGRAM, 32, oracle.LEV, 1),
                                                   (oracle.COMBO, 32, oracle.LEV, 2), (oracle.OCCH, 32, oracle.HAM, 3)])
def test_filter_survivor_set(fpm, small, variant, bits, metric, k):
    """The set of pairs the filter keeps equals {length-compatible pairs with
    F_D <= threshold (2k; bigrams 4k)} computed from the oracle's
    fingerprints and F_D."""
    d, q = small
    q = datagen.take_csr(q, np.arange(200))
    say("survivors", VARIANT_NAMES.get(variant, variant), bits, metric, k)
    ix = fpm.fpm_build_fingerprints(d, variant, bits, "common")
    got = fpm.fpm_filter_pairs(ix, q, metric, k)
    mp = fpm.fpm_get_map(ix)
    fq, fw = oracle.fingerprints(q, variant, bits, mp), oracle.fingerprints(d, variant, bits, mp)
    lq, lw = datagen.csr_lengths(q), datagen.csr_lengths(d)
    rows = []
    for i in range(lq.size):
        gap = np.abs(lw - lq[i])
        cand = np.nonzero(gap == 0 if metric == oracle.HAM else gap <= k)[0]
        f = oracle.fd(np.full(cand.size, fq[i], dtype=np.uint32), fw[cand], variant, bits)
        keep = cand[f <= oracle.threshold(variant, k)]
        rows.append(np.stack([np.full(keep.size, i), keep], axis=1))
    ref = np.concatenate(rows).astype(np.uint32)
    assert np.array_equal(got, ref)


def test_verify_pairs(fpm, small):
    d, q = small
    rng = np.random.default_rng(8)
    pairs = np.stack([rng.integers(0, q[1].size - 1, 5000), rng.integers(0, d[1].size - 1, 5000)], 1).astype(np.uint32)
    ref_pairs = oracle_match("small", d, q, oracle.LEV, 2)[:, :2]
    pairs = np.concatenate([pairs, ref_pairs])
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    pairs = np.concatenate([pairs, oracle_match("small", d, q, oracle.LEV, 3)[:, :2]])
    for metric, k in [(oracle.LEV, 1), (oracle.LEV, 2), (oracle.HAM, 1), (oracle.HAM, 2), (oracle.LEV, 3),
                      (oracle.HAM, 3)]:
        say("verify pairs", metric, k)
        got = fpm.fpm_verify_pairs(ix, q, pairs, metric, k)
        ref = oracle.pair_dist(d, q, pairs, metric)
        assert np.array_equal(got, np.minimum(ref, k + 1))


# ---------------------------------------------------------------- edge cases

def test_edge_cases(fpm):
    words = [b"", b"a", b"ab", b"ba", b"abc", b"x" * 255, b"x" * 254 + b"y", b"x" * 253, b"", b"aaaa", b"aaaa"]
    queries = [b"", b"a", b"b", b"abc", b"x" * 255, b"x" * 254, b"aaaa", b"aaab", b"zzzzzzzz"]
    d, q = datagen.to_csr(words), datagen.to_csr(queries)
    for variant, bits, metric, k in [(oracle.OCC, 16, oracle.LEV, 1), (oracle.OCC, 32, oracle.LEV, 2),
                                     (oracle.COUNT, 16, oracle.HAM, 2), (oracle.POS, 32, oracle.HAM, 1)]:
        for sched in (0, 1, 2):
            say("edge", VARIANT_NAMES[variant], bits, metric, k, sched)
            ix = fpm.fpm_build_fingerprints(d, variant, bits, "common")
            got = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=sched))
            assert np.array_equal(got, oracle.match(d, q, metric, k))


def test_empty_inputs(fpm):
    d = datagen.to_csr([b"abc", b"abd"])
    e = datagen.to_csr([])
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    say("empty queries")
    assert fpm.fpm_match(ix, e, "lev", 1).shape == (0, 3)
    say("empty dictionary")
    ix0 = fpm.fpm_build_fingerprints(e, "occ", 16, "common")
    assert fpm.fpm_match(ix0, d, "lev", 1).shape == (0, 3)
    for variant, bits in [("occ", 16), ("count", 32), ("qgram", 32), ("combo", 32)]:
        say("empty dictionary", variant, bits)
        ix0 = fpm.fpm_build_fingerprints(e, variant, bits, "common")
        assert fpm.fpm_match(ix0, d, "lev", 3).shape == (0, 3)
        if variant in ("occ", "count"):
            assert fpm.fpm_match(ix0, d, "lev", 1, fpm.options(bound="asym")).shape == (0, 3)
            assert fpm.fpm_match(ix, e, "lev", 1, fpm.options(bound="asym")).shape == (0, 3)


def test_everything_survives_and_ragged_buckets(fpm):
    """A map with no symbols makes every fingerprint 0, so every examined pair
    survives: the queues fill on every pass.  Bucket sizes are not multiples
    of 64 or of the tile sizes."""
    rng = np.random.default_rng(12)
    words = [bytes(rng.integers(97, 100, size=int(rng.integers(1, 7)))) for _ in range(3001)]
    queries = [bytes(rng.integers(97, 100, size=int(rng.integers(1, 7)))) for _ in range(77)]
    d, q = datagen.to_csr(words), datagen.to_csr(queries)
    none = np.full(256, 255, dtype=np.uint8)
    for metric, k in [(oracle.LEV, 1), (oracle.LEV, 2), (oracle.HAM, 1), (oracle.LEV, 3)]:
        ref = oracle.match(d, q, metric, k)
        for sched, qt, slab, tail in [(0, 16, 64, 0), (1, 32, 128, 0), (1, 1024, 1 << 20, 0), (0, 64, 16384, 0),
                                      (1, 16, 64, 99), (1, 64, 256, 50), (1, 32, 128, 100)]:
            say("all survive", metric, k, sched, qt, slab, tail)
            ix = fpm.fpm_build_fingerprints(d, "occ", 16, custom_map=none)
            got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=sched, queries_per_item=qt, slab=slab,
                                                                  tail_split=tail), with_stats=True)
            assert np.array_equal(got, ref)
            assert st["survivors"] == st["pairs_examined"]


def test_match_buffer_growth(fpm, small):
    d, q = small
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    for sched in (0, 1):
        say("tiny match buffer", sched)
        got = fpm.fpm_match(ix, q, "lev", 2, fpm.options(schedule=sched, match_capacity=7))
        assert np.array_equal(got, oracle_match("small", d, q, oracle.LEV, 2))


def test_errors(fpm, small):
    d, q = small
    ix_pos = fpm.fpm_build_fingerprints(d, "pos", 16, "common")
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_match(ix_pos, q, "lev", 1)
    assert e.value.status == fpm.FPM_EUNSUPPORTED
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_match(ix, q, "lev", 4)
    assert e.value.status == fpm.FPM_EUNSUPPORTED
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_build_fingerprints(d, "occ", 8, "common")
    assert e.value.status == fpm.FPM_EINVAL
    bad = np.full(256, 255, dtype=np.uint8)
    bad[97] = 8
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_build_fingerprints(d, "count", 16, custom_map=bad)
    assert e.value.status == fpm.FPM_EINVAL
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_match(ix, datagen.to_csr([b"a" * 256]), "lev", 1)
    assert e.value.status == fpm.FPM_EINVAL
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_match(ix, q, "lev", 1, fpm.options(queries_per_item=24))
    assert e.value.status == fpm.FPM_EINVAL
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_match(ix, q, "lev", 1, fpm.options(schedule=1, tail_split=101))
    assert e.value.status == fpm.FPM_EINVAL


def expected_items(d, q, metric, k, qt, slab, tail):
    """Work items of the batched schedule's list: per compatible bucket pair,
    whole slabs covering about (100 - tail)% of the words in full tiles and
    the rest in (qt / 2) x (slab / 4) tiles (tail = 100: full tiles only)."""
    cd = np.bincount(datagen.csr_lengths(d), minlength=260)
    cq = np.bincount(datagen.csr_lengths(q), minlength=260)
    r = 0 if metric == "ham" else k
    qt2, sl2 = max(16, (qt // 2) & ~15), max(64, (slab // 4) & ~63)
    ceil = lambda a, b: -(-a // b)
    items = 0
    for m in range(256):
        for L in range(max(m - r, 0), min(m + r, 255) + 1):
            nq, nd = int(cq[m]), int(cd[L])
            if not nq or not nd:
                continue
            full = nd if tail == 100 else (nd - nd * tail // 100) // slab * slab
            items += (ceil(nq, qt) * ceil(full, slab) if full else 0)
            items += (ceil(nq, qt2) * ceil(nd - full, sl2) if nd - full else 0)
    return items


@pytest.mark.parametrize("tail", [1, 10, 25, 40, 99, 100])
def test_tail_split(fpm, small, tail):
    """The split of each bucket pair into full-size and tail items covers
    every pair once: the match list equals the oracle's whatever the split,
    and the item count is the documented one."""
    d, q = small
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    for metric, k, qt, slab in [("lev", 1, 32, 256), ("lev", 2, 64, 1024), ("ham", 1, 16, 64)]:
        say("tail split", tail, metric, k, qt, slab)
        got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=fpm.FPM_SCHED_BATCHED, queries_per_item=qt,
                                                              slab=slab, tail_split=tail), with_stats=True)
        ref = oracle_match("small", d, q, oracle.LEV if metric == "lev" else oracle.HAM, k)
        assert np.array_equal(got, ref)
        assert st["work_items"] == expected_items(d, q, metric, k, qt, slab, tail)


@pytest.mark.parametrize("nq", [1, 2, 3, 5, 9, 17, 33, 65, 129, 257, 513])
def test_match_order_across_key_widths(fpm, small, nq):
    """The match list is sorted on (query, word) bits whose width depends on
    the batch size (a different number of radix passes, odd or even); every
    width must give the oracle's order."""
    d, q = small
    qs = datagen.take_csr(q, np.arange(nq))
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    say("key widths", nq)
    for sched in (0, 1):
        got = fpm.fpm_match(ix, qs, "lev", 2, fpm.options(schedule=sched))
        assert np.array_equal(got, oracle.match(d, qs, oracle.LEV, 2))


@pytest.mark.parametrize("sched,unit", [(0, "valu"), (1, "valu"), (1, "matrix")])
def test_deterministic_repeats(fpm, small, sched, unit):
    """Ten reruns of one configuration return the same sorted list, equal to
    the oracle's (the queue, staging and match counter take their entries in
    whatever order the waves reach their atomics; the sort makes the result
    unique)."""
    d, q = small
    ix = fpm.fpm_build_fingerprints(d, "occ", 16, "common")
    say("repeats", sched, unit)
    opts = fpm.options(schedule=sched, filter_unit=unit)
    first = fpm.fpm_match(ix, q, "lev", 1, opts)
    assert np.array_equal(first, oracle.match(d, q, oracle.LEV, 1))
    for _ in range(9):
        assert np.array_equal(fpm.fpm_match(ix, q, "lev", 1, opts), first)


# ------------------------------------------------------- URL-like and mixed

@pytest.fixture(scope="module")
def url_small():
    """4,000 URL-like strings x 300 queries, 30% near-matches with 1 or 2 edits."""
    return datagen.url_workload(4000, 300, 5, 0.3, (1, 2))


@pytest.fixture(scope="module")
def mixed_small():
    """2,000 English-like + 2,000 URL-like strings x 300 mixed queries."""
    return datagen.mixed_workload(2000, 2000, 300, 9)


URL_CASES = [
    (oracle.OCC, 32, oracle.LEV, 3), (oracle.COUNT, 32, oracle.HAM, 3),
    (oracle.OCC, 32, oracle.LEV, 1), (oracle.OCC, 32, oracle.LEV, 2), (oracle.COUNT, 32, oracle.LEV, 1),
    (oracle.COUNT, 32, oracle.LEV, 2), (oracle.OCC, 16, oracle.LEV, 2), (oracle.POS, 32, oracle.HAM, 2),
    (oracle.COUNT, 32, oracle.HAM, 1), (oracle.OCCH, 32, oracle.HAM, 1),
]


@pytest.mark.parametrize("variant,bits,metric,k", URL_CASES)
@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("which", ["url", "mixed"])
def test_long_strings_match_equals_oracle(fpm, url_small, mixed_small, variant, bits, metric, k, schedule, which):
    d, q = url_small if which == "url" else mixed_small
    say(which, VARIANT_NAMES[variant], bits, metric, k, schedule)
    ix = fpm.fpm_build_fingerprints(d, variant, bits, "mixed" if which == "url" else "common")
    got, st = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=schedule), with_stats=True)
    ref = oracle_match(which, d, q, metric, k)
    assert np.array_equal(got, ref)
    ex, surv, _ = oracle.filter_stats(d, q, variant, bits, fpm.fpm_get_map(ix), metric, k)
    assert (st["pairs_examined"], st["survivors"]) == (ex, surv)


_workloads = {}


def full_workload(name):
    if name not in _workloads:
        _workloads.clear()  # one full-size workload in memory at a time
        _workloads[name] = datagen.workload(name)
    return _workloads[name]


FULL_CASES = [
    # the 1M English-like x 10K configuration: occurrence, count, position at 16 and 32 bits
    ("english_1m_q10k", oracle.OCC, 16, oracle.LEV, 1), ("english_1m_q10k", oracle.OCC, 16, oracle.HAM, 1),
    ("english_1m_q10k", oracle.OCC, 32, oracle.LEV, 1), ("english_1m_q10k", oracle.OCC, 32, oracle.HAM, 1),
    ("english_1m_q10k", oracle.COUNT, 16, oracle.LEV, 1), ("english_1m_q10k", oracle.COUNT, 16, oracle.HAM, 1),
    ("english_1m_q10k", oracle.COUNT, 32, oracle.LEV, 1), ("english_1m_q10k", oracle.COUNT, 32, oracle.HAM, 1),
    ("english_1m_q10k", oracle.POS, 16, oracle.HAM, 1), ("english_1m_q10k", oracle.POS, 32, oracle.HAM, 1),
    # the 1M URL-like x 10K configuration: occurrence and count at 32 bits, Lev k = 1, 2
    ("url_1m_q10k", oracle.OCC, 32, oracle.LEV, 1), ("url_1m_q10k", oracle.OCC, 32, oracle.LEV, 2),
    ("url_1m_q10k", oracle.COUNT, 32, oracle.LEV, 1), ("url_1m_q10k", oracle.COUNT, 32, oracle.LEV, 2),
    # the batched uneven workload, Lev k = 1 and k = 2
    ("mixed_2m_q64k", oracle.OCC, 32, oracle.LEV, 1), ("mixed_2m_q64k", oracle.OCC, 32, oracle.LEV, 2),
]


@pytest.mark.parametrize("name,variant,bits,metric,k", FULL_CASES)
def test_full_size_sampled_parity(fpm, name, variant, bits, metric, k):
    """Full-size workloads in the benchmark's launch configuration (batched,
    persistent, hipGraph) with the paper's common map: the rows of 48
    sampled queries equal the oracle's (length-pruned mode, exact since
    Lev >= |m - n|), the filtered result equals the GPU brute force on every
    query, and on the sampled queries the filter keeps exactly the pairs
    the oracle's F_D counts (F_D <= 2k)."""
    import torch

    d, q = full_workload(name)
    nq = q[1].size - 1
    say("full size", name, VARIANT_NAMES[variant], bits, metric, k)
    ix = fpm.fpm_build_fingerprints(d, variant, bits, "common")
    qb = torch.from_numpy(q[0].copy()).cuda()
    qo = torch.from_numpy(q[1].view(np.int64).copy()).cuda()
    torch.cuda.synchronize()  # the plans run on their own streams
    res = {}
    for sched in (fpm.FPM_SCHED_BATCHED, fpm.FPM_SCHED_BRUTE):
        plan = fpm.fpm_plan_create(ix, nq, int(q[1][-1]), metric, k, fpm.options(schedule=sched))
        fpm.fpm_plan_run(plan, qb.data_ptr(), qo.data_ptr(), nq)
        res[sched] = fpm.fpm_plan_copy_matches(plan)
        del plan
    assert np.array_equal(res[fpm.FPM_SCHED_BATCHED], res[fpm.FPM_SCHED_BRUTE])
    sample = np.random.default_rng(11).choice(nq, 48, replace=False)
    sample.sort()
    qs = datagen.take_csr(q, sample)
    ref = oracle.match(d, qs, metric, k, length_pruned=True)
    ref[:, 0] = sample[ref[:, 0]]
    got = res[fpm.FPM_SCHED_BATCHED]
    got = got[np.isin(got[:, 0], sample)]
    assert np.array_equal(got, ref)
    _, surv, _ = oracle.filter_stats(d, qs, variant, bits, fpm.fpm_get_map(ix), metric, k)
    assert fpm.fpm_filter_pairs(ix, qs, metric, k).shape[0] == surv


@pytest.mark.parametrize("k,unit", [(1, "valu"), (2, "valu"), (1, "matrix")])
def test_headline_as_benched(fpm, k, unit):
    """The benchmark's headline exactly as it is timed (k = 1; k = 2 with
    its own stored map and tuning entry; the matrix-core form with its own
    tuning entry): 2M mixed words x 65,536 queries,
    the stored learned occ32 map, the tuning table's tiles and batches in
    flight, one plan per batch, runs alternating over the plans with the
    kernel-timed (split graph) and whole-graph forms: every run returns the
    GPU brute force's list, and 48 sampled query rows equal the oracle's."""
    import json
    import os

    import torch

    from paper_1711_08475_amd import learn

    name = "mixed_2m_q64k"
    table = json.load(open(os.path.join(os.path.dirname(learn.__file__), "tuned.json")))
    entry = dict(table[f"{name}|occ32|lev{k}|learned" + ("|matrix" if unit == "matrix" else "")])
    entry["filter_unit"] = fpm.FPM_UNIT_MATRIX if unit == "matrix" else fpm.FPM_UNIT_VALU
    inflight = entry.pop("inflight", 2)
    mp, _ = learn.load_map(f"{name}_occ32_k{k}")
    d, q = full_workload(name)
    nq = q[1].size - 1
    say("headline as benched", k, unit, entry, inflight)
    ix = fpm.fpm_build_fingerprints(d, "occ", 32, custom_map=mp)
    qb = torch.from_numpy(q[0].copy()).cuda()
    qo = torch.from_numpy(q[1].view(np.int64).copy()).cuda()
    torch.cuda.synchronize()
    plan = fpm.fpm_plan_create(ix, nq, int(q[1][-1]), "lev", k, fpm.options(schedule=fpm.FPM_SCHED_BRUTE))
    fpm.fpm_plan_run(plan, qb.data_ptr(), qo.data_ptr(), nq)
    brute = fpm.fpm_plan_copy_matches(plan)
    del plan
    for timed in (1, 0):
        plans = [fpm.fpm_plan_create(ix, nq, int(q[1][-1]), "lev", k, fpm.options(**entry, time_kernel=timed))
                 for _ in range(inflight)]
        for step in range(2 * inflight):
            fpm.fpm_plan_run(plans[step % inflight], qb.data_ptr(), qo.data_ptr(), nq)
        for p in plans:
            assert np.array_equal(fpm.fpm_plan_copy_matches(p), brute)
        if timed:
            assert all(fpm.fpm_plan_kernel_ms(p).size >= 2 for p in plans)  # a run that grew the match buffer repeats
        del plans
    sample = np.random.default_rng(12).choice(nq, 48, replace=False)
    sample.sort()
    ref = oracle.match(d, datagen.take_csr(q, sample), oracle.LEV, k, length_pruned=True)
    ref[:, 0] = sample[ref[:, 0]]
    assert np.array_equal(brute[np.isin(brute[:, 0], sample)], ref)


@pytest.mark.parametrize("length", [1, 5, 17, 33, 49, 241])
def test_single_length_layout_capacity(fpm, length):
    """Every word and query of one length L with L = 1 (mod 16) or 1 (mod 4):
    the padded slots are then widest relative to the bytes (L = 17: 8 dwords
    for 17 bytes), which the string buffers must hold for every word."""
    d, q = datagen.fixed_length_workload(3000, 120, length, 77 + length)
    say("single length", length)
    ix = fpm.fpm_build_fingerprints(d, "occ", 32, "common")
    m = fpm.fpm_get_map(ix)
    assert np.array_equal(fpm.fpm_get_fingerprints(ix), oracle.fingerprints(d, oracle.OCC, 32, m))
    assert np.array_equal(fpm.fpm_fingerprints(ix, q), oracle.fingerprints(q, oracle.OCC, 32, m))
    for metric, k in [(oracle.HAM, 1), (oracle.LEV, 2)] if length < 64 else [(oracle.HAM, 1)]:
        ref = oracle.match(d, q, metric, k)
        for sched in (0, 1, 2):
            got = fpm.fpm_match(ix, q, metric, k, fpm.options(schedule=sched))
            assert np.array_equal(got, ref)
    # exact distances of every (query, last words) pair through the verifier
    pairs = np.array([[i, j] for i in range(0, 120, 7) for j in range(2990, 3000)], dtype=np.uint32)
    dist = fpm.fpm_verify_pairs(ix, q, pairs, "ham", 1)
    ref = oracle.pair_dist(d, q, pairs, oracle.HAM)
    assert np.array_equal(dist, np.minimum(ref, 2))
