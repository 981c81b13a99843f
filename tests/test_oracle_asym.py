"""Pins for the oracle's asymmetric bound (CPU only).

The bound is an extension beyond the paper: F_D (Section 3.3) splits into the
fields where the query fingerprint exceeds the word's and the fields where the
word's exceeds the query's.  The per-edit argument of Theorem 1, applied to
each direction on its own, shows that one edit lowers either excess by at most
one, so the distance is at least the larger excess, which is at least
ceil(F_D / 2).  These tests fix the arithmetic by hand-worked cases, by the
identity with F_D, by exhaustive soundness on tiny alphabets against the exact
distances, and by the dominance over Eq. 1."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1711_08475_amd import datagen


def letters_map(letters: str) -> np.ndarray:
    m = np.full(256, oracle.NONE, dtype=np.uint8)
    for i, c in enumerate(letters):
        m[ord(c)] = i
    return m


def asym(fq, fw, variant, bits):
    a = oracle.excess(fq, fw, variant, bits)
    b = oracle.excess(fw, fq, variant, bits)
    return np.maximum(np.asarray(a, np.int64), np.asarray(b, np.int64))


def test_hand_worked_occurrence():
    """occ over fields a, b, c, d: "ab" vs "abcd" -- F_D = 2 passes Eq. 1 at
    k = 1, but the word holds two fields the query lacks (Lev = 2)."""
    mp = letters_map("abcd")
    q, w = oracle.fingerprint("ab", oracle.OCC, 16, mp), oracle.fingerprint("abcd", oracle.OCC, 16, mp)
    assert (q, w) == (0b0011, 0b1111)
    assert oracle.fd(q, w, oracle.OCC, 16) == 2
    assert oracle.excess(q, w, oracle.OCC, 16) == 0
    assert oracle.excess(w, q, oracle.OCC, 16) == 2
    assert oracle.lev("ab", "abcd") == 2
    # one substitution: one field on each side, both bounds accept at k = 1
    q, w = oracle.fingerprint("abc", oracle.OCC, 16, mp), oracle.fingerprint("abd", oracle.OCC, 16, mp)
    assert oracle.fd(q, w, oracle.OCC, 16) == 2
    assert oracle.excess(q, w, oracle.OCC, 16) == 1 and oracle.excess(w, q, oracle.OCC, 16) == 1


def test_hand_worked_count():
    """count (2-bit saturating): "aaab" holds a:3 b:1, "ab" holds a:1 b:1;
    the query exceeds by 2 in field a, the word by nothing."""
    mp = letters_map("ab")
    q, w = oracle.fingerprint("aaab", oracle.COUNT, 16, mp), oracle.fingerprint("ab", oracle.COUNT, 16, mp)
    assert (q, w) == (0b0111, 0b0101)
    assert oracle.fd(q, w, oracle.COUNT, 16) == 2
    assert oracle.excess(q, w, oracle.COUNT, 16) == 2
    assert oracle.excess(w, q, oracle.COUNT, 16) == 0
    assert oracle.lev("aaab", "ab") == 2
    # saturation: five a's read as three
    q5 = oracle.fingerprint("aaaaa", oracle.COUNT, 16, mp)
    assert oracle.excess(q5, w, oracle.COUNT, 16) == 2


def test_hand_worked_halved():
    """occh over fields a, b: "ab" sets a in the first half and b in the
    second; "ba" the reverse -- each side exceeds in two bits (Ham = 2)."""
    mp = letters_map("ab")
    q, w = oracle.fingerprint("ab", oracle.OCCH, 16, mp), oracle.fingerprint("ba", oracle.OCCH, 16, mp)
    assert (q, w) == (0b1001, 0b0110)
    assert oracle.excess(q, w, oracle.OCCH, 16) == 2 and oracle.excess(w, q, oracle.OCCH, 16) == 2
    assert oracle.ham("ab", "ba") == 2


def test_position_variant_has_no_excess():
    assert oracle.excess(1, 2, oracle.POS, 16) == oracle.INF


@pytest.mark.parametrize("variant", [oracle.OCC, oracle.OCCH, oracle.COUNT])
@pytest.mark.parametrize("bits", [16, 32])
def test_excess_halves_sum_to_fd(variant, bits):
    """excess(a, b) + excess(b, a) = F_D for every pair of valid fingerprints
    (count: fields 0..3 each; F_D is the L1 distance of the counts)."""
    rng = np.random.default_rng(7 + variant + bits)
    n = 20000
    if variant == oracle.COUNT:
        a = np.zeros(n, np.uint64)
        b = np.zeros(n, np.uint64)
        for j in range(bits // 2):
            a |= rng.integers(0, 4, n).astype(np.uint64) << np.uint64(2 * j)
            b |= rng.integers(0, 4, n).astype(np.uint64) << np.uint64(2 * j)
    else:
        a = rng.integers(0, 1 << bits, n, dtype=np.uint64)
        b = rng.integers(0, 1 << bits, n, dtype=np.uint64)
    a, b = a.astype(np.uint32), b.astype(np.uint32)
    ab = oracle.excess(a, b, variant, bits).astype(np.int64)
    ba = oracle.excess(b, a, variant, bits).astype(np.int64)
    fd = oracle.fd(a, b, variant, bits).astype(np.int64)
    assert np.array_equal(ab + ba, fd)
    # and each half is at least ceil(F_D / 2) for the larger one
    assert np.all(np.maximum(ab, ba) >= (fd + 1) // 2)
    # the difference of the halves is the difference of the totals
    if variant != oracle.COUNT:
        pa = np.array([bin(int(x)).count("1") for x in a])
        pb = np.array([bin(int(x)).count("1") for x in b])
        assert np.array_equal(ab - ba, pa - pb)


def _tiny_universe(alphabet: str, max_len: int):
    out = [""]
    for n in range(1, max_len + 1):
        out += ["".join(t) for t in itertools.product(alphabet, repeat=n)]
    return out


def _maps(rng, variant, bits, n=3):
    nf = oracle.num_fields(variant, bits)
    maps = [letters_map("etaz"[:nf])]
    for _ in range(n):
        m = np.full(256, oracle.NONE, dtype=np.uint8)
        for c in "etaz":
            if rng.random() < 0.85:
                m[ord(c)] = int(rng.integers(min(nf, 3)))  # many-to-one groupings
        maps.append(m)
    return maps


@pytest.mark.parametrize("metric,variant", [
    (oracle.HAM, oracle.OCC), (oracle.LEV, oracle.OCC),
    (oracle.HAM, oracle.COUNT), (oracle.LEV, oracle.COUNT),
    (oracle.HAM, oracle.OCCH),
])
def test_asym_never_rejects_a_true_match_exhaustive(metric, variant):
    """Over all strings on {e,t,a,z} up to length 5, every pair within
    distance d <= 3 has max(excess(q, w), excess(w, q)) <= d."""
    U = _tiny_universe("etaz", 5)
    res = oracle.match(U, U, metric, 3)
    rng = np.random.default_rng(11)
    for bits in (16, 32):
        for mp in _maps(rng, variant, bits):
            fps = oracle.fingerprints(U, variant, bits, mp)
            m = asym(fps[res[:, 0]], fps[res[:, 1]], variant, bits)
            assert np.all(m <= res[:, 2].astype(np.int64))


def test_asym_is_tight_somewhere():
    """The bound is attained: some pair at distance 1 and 2 has the larger
    excess equal to its distance (so no sharper constant holds)."""
    U = _tiny_universe("eta", 4)
    res = oracle.match(U, U, oracle.LEV, 2)
    mp = letters_map("eta")
    f = oracle.fingerprints(U, oracle.OCC, 16, mp)
    m = asym(f[res[:, 0]], f[res[:, 1]], oracle.OCC, 16)
    d = res[:, 2].astype(np.int64)
    for dist in (1, 2):
        assert np.any((d == dist) & (m == dist))


def test_lev_occh_halves_are_unsound():
    """occ-halved stays a Hamming-only fingerprint: under Lev an insertion
    shifts the halves, and the bound rejects true matches."""
    U = _tiny_universe("etaz", 5)
    res = oracle.match(U, U, oracle.LEV, 1)
    f = oracle.fingerprints(U, oracle.OCCH, 16, letters_map("etaz"))
    m = asym(f[res[:, 0]], f[res[:, 1]], oracle.OCCH, 16)
    assert np.any(m > res[:, 2])


@pytest.mark.parametrize("variant,bits,metric,k", [
    (oracle.OCC, 16, oracle.LEV, 1), (oracle.OCC, 32, oracle.LEV, 2),
    (oracle.COUNT, 16, oracle.LEV, 1), (oracle.COUNT, 32, oracle.HAM, 1),
    (oracle.OCCH, 16, oracle.HAM, 1),
])
def test_filter_stats_asym_dominates_eq1(variant, bits, metric, k):
    """On an English-like sample: the same examined pairs as Eq. 1, no more
    survivors than Eq. 1, at least every true match; every surviving pair of
    the loop is one that the per-pair definition keeps."""
    d, q = datagen.english_workload(2000, 150, 23, "3-15", 0.5)
    m = oracle.select_symbols(oracle.histogram(d), variant, bits, oracle.COMMON)
    ex, surv, _ = oracle.filter_stats(d, q, variant, bits, m, metric, k)
    ex_a, surv_a = oracle.filter_stats_asym(d, q, variant, bits, m, metric, k)
    matches = oracle.match(d, q, metric, k)
    assert ex_a == ex
    assert matches.shape[0] <= surv_a <= surv
    fq = oracle.fingerprints(q, variant, bits, m)
    fw = oracle.fingerprints(d, variant, bits, m)
    assert np.all(asym(fq[matches[:, 0]], fw[matches[:, 1]], variant, bits) <= k)
    # count the survivors pair by pair from the definition
    lq, lw = datagen.csr_lengths(q).astype(np.int64), datagen.csr_lengths(d).astype(np.int64)
    total = 0
    for i in range(len(lq)):
        gap = np.abs(lw - lq[i])
        ok = gap == 0 if metric == oracle.HAM else gap <= k
        mm = asym(np.full(len(fw), fq[i], np.uint32), fw, variant, bits)
        total += int(np.count_nonzero(ok & (mm <= k)))
    assert total == surv_a


def test_filter_stats_asym_rejects_position():
    d, q = datagen.english_workload(50, 5, 1, "3-15", 0.5)
    m = oracle.select_symbols(oracle.histogram(d), oracle.POS, 16, oracle.COMMON)
    with pytest.raises(ValueError):
        oracle.filter_stats_asym(d, q, oracle.POS, 16, m, oracle.HAM, 1)
