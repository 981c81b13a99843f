"""Pins for the oracle's distances and brute-force matcher (CPU only).

The oracle is pinned against things other than itself: textbook values,
closed forms, an independent breadth-first enumeration of edit
neighbourhoods over tiny alphabets, and metric invariants."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1711_08475_amd import datagen


def universe(alphabet: str, max_len: int):
    out = [""]
    for n in range(1, max_len + 1):
        out += ["".join(t) for t in itertools.product(alphabet, repeat=n)]
    return out


def edit_neighbours(s: str, alphabet: str, subs_only: bool = False):
    """Strings one insertion, deletion or substitution away from s."""
    out = set()
    for i in range(len(s)):
        for c in alphabet:
            if c != s[i]:
                out.add(s[:i] + c + s[i + 1:])
    if not subs_only:
        for i in range(len(s) + 1):
            for c in alphabet:
                out.add(s[:i] + c + s[i:])
        for i in range(len(s)):
            out.add(s[:i] + s[i + 1:])
    return out


def bfs_levels(s: str, alphabet: str, radius: int, subs_only: bool = False):
    """dict string -> edit distance, for every string within `radius` edits."""
    level = {s: 0}
    frontier = {s}
    for r in range(1, radius + 1):
        nxt = set()
        for t in frontier:
            for u in edit_neighbours(t, alphabet, subs_only):
                if u not in level:
                    level[u] = r
                    nxt.add(u)
        frontier = nxt
    return level


# -------------------------------------------------------------- closed forms

@pytest.mark.parametrize("a,b,d", [
    ("kitten", "sitting", 3),
    ("flaw", "lawn", 2),
    ("intention", "execution", 5),
    ("abc", "acb", 2),          # no transposition operation
    ("", "", 0),
    ("abc", "", 3),
    ("", "abcd", 4),
    ("abc", "abc", 0),
    ("abc", "abd", 1),          # substitution
    ("abc", "abxc", 1),         # insertion
    ("abc", "ac", 1),           # deletion
    ("run", "ran", 1),          # Section 3.3 example
])
def test_lev_textbook(a, b, d):
    assert oracle.lev(a, b) == d
    assert oracle.lev(b, a) == d


@pytest.mark.parametrize("a,b,d", [
    ("karolin", "kathrin", 3),
    ("1011101", "1001001", 2),
    ("2173896", "2233796", 3),
    ("", "", 0),
    ("abc", "abc", 0),
    ("run", "ran", 1),
])
def test_ham_textbook(a, b, d):
    assert oracle.ham(a, b) == d


def test_ham_infinite_for_unequal_lengths():
    assert oracle.ham("abc", "ab") is None
    assert oracle.ham("", "a") is None


def test_lev_of_empty_is_length():
    rng = np.random.default_rng(5)
    for _ in range(50):
        s = bytes(rng.integers(97, 123, size=int(rng.integers(0, 60))))
        assert oracle.lev(s, b"") == len(s)
        assert oracle.lev(b"", s) == len(s)
        assert oracle.lev(s, s) == 0


def test_lev_against_bfs_exhaustive():
    """Every pair of strings over {a,b,c} up to length 5: the oracle's
    distance (k = 2) equals the level in a breadth-first search of single
    edits, and pairs beyond two edits are absent."""
    alph = "abc"
    U = universe(alph, 5)
    res = oracle.match(U, U, oracle.LEV, 2)
    got = {(int(q), int(w)): int(d) for q, w, d in res}
    index = {s: i for i, s in enumerate(U)}
    expect = {}
    for i, s in enumerate(U):
        for t, lvl in bfs_levels(s, alph, 2).items():
            j = index.get(t)
            if j is not None:
                expect[(i, j)] = lvl
    assert got == expect


def test_ham_against_bfs_exhaustive():
    alph = "abcd"
    U = universe(alph, 4)
    res = oracle.match(U, U, oracle.HAM, 2)
    got = {(int(q), int(w)): int(d) for q, w, d in res}
    index = {s: i for i, s in enumerate(U)}
    expect = {}
    for i, s in enumerate(U):
        for t, lvl in bfs_levels(s, alph, 2, subs_only=True).items():
            expect[(i, index[t])] = lvl
    assert got == expect


def test_lev_k1_characterisation_exhaustive():
    """Lev <= 1 for |m-n| = 1 iff the longest common prefix plus the longest
    common suffix covers the shorter string; for m = n iff Ham <= 1."""
    U = universe("abc", 5)
    res = oracle.match(U, U, oracle.LEV, 1)
    got = {(int(q), int(w)) for q, w, _ in res}

    def lcp(a, b):
        i = 0
        while i < min(len(a), len(b)) and a[i] == b[i]:
            i += 1
        return i

    def lcs(a, b):
        return lcp(a[::-1], b[::-1])

    expect = set()
    for i, a in enumerate(U):
        for j, b in enumerate(U):
            if len(a) == len(b):
                if sum(x != y for x, y in zip(a, b)) <= 1:
                    expect.add((i, j))
            elif abs(len(a) - len(b)) == 1:
                if lcp(a, b) + lcs(a, b) >= min(len(a), len(b)):
                    expect.add((i, j))
    assert got == expect


# ---------------------------------------------------------------- invariants

def _random_strings(n, seed, lo=0, hi=12, alphabet=b"abcde"):
    rng = np.random.default_rng(seed)
    a = np.frombuffer(alphabet, dtype=np.uint8)
    return [bytes(a[rng.integers(0, a.size, size=int(rng.integers(lo, hi + 1)))]) for _ in range(n)]


def test_metric_invariants():
    S = _random_strings(120, 7)
    for a, b, c in zip(S[0::3], S[1::3], S[2::3]):
        dab, dba = oracle.lev(a, b), oracle.lev(b, a)
        assert dab == dba
        assert dab >= abs(len(a) - len(b))
        assert dab <= max(len(a), len(b))
        assert oracle.lev(a, c) <= dab + oracle.lev(b, c)
        if len(a) == len(b):
            assert dab <= oracle.ham(a, b)
            assert oracle.ham(a, b) == oracle.ham(b, a)


def test_match_sorted_threads_and_pruned_mode_agree():
    d, q = datagen.english_workload(2000, 150, 9, "3-15", 0.5)
    full = oracle.match(d, q, oracle.LEV, 2)
    one = oracle.match(d, q, oracle.LEV, 2, threads=1)
    pruned = oracle.match(d, q, oracle.LEV, 2, length_pruned=True)
    assert np.array_equal(full, one)
    assert np.array_equal(full, pruned)
    keys = full[:, 0].astype(np.uint64) << np.uint64(32) | full[:, 1].astype(np.uint64)
    assert np.all(np.diff(keys.astype(np.int64)) > 0)
    # every near-match query (one edit of a dictionary word) has a match
    assert len(set(full[:, 0].tolist())) >= 60
    dist = oracle.pair_dist(d, q, full[:, :2], oracle.LEV)
    assert np.array_equal(dist, full[:, 2])


def test_match_k_monotone_and_ham_subset():
    d, q = datagen.english_workload(1500, 100, 10, "3-15", 0.5)
    m1 = {tuple(r[:2]) for r in oracle.match(d, q, oracle.LEV, 1)}
    m2 = {tuple(r[:2]) for r in oracle.match(d, q, oracle.LEV, 2)}
    h1 = {tuple(r[:2]) for r in oracle.match(d, q, oracle.HAM, 1)}
    assert m1 <= m2
    assert h1 <= m1


def test_rejects_overlong_strings():
    with pytest.raises(ValueError):
        oracle.match([b"a" * 256], [b"a"], oracle.LEV, 1)


def test_fixed_length_workload_shape():
    """Single-length words and queries; about half of the queries are one
    substitution away from a dictionary word, so Ham k = 1 finds them."""
    from paper_1711_08475_amd import datagen

    d, q = datagen.fixed_length_workload(3000, 200, 9, 5)
    assert set(datagen.csr_lengths(d)) == {9} and set(datagen.csr_lengths(q)) == {9}
    hits = oracle.match(d, q, oracle.HAM, 1)
    near = np.unique(hits[hits[:, 2] == 1, 0]).size
    assert 70 <= near <= 130
