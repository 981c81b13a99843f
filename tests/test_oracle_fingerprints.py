"""Pins for the oracle's fingerprints, fingerprint distance and symbol
selection (CPU only): the paper's worked example, its prose examples, the
per-edit bounds of Theorems 1 and 2, exhaustive soundness of Eq. 1 on tiny
alphabets and hand-computed symbol selections."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from paper_1711_08475_amd import datagen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def letters_map(letters: str) -> np.ndarray:
    m = np.full(256, oracle.NONE, dtype=np.uint8)
    for i, c in enumerate(letters):
        m[ord(c)] = i
    return m


def decode_printed(variant: str, printed: str) -> int:
    """Integer of a printed fingerprint under the layout used throughout:
    field j (printed j-th from the left) sits at the j-th lowest bits."""
    groups = printed.split() if " " in printed else list(printed)
    v = 0
    if variant == "occ":
        for j, g in enumerate(groups):
            v |= int(g) << j
    elif variant == "count":
        for j, g in enumerate(groups):
            v |= int(g, 2) << (2 * j)
    elif variant == "occh":
        for j, g in enumerate(groups):
            v |= int(g[0]) << (2 * j)
            v |= int(g[1]) << (2 * j + 1)
    elif variant == "pos":
        *pos, occ = groups
        for j, g in enumerate(pos):
            v |= int(g, 2) << (3 * j)
        for t, bit in enumerate(occ):
            v |= int(bit) << (3 * len(pos) + t)
    return v


def test_instance_example_all_variants():
    ex = json.load(open(os.path.join(GOLDEN, "instance_example.json")))
    w, L = ex["word"], ex["letters"]
    cases = {"occ": (oracle.OCC, L), "occh": (oracle.OCCH, L[:8]),
             "count": (oracle.COUNT, L[:8]), "pos": (oracle.POS, L[:6])}
    got = {}
    for name, (variant, letters) in cases.items():
        got[name] = oracle.fingerprint(w, variant, 16, letters_map(letters))
        assert got[name] == decode_printed(name, ex["printed"][name]), name
    # the integer values under this layout
    assert got == {"occ": 0x0877, "occh": 0x1D26, "count": 0x1915, "pos": 0x8F1F}


def test_run_ran_example():
    """Section 3.3: run / ran differ in the occurrence of 'a' and 'u' (F_D = 2)
    yet only one substitution apart, so Eq. 1 keeps the pair at k = 1."""
    m = letters_map("etaoinshrdlcumwf")
    a = oracle.fingerprint("run", oracle.OCC, 16, m)
    b = oracle.fingerprint("ran", oracle.OCC, 16, m)
    assert oracle.fd(a, b, oracle.OCC, 16) == 2
    assert oracle.ham("run", "ran") == 1
    assert -(-2 // 2) <= 1  # ceil(F_D / 2) <= k: not rejected


def test_repeated_symbol_example():
    """Section 3.3: two strings of one repeated, different symbol each are n
    mismatches apart, but F_D is 1 (one symbol outside the set) or 0."""
    m = letters_map("etaoinshrdlcumwf")
    e, z, q = (oracle.fingerprint(s, oracle.OCC, 16, m) for s in ("eeeeee", "zzzzzz", "qqqqqq"))
    assert oracle.fd(e, z, oracle.OCC, 16) == 1
    assert oracle.fd(z, q, oracle.OCC, 16) == 0
    assert oracle.ham("eeeeee", "zzzzzz") == 6


def test_count_saturates_at_three():
    m = letters_map("etaoinsh")
    for n, expect in [(0, 0), (1, 1), (2, 2), (3, 3), (4, 3), (9, 3)]:
        assert oracle.fingerprint("e" * n + "xy", oracle.COUNT, 16, m) & 3 == expect


def test_count_literal_underestimates_three_vs_one():
    """Section 3.3: counters 3 (11) and 1 (01) differ in one bit although the
    counts differ by 2; the sound distance is the count difference."""
    m = letters_map("etaoinsh")
    a = oracle.fingerprint("eee", oracle.COUNT, 16, m)
    b = oracle.fingerprint("e", oracle.COUNT, 16, m)
    assert oracle.fd(a, b, oracle.COUNT, 16, literal=True) == 1
    assert oracle.fd(a, b, oracle.COUNT, 16) == 2


def test_count_literal_is_unsound_eet_ett():
    """One substitution turns eet into ett; the binary counters 2,1 vs 1,2
    differ in 4 bits, so the literal XOR weight would reject a true match at
    k = 1.  The count-difference distance gives 2 (kept)."""
    m = letters_map("etaoinsh")
    a = oracle.fingerprint("eet", oracle.COUNT, 16, m)
    b = oracle.fingerprint("ett", oracle.COUNT, 16, m)
    assert oracle.ham("eet", "ett") == 1 and oracle.lev("eet", "ett") == 1
    assert oracle.fd(a, b, oracle.COUNT, 16, literal=True) == 4
    assert oracle.fd(a, b, oracle.COUNT, 16) == 2


def test_pos_sentinel_and_positions():
    m = letters_map("etaoin")  # 5 position letters + 'n' as the occurrence bit
    f = lambda s: oracle.fingerprint(s, oracle.POS, 16, m)
    assert f("xxxxxxe") & 7 == 6          # 0-indexed position 6 is stored
    assert f("xxxxxxxe") & 7 == 7         # position 7 = 2^p - 1 -> all ones
    assert f("xxxxxxxxxe") & 7 == 7       # beyond -> all ones
    assert f("xyz") & 7 == 7              # absent -> all ones
    assert f("exe") & 7 == 0              # first occurrence counts
    assert (f("n") >> 15) & 1 == 1 and (f("x") >> 15) & 1 == 0
    # every absent position field is all ones
    assert f("") == 0x7FFF


def test_pos_distance_counts_fields():
    m = letters_map("etaoin")
    a, b = oracle.fingerprint("eta", oracle.POS, 16, m), oracle.fingerprint("tea", oracle.POS, 16, m)
    # e: 0 vs 1, t: 1 vs 0, a: 2 vs 2 -> two mismatching 3-bit fields
    assert oracle.fd(a, b, oracle.POS, 16) == 2
    assert oracle.fd(a, a, oracle.POS, 16) == 0
    c = oracle.fingerprint("etan", oracle.POS, 16, m)
    # n adds the occurrence bit; 'n' also has no position field
    assert oracle.fd(a, c, oracle.POS, 16) == 1


def test_num_fields():
    assert [oracle.num_fields(v, 16) for v in (oracle.OCC, oracle.COUNT, oracle.POS, oracle.OCCH)] == [16, 8, 6, 8]
    assert [oracle.num_fields(v, 32) for v in (oracle.OCC, oracle.COUNT, oracle.POS, oracle.OCCH)] == [32, 16, 12, 16]


# ------------------------------------------------------------ symbol sets

def test_select_symbols_hand_cases():
    h = np.zeros(256, dtype=np.uint64)
    for c, n in {"a": 5, "b": 3, "c": 3, "d": 1, "e": 9}.items():
        h[ord(c)] = n
    # order by frequency, ties by byte: e(9) a(5) b(3) c(3) d(1)
    common = oracle.select_symbols(h, oracle.OCC, 16, oracle.COMMON)
    assert {chr(c): int(common[c]) for c in range(256) if common[c] != oracle.NONE} == \
        {"e": 0, "a": 1, "b": 2, "c": 3, "d": 4}
    rare = oracle.select_symbols(h, oracle.OCC, 16, oracle.RARE)
    assert {chr(c): int(rare[c]) for c in range(256) if rare[c] != oracle.NONE} == \
        {"d": 0, "b": 1, "c": 2, "a": 3, "e": 4}
    # pos at 16 bits has 6 fields; fewer symbols than fields -> all present
    mixed = oracle.select_symbols(h, oracle.POS, 16, oracle.MIXED)
    assert {chr(c): int(mixed[c]) for c in range(256) if mixed[c] != oracle.NONE} == \
        {"e": 0, "a": 1, "b": 2, "d": 3, "c": 4}


def test_select_symbols_truncates_to_field_count():
    h = np.zeros(256, dtype=np.uint64)
    for i, c in enumerate("abcdefghijklmnopqrstuvwxyz"):
        h[ord(c)] = 1000 - 10 * i  # a most frequent ... z least
    common = oracle.select_symbols(h, oracle.COUNT, 16, oracle.COMMON)
    assert [chr(c) for c in np.argsort(np.where(common == 255, 999, common))[:8]] == list("abcdefgh")
    assert int((common != 255).sum()) == 8
    rare = oracle.select_symbols(h, oracle.COUNT, 16, oracle.RARE)
    assert [chr(c) for c in np.argsort(np.where(rare == 255, 999, rare))[:8]] == list("zyxwvuts")
    mixed = oracle.select_symbols(h, oracle.COUNT, 16, oracle.MIXED)
    assert [chr(c) for c in np.argsort(np.where(mixed == 255, 999, mixed))[:8]] == list("abcdzyxw")
    pos = oracle.select_symbols(h, oracle.POS, 32, oracle.COMMON)
    assert int((pos != 255).sum()) == 12


# ------------------------------------------- Theorems 1 and 2, Eq. 1 soundness

def random_edit(s: bytes, rng, alphabet: bytes, ops):
    s = bytearray(s)
    op = ops[int(rng.integers(len(ops)))]
    if op == "sub" and s:
        i = int(rng.integers(len(s)))
        c = s[i]
        while c == s[i]:
            c = alphabet[int(rng.integers(len(alphabet)))]
        s[i] = c
    elif op == "ins":
        s.insert(int(rng.integers(len(s) + 1)), alphabet[int(rng.integers(len(alphabet)))])
    elif op == "del" and s:
        del s[int(rng.integers(len(s)))]
    return bytes(s)


def random_maps(rng, variant, bits, n=4):
    """Paper-style one-to-one maps plus random many-to-one groupings."""
    nf = oracle.num_fields(variant, bits)
    maps = [letters_map("etaoinshrdlcumwfgypbvkjxqz"[:nf])]
    for _ in range(n):
        m = np.full(256, oracle.NONE, dtype=np.uint8)
        for c in range(97, 123):
            if rng.random() < 0.85:
                m[c] = int(rng.integers(nf))
        maps.append(m)
    return maps


@pytest.mark.parametrize("variant,ops", [
    (oracle.OCC, ("sub", "ins", "del")),
    (oracle.COUNT, ("sub", "ins", "del")),
    (oracle.POS, ("sub",)),
    (oracle.OCCH, ("sub",)),
])
@pytest.mark.parametrize("bits", [16, 32])
def test_single_edit_raises_fd_by_at_most_two(variant, ops, bits):
    """Theorem 1 (occ, count; Ham and Lev) and Theorem 2 (pos; Ham): if S3 is
    one edit from S2 then F_D(S1, S3) <= F_D(S1, S2) + 2."""
    rng = np.random.default_rng(100 + variant + bits)
    alpha = b"etaoinshrdlcumwfgypbvkjxqz"
    for mp in random_maps(rng, variant, bits):
        S1 = [bytes(rng.choice(np.frombuffer(alpha, np.uint8), size=int(rng.integers(0, 14)))) for _ in range(300)]
        S2 = [bytes(rng.choice(np.frombuffer(alpha, np.uint8), size=len(s) if ops == ("sub",) else int(rng.integers(0, 14)))) for s in S1]
        S3 = [random_edit(s, rng, alpha, ops) for s in S2]
        f1 = oracle.fingerprints(S1, variant, bits, mp)
        f2 = oracle.fingerprints(S2, variant, bits, mp)
        f3 = oracle.fingerprints(S3, variant, bits, mp)
        d12 = oracle.fd(f1, f2, variant, bits).astype(np.int64)
        d13 = oracle.fd(f1, f3, variant, bits).astype(np.int64)
        assert np.all(d13 <= d12 + 2)
        # the bound is tight somewhere for occ and count
        d23 = oracle.fd(f2, f3, variant, bits).astype(np.int64)
        assert np.all(d23 <= 2)


def _tiny_universe(alphabet: str, max_len: int):
    out = [""]
    for n in range(1, max_len + 1):
        out += ["".join(t) for t in itertools.product(alphabet, repeat=n)]
    return out


@pytest.mark.parametrize("metric,variant", [
    (oracle.HAM, oracle.OCC), (oracle.LEV, oracle.OCC),
    (oracle.HAM, oracle.COUNT), (oracle.LEV, oracle.COUNT),
    (oracle.HAM, oracle.POS), (oracle.HAM, oracle.OCCH),
])
def test_eq1_never_rejects_a_true_match_exhaustive(metric, variant):
    """Eq. 1: D >= ceil(F_D/2).  Over all strings on {e,t,a,z} up to length 5
    and several symbol maps, every pair within k <= 3 keeps F_D <= 2k."""
    U = _tiny_universe("etaz", 5)
    res = oracle.match(U, U, metric, 3)
    rng = np.random.default_rng(3)
    for bits in (16, 32):
        for mp in random_maps(rng, variant, bits, n=3):
            fps = oracle.fingerprints(U, variant, bits, mp)
            f = oracle.fd(fps[res[:, 0]], fps[res[:, 1]], variant, bits).astype(np.int64)
            assert np.all(f <= 2 * res[:, 2].astype(np.int64))


def test_literal_count_and_lev_occh_violate_eq1():
    """The readings that are kept out of the filter: the literal count XOR
    weight and occurrence-halved under Lev both reject true matches."""
    U = _tiny_universe("etaz", 5)
    res = oracle.match(U, U, oracle.LEV, 1)
    mp = letters_map("etaz")
    fc = oracle.fingerprints(U, oracle.COUNT, 16, mp)
    lit = oracle.fd(fc[res[:, 0]], fc[res[:, 1]], oracle.COUNT, 16, literal=True)
    assert np.any(lit > 2 * res[:, 2])
    fh = oracle.fingerprints(U, oracle.OCCH, 16, mp)
    h = oracle.fd(fh[res[:, 0]], fh[res[:, 1]], oracle.OCCH, 16)
    assert np.any(h > 2 * res[:, 2])


def test_filter_stats_examined_closed_form_and_soundness():
    d, q = datagen.english_workload(3000, 200, 21, "3-15", 0.5)
    m = oracle.select_symbols(oracle.histogram(d), oracle.OCC, 16, oracle.COMMON)
    ld, lq = datagen.csr_lengths(d), datagen.csr_lengths(q)
    hd, hq = np.bincount(ld, minlength=256), np.bincount(lq, minlength=256)
    for metric, k in ((oracle.HAM, 1), (oracle.LEV, 1), (oracle.LEV, 2)):
        ex, surv, _ = oracle.filter_stats(d, q, oracle.OCC, 16, m, metric, k)
        if metric == oracle.HAM:
            closed = int((hd * hq).sum())
        else:
            closed = sum(int(hq[a]) * int(hd[b]) for a in range(256) for b in range(256) if abs(a - b) <= k)
        assert ex == closed
        matches = oracle.match(d, q, metric, k)
        assert matches.shape[0] <= surv <= ex
        fq = oracle.fingerprints(q, oracle.OCC, 16, m)
        fw = oracle.fingerprints(d, oracle.OCC, 16, m)
        assert np.all(oracle.fd(fq[matches[:, 0]], fw[matches[:, 1]], oracle.OCC, 16) <= 2 * k)


def test_check_map_rejects_out_of_range_fields():
    m = np.full(256, oracle.NONE, dtype=np.uint8)
    m[ord("a")] = 8
    assert not oracle.check_map(m, oracle.COUNT, 16)
    assert oracle.check_map(m, oracle.OCC, 16)
    with pytest.raises(ValueError):
        oracle.fingerprint("a", oracle.COUNT, 16, m)
