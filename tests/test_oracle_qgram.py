"""Pins for the oracle's bigram (q = 2) fingerprints, the q-gram direction of
the paper's future work (Section 5).  A bigram fingerprint sets one hashed
field per distinct bigram of the raw bytes.  One edit removes at most two
bigram occurrences and adds at most two, so F_D moves by at most 4 per edit
and a pair within distance k has F_D <= 4k; the pins check the set
semantics, the per-edit bound, exhaustive soundness on tiny alphabets, that
the 2k threshold of Eq. 1 would be unsound here, and the filter counts."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1711_08475_amd import datagen

NOMAP = np.full(256, oracle.NONE, dtype=np.uint8)  # bigram fingerprints ignore the symbol map


def fp(s, bits=16):
    return oracle.fingerprint(s, oracle.QGRAM, bits, NOMAP)


@pytest.mark.parametrize("bits", [16, 32])
def test_bigram_set_semantics(bits):
    # no bigram below length 2
    assert fp("", bits) == 0 and fp("a", bits) == 0
    # one bigram sets exactly one field
    for s in ("ab", "zz", "q7", "//"):
        assert bin(fp(s, bits)).count("1") == 1
    # a fingerprint is the union of its bigrams' fields: only the set matters
    assert fp("aba", bits) == fp("abab", bits) == fp("ababab", bits) == fp("ab", bits) | fp("ba", bits)
    assert fp("abc", bits) == fp("ab", bits) | fp("bc", bits)
    assert fp("aab", bits) == fp("aa", bits) | fp("ab", bits)
    # order matters (unlike symbol occurrence): most reversed bigrams differ
    letters = "abcdefghijklmnopqrstuvwxyz"
    differ = sum(fp(x + y, bits) != fp(y + x, bits) for x in letters for y in letters if x < y)
    assert differ > 0.8 * 325


# Field indices of the documented hash, worked by hand: v = 256 * first
# byte + second byte; h = v * 2654435761 mod 2^32; field = top log2(bits)
# bits of h.  "ab": v = 97 * 256 + 98 = 24930; 24930 * 2654435761 =
# 66,175,083,521,730 = 15407 * 2^32 + 2,522,392,258 (0x9658A6C2), so field
# 9 of 16 (0x9) and 18 of 32 (0x9658A6C2 >> 27).  "ba": v = 25185, h =
# 0x2F9ADE11: fields 2 and 5 -- swapping the two bytes of v would swap the
# fields of "ab" and "ba".  "zz": v = 31354, h = 0xD66E585A: 13 and 26.
# "//": v = 12079, h = 0x3B86D67F: 3 and 7.  "q7": v = 28983,
# h = 0x7AA24607: 7 and 15.
HAND_FIELDS = {"ab": (9, 18), "ba": (2, 5), "zz": (13, 26), "//": (3, 7), "q7": (7, 15)}


@pytest.mark.parametrize("bigram", sorted(HAND_FIELDS))
def test_bigram_field_index_worked_by_hand(bigram):
    f16, f32 = HAND_FIELDS[bigram]
    assert fp(bigram, 16) == 1 << f16
    assert fp(bigram, 32) == 1 << f32
    # a longer string is the union of its bigrams' fields
    assert fp("abzz", 16) == (1 << 9) | (1 << 13) | fp("bz", 16)  # bigrams ab, bz, zz


@pytest.mark.parametrize("bits", [16, 32])
def test_hash_reaches_every_field(bits):
    letters = "abcdefghijklmnopqrstuvwxyz"
    seen = 0
    for x in letters:
        for y in letters:
            seen |= fp(x + y, bits)
    assert seen == (1 << bits) - 1
    assert oracle.num_fields(oracle.QGRAM, bits) == bits


def _random_edit(s: bytes, rng, alphabet: bytes, op: str) -> bytes:
    s = bytearray(s)
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


@pytest.mark.parametrize("bits", [16, 32])
@pytest.mark.parametrize("op,bound", [("sub", 4), ("ins", 3), ("del", 3)])
def test_single_edit_moves_fd_by_at_most_four(bits, op, bound):
    """A substitution replaces at most two bigrams (F_D moves by <= 4); an
    insertion or a deletion replaces one bigram by two or two by one (<= 3).
    The bounds are attained."""
    rng = np.random.default_rng(50 + bits + len(op))
    alpha = b"etaoinshrdlcumwfgypbvkjxqz"
    S2 = [bytes(rng.choice(np.frombuffer(alpha, np.uint8), size=int(rng.integers(0, 14)))) for _ in range(3000)]
    S3 = [_random_edit(s, rng, alpha, op) for s in S2]
    f2 = oracle.fingerprints(S2, oracle.QGRAM, bits, NOMAP)
    f3 = oracle.fingerprints(S3, oracle.QGRAM, bits, NOMAP)
    d = oracle.fd(f2, f3, oracle.QGRAM, bits).astype(np.int64)
    assert np.all(d <= bound)
    assert np.any(d == bound)


def _tiny_universe(alphabet: str, max_len: int):
    out = [""]
    for n in range(1, max_len + 1):
        out += ["".join(t) for t in itertools.product(alphabet, repeat=n)]
    return out


@pytest.mark.parametrize("metric", [oracle.HAM, oracle.LEV])
def test_bigram_filter_never_rejects_a_true_match_exhaustive(metric):
    """Over all strings on {e,t,a,z} up to length 5, every pair within distance
    d <= 3 has F_D <= 4d, at both widths."""
    U = _tiny_universe("etaz", 5)
    res = oracle.match(U, U, metric, 3)
    d = res[:, 2].astype(np.int64)
    for bits in (16, 32):
        f = oracle.fingerprints(U, oracle.QGRAM, bits, NOMAP)
        fd = oracle.fd(f[res[:, 0]], f[res[:, 1]], oracle.QGRAM, bits).astype(np.int64)
        assert np.all(fd <= 4 * d)
        assert oracle.threshold(oracle.QGRAM, 3) == 12 and oracle.threshold(oracle.OCC, 3) == 6


def test_eq1_threshold_would_reject_true_matches():
    """With the 2k threshold of the symbol fingerprints, bigram fingerprints
    reject true matches: the 4k threshold is needed."""
    U = _tiny_universe("etaz", 4)
    res = oracle.match(U, U, oracle.LEV, 1)
    f = oracle.fingerprints(U, oracle.QGRAM, 32, NOMAP)
    fd = oracle.fd(f[res[:, 0]], f[res[:, 1]], oracle.QGRAM, 32).astype(np.int64)
    assert np.any(fd > 2 * res[:, 2].astype(np.int64))


def test_filter_stats_bigram_closed_form_and_soundness():
    d, q = datagen.english_workload(3000, 200, 21, "3-15", 0.5)
    ld, lq = datagen.csr_lengths(d), datagen.csr_lengths(q)
    hd, hq = np.bincount(ld, minlength=256), np.bincount(lq, minlength=256)
    for bits in (16, 32):
        for metric, k in ((oracle.HAM, 1), (oracle.LEV, 1), (oracle.LEV, 2)):
            ex, surv, _ = oracle.filter_stats(d, q, oracle.QGRAM, bits, NOMAP, metric, k)
            if metric == oracle.HAM:
                closed = int((hd * hq).sum())
            else:
                closed = sum(int(hq[a]) * int(hd[b]) for a in range(256) for b in range(256) if abs(a - b) <= k)
            assert ex == closed
            matches = oracle.match(d, q, metric, k)
            assert matches.shape[0] <= surv <= ex
            fq = oracle.fingerprints(q, oracle.QGRAM, bits, NOMAP)
            fw = oracle.fingerprints(d, oracle.QGRAM, bits, NOMAP)
            assert np.all(oracle.fd(fq[matches[:, 0]], fw[matches[:, 1]], oracle.QGRAM, bits) <= 4 * k)
