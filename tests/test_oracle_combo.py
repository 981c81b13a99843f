"""Pins for the oracle's combined fingerprint (occurrence and count in one
word, a future-work direction of Section 5): its two parts equal the pinned
occurrence and count constructions, its F_D is the larger of the parts'
F_D, one edit moves it by at most 2 (Theorem 1 holds for each part), and it
never rejects a true match on an exhaustive tiny alphabet."""
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


def restrict(mp, nf):
    m = mp.copy()
    m[(m != oracle.NONE) & (m >= nf)] = oracle.NONE
    return m


@pytest.mark.parametrize("bits", [16, 32])
def test_parts_are_the_occurrence_and_count_fingerprints(bits):
    d, _ = datagen.english_workload(3000, 10, 3, "3-15", 0.5)
    mp = oracle.select_symbols(oracle.histogram(d), oracle.COMBO, bits, oracle.COMMON)
    assert oracle.num_fields(oracle.COMBO, bits) == bits // 2
    f = oracle.fingerprints(d, oracle.COMBO, bits, mp).astype(np.uint64)
    half = bits // 2
    occ = oracle.fingerprints(d, oracle.OCC, 16 if bits == 16 else 32, mp).astype(np.uint64)
    cnt = oracle.fingerprints(d, oracle.COUNT, 16, restrict(mp, bits // 4)).astype(np.uint64)
    assert np.array_equal(f & np.uint64((1 << half) - 1), occ)
    assert np.array_equal(f >> np.uint64(half), cnt)


def test_hand_worked():
    """Fields e, t, a, z at 16 bits: occurrence bits 0..3 of 8, counters for
    e, t, a, z (the first four fields) above bit 8."""
    mp = letters_map("etaz")
    f = oracle.fingerprint("teeth", oracle.COMBO, 16, mp)
    assert f & 0xFF == 0b0011             # e and t occur (h is not in the map)
    assert f >> 8 == (2 << 0) | (2 << 2)  # e x2, t x2
    g = oracle.fingerprint("tea", oracle.COMBO, 16, mp)
    # occurrence part differs in a (1 bit); counts differ by |2-1| + |2-1| + |0-1| = 3
    assert oracle.fd(f, g, oracle.COMBO, 16) == 3
    # saturation: four e's count as three
    assert oracle.fingerprint("eeee", oracle.COMBO, 16, mp) == 0b0001 | (3 << 8)


@pytest.mark.parametrize("bits", [16, 32])
def test_fd_is_the_larger_part(bits):
    rng = np.random.default_rng(9 + bits)
    half = bits // 2
    n = 5000
    a = rng.integers(0, 1 << half, n).astype(np.uint32)
    b = rng.integers(0, 1 << half, n).astype(np.uint32)
    ca = np.zeros(n, np.uint32)
    cb = np.zeros(n, np.uint32)
    for j in range(bits // 4):
        ca |= rng.integers(0, 4, n).astype(np.uint32) << np.uint32(2 * j)
        cb |= rng.integers(0, 4, n).astype(np.uint32) << np.uint32(2 * j)
    fa = a | (ca << np.uint32(half))
    fb = b | (cb << np.uint32(half))
    got = oracle.fd(fa, fb, oracle.COMBO, bits).astype(np.int64)
    occ = oracle.fd(a, b, oracle.OCC, 32).astype(np.int64)
    cnt = oracle.fd(ca, cb, oracle.COUNT, 16).astype(np.int64)
    assert np.array_equal(got, np.maximum(occ, cnt))


def _tiny_universe(alphabet: str, max_len: int):
    out = [""]
    for n in range(1, max_len + 1):
        out += ["".join(t) for t in itertools.product(alphabet, repeat=n)]
    return out


@pytest.mark.parametrize("metric", [oracle.HAM, oracle.LEV])
def test_combined_never_rejects_a_true_match_exhaustive(metric):
    U = _tiny_universe("etaz", 5)
    res = oracle.match(U, U, metric, 3)
    d = res[:, 2].astype(np.int64)
    rng = np.random.default_rng(5)
    for bits in (16, 32):
        maps = [letters_map("etaz")]
        for _ in range(3):
            m = np.full(256, oracle.NONE, dtype=np.uint8)
            for c in "etaz":
                if rng.random() < 0.85:
                    m[ord(c)] = int(rng.integers(3))
            maps.append(m)
        for mp in maps:
            f = oracle.fingerprints(U, oracle.COMBO, bits, mp)
            fd = oracle.fd(f[res[:, 0]], f[res[:, 1]], oracle.COMBO, bits).astype(np.int64)
            assert np.all(fd <= 2 * d)


def test_single_edit_moves_fd_by_at_most_two():
    rng = np.random.default_rng(77)
    alpha = b"etaoinshrdlcumwfgypbvkjxqz"
    mp = letters_map("etaoinshrdlcumwf")
    S2 = [bytes(rng.choice(np.frombuffer(alpha, np.uint8), size=int(rng.integers(0, 14)))) for _ in range(3000)]
    S3 = []
    for s in S2:
        s = bytearray(s)
        op = int(rng.integers(3))
        if op == 0 and s:
            i = int(rng.integers(len(s)))
            c = s[i]
            while c == s[i]:
                c = alpha[int(rng.integers(len(alpha)))]
            s[i] = c
        elif op == 1:
            s.insert(int(rng.integers(len(s) + 1)), alpha[int(rng.integers(len(alpha)))])
        elif s:
            del s[int(rng.integers(len(s)))]
        S3.append(bytes(s))
    for bits in (16, 32):
        f2 = oracle.fingerprints(S2, oracle.COMBO, bits, restrict(mp, bits // 2))
        f3 = oracle.fingerprints(S3, oracle.COMBO, bits, restrict(mp, bits // 2))
        d = oracle.fd(f2, f3, oracle.COMBO, bits).astype(np.int64)
        assert np.all(d <= 2) and np.any(d == 2)
