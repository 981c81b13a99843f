"""CPU pin of the bound behind popcount pruning: for every key family it is
offered for, F_D of two fingerprints (the oracle's, Section 3.3) is at least
the difference of their weights -- the popcount for occurrence,
occurrence-halved and bigram fingerprints, the sum of the 2-bit counters for
count fingerprints (the popcount of the thermometer key the kernel tests) --
so a pair whose weights differ by more than the threshold fails Eq. 1 and
may be skipped untested.  Checked on every pair of a few hundred random and
workload strings, with the extreme cases (empty strings, all fields set)."""
import numpy as np
import pytest

import oracle
from paper_1711_08475_amd import datagen


def weight(fp, variant, bits):
    fp = int(fp)
    if variant == oracle.COUNT:
        return sum((fp >> (2 * j)) & 3 for j in range(oracle.num_fields(variant, bits)))
    return bin(fp).count("1")


def strings(seed, n=160):
    rng = np.random.default_rng(seed)
    d, q = datagen.workload("english_10k_q1k")
    words = datagen.from_csr(d)[:n // 2]
    alpha = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz0123456789/.-", np.uint8)
    words += [bytes(rng.choice(alpha, int(rng.integers(0, 40)))) for _ in range(n // 2)]
    return words + [b"", bytes(alpha[:32])], d


@pytest.mark.parametrize("variant,bits", [(oracle.OCC, 16), (oracle.OCC, 32), (oracle.OCCH, 16), (oracle.OCCH, 32),
                                          (oracle.COUNT, 16), (oracle.COUNT, 32), (oracle.QGRAM, 16),
                                          (oracle.QGRAM, 32)])
def test_fd_is_at_least_the_weight_difference(variant, bits):
    words, d = strings(bits + variant)
    mp = oracle.select_symbols(oracle.histogram(d), variant, bits, oracle.COMMON)
    fps = oracle.fingerprints(datagen.to_csr(words), variant, bits, mp)
    w = np.array([weight(f, variant, bits) for f in fps])
    n = len(fps)
    a = np.repeat(fps, n)
    b = np.tile(fps, n)
    fd = oracle.fd(a, b, variant, bits).astype(np.int64)
    gap = np.abs(np.repeat(w, n) - np.tile(w, n))
    assert (fd >= gap).all()
    # the bound is tight somewhere (a pair whose fields nest), so it is the
    # right quantity and not a looser one
    assert (fd == gap).any() and (gap > 0).any()
    # so every pruned pair fails the filter at every threshold the library uses
    for k in (1, 2, 3):
        t = oracle.threshold(variant, k)
        assert not ((gap > t) & (fd <= t)).any()
