"""Host-side model of the matrix-core filter's arithmetic (CPU only).

F_D of 16-bit keys is computed as an 8-bit integer contraction: key bit j
is +1 / -1 on the query side (clear / set) and -1 / +1 on the word side, so
a row-column product over the key positions is 2 F_D - 16; one spare
position carries 2t - 15 on the query side against -1 on the word side, so
the product is 2 F_D - 2t - 1, negative exactly when F_D <= t (Eq. 1,
t = 2k; bigrams 4k).  These tests rebuild the byte rows and columns, the
32 x 32 x 32 tile's lane layout and the query-row permutation with numpy,
and check that the sign bits land in the mask bit of the right query --
the index arithmetic the kernel relies on, independent of the GPU."""
import numpy as np
import pytest


def popc(x):
    return np.array([bin(int(v)).count("1") for v in np.ravel(x)]).reshape(np.shape(x))


def nibble_sel(nib):
    # byte i of (nib * 0x00810204) & 0x04040404 is 4 * bit i of nib
    return (int(nib) * 0x00810204) & 0x04040404


def perm_bytes(s0, s1, sel):
    # selector byte 0..3 picks that byte of s1, 4..7 that byte of s0 - 4
    src = list(int(s1).to_bytes(4, "little")) + list(int(s0).to_bytes(4, "little"))
    return bytes(src[(sel >> (8 * i)) & 0xFF] for i in range(4))


def signed(b):
    return np.frombuffer(bytes(b), dtype=np.int8).astype(np.int64)


def query_row(key, t, threshold_byte=None):
    row = bytearray(32)
    for d, nib_shift in ((0, 0), (4, 4), (16, 8), (20, 12)):
        row[d:d + 4] = perm_bytes(0xFFFFFFFF, 0x01010101, nibble_sel((key >> nib_shift) & 15))
    row[8] = (2 * t - 15 if threshold_byte is None else threshold_byte) & 0xFF
    return signed(row)


def word_column(key):
    col = bytearray(32)
    for h in (0, 1):
        x = key >> (8 * h)
        col[16 * h:16 * h + 4] = perm_bytes(0x01010101, 0xFFFFFFFF, nibble_sel(x & 15))
        col[16 * h + 4:16 * h + 8] = perm_bytes(0x01010101, 0xFFFFFFFF, nibble_sel((x >> 4) & 15))
        col[16 * h + 8:16 * h + 16] = b"\xff" * 8
    return signed(col)


def test_nibble_spread_is_exact():
    for nib in range(16):
        sel = nibble_sel(nib)
        assert [(sel >> (8 * i)) & 0xFF for i in range(4)] == [4 * ((nib >> i) & 1) for i in range(4)]


@pytest.mark.parametrize("t", [2, 4, 6, 8, 12])
def test_product_is_twice_fd_minus_threshold(t):
    rng = np.random.default_rng(t)
    qs = rng.integers(0, 1 << 16, 300)
    ws = rng.integers(0, 1 << 16, 300)
    # keys near each other too, so that both signs occur
    ws[:150] = qs[:150] ^ (1 << rng.integers(0, 16, 150)) ^ (1 << rng.integers(0, 16, 150))
    A = np.stack([query_row(int(q), t) for q in qs])
    B = np.stack([word_column(int(w)) for w in ws])
    prod = A @ B.T
    fd = popc(qs[:, None] ^ ws[None, :])
    assert np.array_equal(prod, 2 * fd - 2 * t - 1)
    assert np.array_equal(prod < 0, fd <= t)
    assert (prod < 0).any() and (prod >= 0).any()


def test_tile_layout_and_row_permutation():
    """v_mfma_i32_32x32x32_i8 layout (lane l: A row / B column l % 32, bytes
    16 (l / 32) .. + 15 of the contraction; result register r of lane l:
    row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32).  With tile t's row
    i holding query 32 ((i / 4) % 2) + 16 t + 4 (i / 8) + i % 4, shifting
    tile 1's registers 15..0 and then tile 0's into a mask leaves bit b of
    lane l's mask = query 32 (l / 32) + b against word l % 32."""
    rng = np.random.default_rng(3)
    t = 2
    qkeys = rng.integers(0, 1 << 16, 64)
    wkeys = rng.integers(0, 1 << 16, 32)
    wkeys[::3] = qkeys[:32:3] ^ 1  # some survivors
    rows = np.stack([query_row(int(k), t) for k in qkeys])
    cols = np.stack([word_column(int(k)) for k in wkeys])

    def qrow(i, tile):
        return 32 * ((i >> 2) & 1) + 16 * tile + 4 * (i >> 3) + (i & 3)

    masks = np.zeros(64, dtype=np.uint64)
    for tile in (1, 0):
        A = np.stack([rows[qrow(i, tile)] for i in range(32)])  # A[i] = row i of the tile
        D = A @ cols.T  # D[i, j]
        for lane in range(64):
            # each lane feeds its 16 contraction bytes; the product is the same
            for r in range(15, -1, -1):
                i = 8 * (r // 4) + 4 * (lane // 32) + r % 4
                sign = 1 if D[i, lane % 32] < 0 else 0
                masks[lane] = ((int(masks[lane]) << 1) | sign) & 0xFFFFFFFF
    for lane in range(64):
        h, j = lane // 32, lane % 32
        for b in range(32):
            q = 32 * h + b
            want = bin(int(qkeys[q]) ^ int(wkeys[j])).count("1") <= t
            assert ((int(masks[lane]) >> b) & 1) == int(want)


@pytest.mark.parametrize("t", [2, 4, 6, 12])
def test_two_part_product_for_32_bit_keys(t):
    """32-bit keys: bits 0..15 with the threshold byte 2t - 31, then bits
    16..31 with a zero threshold byte, the second product accumulated onto
    the first: (2 F_D0 - 16 + 31 - 2t) + (2 F_D1 - 16) = 2 F_D - 2t - 1."""
    rng = np.random.default_rng(40 + t)
    qs = rng.integers(0, 1 << 32, 200, dtype=np.uint64)
    ws = rng.integers(0, 1 << 32, 200, dtype=np.uint64)
    ws[:100] = qs[:100] ^ (np.uint64(1) << rng.integers(0, 32, 100).astype(np.uint64))
    A0 = np.stack([query_row(int(q) & 0xFFFF, t, 2 * t - 31) for q in qs])
    A1 = np.stack([query_row(int(q) >> 16, t, 0) for q in qs])
    B0 = np.stack([word_column(int(w) & 0xFFFF) for w in ws])
    B1 = np.stack([word_column(int(w) >> 16) for w in ws])
    prod = A0 @ B0.T + A1 @ B1.T
    fd = popc(qs[:, None] ^ ws[None, :])
    assert np.array_equal(prod, 2 * fd - 2 * t - 1)
    assert np.array_equal(prod < 0, fd <= t)
    assert (prod < 0).any() and (prod >= 0).any()
