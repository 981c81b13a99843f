"""Host-side model of the matrix-core filter's arithmetic (CPU only).

F_D of W-bit keys (W = 16 or 32) is computed as an 8-bit integer
contraction: key bit j is +1 / -1 on the query side (clear / set) and -1 /
+1 on the word side, so a row-column product over the W key positions is
2 F_D - W; the accumulator input W - 1 - 2t makes the output 2 F_D - 2t - 1,
negative exactly when F_D <= t (Eq. 1, t = 2k; bigrams 4k).  The second
tile of a pass takes doubled query bytes and the constant 2W - 1 - 4t
(output 4 F_D - 4t - 1, same sign).  These tests rebuild the byte rows and
columns, the 32 x 32 tile's lane layout and the query-row permutation with
numpy, and check that the sign bits land in the mask bit of the right
query -- the index arithmetic the kernel relies on, independent of the
GPU."""
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


def query_row(key, width):
    """The expanded query row: byte j = +1 (0x01) for a clear bit j, -1
    (0xFF) for a set one (nibble by nibble, as the expansion kernel)."""
    row = bytearray(width)
    for n in range(width // 4):
        row[4 * n:4 * n + 4] = perm_bytes(0xFFFFFFFF, 0x01010101, nibble_sel((key >> (4 * n)) & 15))
    return signed(row)


def twice(row):
    # the kernel's (x << 1) & 0xFE per byte: +1 -> +2, -1 -> -2
    b = (row.astype(np.int64) & 0xFF)
    return signed(bytes(int(((v << 1) & 0xFE)) for v in b))


def word_column(key, width):
    """Concatenation of the two lane halves' contraction bytes: half h holds
    key bits (W / 2) h .. + W / 2 - 1, +1 for a set bit, -1 for a clear one."""
    col = bytearray(width)
    for h in (0, 1):
        x = key >> ((width // 2) * h)
        for n in range(width // 8):
            col[(width // 2) * h + 4 * n:(width // 2) * h + 4 * n + 4] = perm_bytes(
                0x01010101, 0xFFFFFFFF, nibble_sel((x >> (4 * n)) & 15))
    return signed(col)


def test_nibble_spread_is_exact():
    for nib in range(16):
        sel = nibble_sel(nib)
        assert [(sel >> (8 * i)) & 0xFF for i in range(4)] == [4 * ((nib >> i) & 1) for i in range(4)]


@pytest.mark.parametrize("width", [16, 32])
@pytest.mark.parametrize("t", [2, 4, 6, 8, 12])
def test_product_plus_constant_is_the_threshold_test(width, t):
    rng = np.random.default_rng(t + width)
    qs = rng.integers(0, 1 << width, 300, dtype=np.uint64)
    ws = rng.integers(0, 1 << width, 300, dtype=np.uint64)
    # keys near each other too, so that both signs occur
    one = np.uint64(1)
    ws[:150] = qs[:150] ^ (one << rng.integers(0, width, 150).astype(np.uint64)) ^ \
        (one << rng.integers(0, width, 150).astype(np.uint64))
    A = np.stack([query_row(int(q), width) for q in qs])
    B = np.stack([word_column(int(w), width) for w in ws])
    fd = popc(qs[:, None] ^ ws[None, :])
    prod1 = A @ B.T + (width - 1 - 2 * t)
    assert np.array_equal(prod1, 2 * fd - 2 * t - 1)
    prod0 = np.stack([twice(r) for r in A]) @ B.T + (2 * width - 1 - 4 * t)
    assert np.array_equal(prod0, 4 * fd - 4 * t - 1)
    assert np.array_equal(prod1 < 0, fd <= t) and np.array_equal(prod0 < 0, fd <= t)
    assert (prod1 < 0).any() and (prod1 >= 0).any()


def test_unused_key_positions_count_as_equal_bits():
    """A 24-bit thermometer key (16-bit count fingerprints) in the 32-bit
    tile: its clear top 8 bits are equal positions (-1 each), so the product
    is still 2 F_D - 32."""
    rng = np.random.default_rng(5)
    qs = rng.integers(0, 1 << 24, 100)
    ws = rng.integers(0, 1 << 24, 100)
    A = np.stack([query_row(int(q), 32) for q in qs])
    B = np.stack([word_column(int(w), 32) for w in ws])
    assert np.array_equal(A @ B.T, 2 * popc(qs[:, None] ^ ws[None, :]) - 32)


@pytest.mark.parametrize("width", [16, 32])
def test_inline_constants_fit(width):
    """Both accumulator constants are inline integer constants (-16 .. 64)
    for every threshold the library uses except 16-bit bigrams at k = 3,
    whose second constant the compiler keeps in registers."""
    for t in (2, 4, 6, 8, 12):
        assert -16 <= width - 1 - 2 * t <= 64
        c0 = 2 * width - 1 - 4 * t
        assert (-16 <= c0 <= 64) == (not (width == 16 and t == 12))


@pytest.mark.parametrize("width", [16, 32])
def test_tile_layout_and_row_permutation(width):
    """32 x 32 tile layout (lane l: A row / B column l % 32, contraction
    bytes of half l / 32; result register r of lane l: row 8 (r / 4) +
    4 (l / 32) + r % 4, column l % 32).  With tile t's row i holding query
    32 ((i / 4) % 2) + 16 t + 4 (i / 8) + i % 4, shifting tile 1's registers
    15..0 and then tile 0's into a mask leaves bit b of lane l's mask =
    query 32 (l / 32) + b against word l % 32."""
    rng = np.random.default_rng(3)
    t = 2
    qkeys = rng.integers(0, 1 << width, 64)
    wkeys = rng.integers(0, 1 << width, 32)
    wkeys[::3] = qkeys[:32:3] ^ 1  # some survivors
    rows = np.stack([query_row(int(k), width) for k in qkeys])
    cols = np.stack([word_column(int(k), width) for k in wkeys])

    def qrow(i, tile):
        return 32 * ((i >> 2) & 1) + 16 * tile + 4 * (i >> 3) + (i & 3)

    masks = np.zeros(64, dtype=np.uint64)
    for tile in (1, 0):
        A = np.stack([rows[qrow(i, tile)] for i in range(32)])  # A[i] = row i of the tile
        if tile == 0:
            A = np.stack([twice(r) for r in A])
            D = A @ cols.T + (2 * width - 1 - 4 * t)
        else:
            D = A @ cols.T + (width - 1 - 2 * t)
        for lane in range(64):
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
