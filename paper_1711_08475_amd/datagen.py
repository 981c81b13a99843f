"""Seeded synthetic workloads for approximate dictionary matching.

This module only draws strings; it holds none of the matching method's
arithmetic (no fingerprints, no distances), so the HIP path and the CPU oracle
can both be fed from it.

The paper's datasets (synthetic English built from letter frequencies, an
English word list, a URL crawl; Section 4) are not available, so seeded
stand-ins with the same shape replace them:

* English-like words: letters a-z, i.i.d., with Zipf(1.0) unigram weights over
  a seeded permutation of the alphabet; binomial length laws.
* URL-like strings: 72 symbols (a-z, A-Z, 0-9, ``-._~:/?=&%``), a scheme, a
  Zipf-drawn host from a seeded vocabulary, 2-7 path segments from a per-host
  Zipf vocabulary and a suffix; lengths 20-120 with shared prefixes.
* Queries: a fraction ``rho`` are dictionary words with ``e`` random edits
  (substitution / insertion / deletion, equally likely, uniform position),
  the rest fresh generator strings.

Strings are returned in CSR form: ``(bytes uint8[total], offsets uint64[n+1])``.
"""
from __future__ import annotations

import numpy as np

LETTERS = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz", dtype=np.uint8)
URL_EXTRA = b"-._~:/?=&%"
URL_ALPHABET = b"abcdefghijklmnopqrstuvwxyz" + b"ABCDEFGHIJKLMNOPQRSTUVWXYZ" + b"0123456789" + URL_EXTRA


def to_csr(strings) -> tuple[np.ndarray, np.ndarray]:
    items = [s.encode("latin-1") if isinstance(s, str) else bytes(s) for s in strings]
    offs = np.zeros(len(items) + 1, dtype=np.uint64)
    if items:
        offs[1:] = np.cumsum([len(s) for s in items], dtype=np.uint64)
    data = np.frombuffer(b"".join(items), dtype=np.uint8).copy()
    return data, offs


def from_csr(csr) -> list[bytes]:
    b, o = csr
    raw = b.tobytes()
    return [raw[int(o[i]):int(o[i + 1])] for i in range(o.size - 1)]


def csr_lengths(csr) -> np.ndarray:
    return np.diff(csr[1]).astype(np.int64)


def concat_csr(a, b):
    ob = b[1][1:] + a[1][-1]
    return np.concatenate([a[0], b[0]]), np.concatenate([a[1], ob])


def take_csr(csr, idx) -> tuple[np.ndarray, np.ndarray]:
    """Sub-list of strings ``idx`` (in that order)."""
    b, o = csr
    idx = np.asarray(idx, dtype=np.int64)
    starts = o[:-1][idx].astype(np.int64)
    lens = (o[1:][idx] - o[:-1][idx]).astype(np.int64)
    offs = np.zeros(idx.size + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(lens)
    if idx.size == 0 or offs[-1] == 0:
        return np.zeros(0, dtype=np.uint8), offs
    rel = np.arange(int(offs[-1]), dtype=np.int64) - np.repeat(offs[:-1].astype(np.int64), lens)
    src = np.repeat(starts, lens) + rel
    return b[src], offs


def zipf_weights(n: int, s: float = 1.0) -> np.ndarray:
    w = 1.0 / np.arange(1, n + 1, dtype=np.float64) ** s
    return w / w.sum()


class EnglishLike:
    """Letters a-z with Zipf(1.0) weights over a seeded rank permutation."""

    def __init__(self, seed: int):
        rng = np.random.default_rng([seed, 0xE1])
        perm = rng.permutation(26)
        self.probs = np.zeros(26)
        self.probs[perm] = zipf_weights(26, 1.0)
        self.symbols = LETTERS

    def draw(self, rng, n: int) -> np.ndarray:
        return self.symbols[rng.choice(26, size=n, p=self.probs)]


def english_lengths(rng, n: int, law: str) -> np.ndarray:
    if law == "3-15":  # 3 + Binomial(12, 1/3): 3..15, mode 7
        return 3 + rng.binomial(12, 1.0 / 3.0, size=n)
    if law == "2-20":  # 2 + Binomial(18, 5/18): 2..20, mode 7
        return 2 + rng.binomial(18, 5.0 / 18.0, size=n)
    if law.startswith("fixed:"):  # every word of one length
        return np.full(n, int(law[6:]), dtype=np.int64)
    raise ValueError(law)


def english_words(n: int, seed: int, law: str = "2-20", alphabet: EnglishLike | None = None):
    rng = np.random.default_rng([seed, 0xE2])
    alpha = alphabet or EnglishLike(seed)
    lens = english_lengths(rng, n, law).astype(np.int64)
    offs = np.zeros(n + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(lens)
    data = alpha.draw(rng, int(offs[-1]))
    return data.astype(np.uint8), offs


class UrlLike:
    """URL-like strings: scheme + Zipf host + Zipf path segments + suffix."""

    TLDS = [b".com", b".org", b".net", b".io", b".info", b".edu", b".biz", b".co"]
    SUFFIXES = [b"", b"/", b".html", b".htm", b".php", b"?id=", b"?p=", b"/index.html", b"&s=", b"%20"]

    def __init__(self, seed: int, n_hosts: int = 256, n_segments: int = 64):
        rng = np.random.default_rng([seed, 0x71])
        self.lower = EnglishLike(seed + 1)
        seg_syms = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz0123456789ABCDEFGHIJKLMNOPQRSTUVWXYZ-_~", dtype=np.uint8)
        w = np.concatenate([self.lower.probs * 0.80, np.full(10, 0.12 / 10), np.full(26, 0.06 / 26), np.full(3, 0.02 / 3)])
        self.seg_syms, self.seg_probs = seg_syms, w / w.sum()
        self.hosts = []
        for _ in range(n_hosts):
            label = bytes(self.lower.draw(rng, int(rng.integers(5, 15))))
            www = b"www." if rng.random() < 0.5 else b""
            self.hosts.append(www + label + self.TLDS[int(rng.integers(len(self.TLDS)))])
        self.host_w = zipf_weights(n_hosts, 1.1)
        self.segments = []
        for _ in range(n_hosts):
            segs = []
            for _ in range(n_segments):
                L = int(rng.integers(3, 15))
                segs.append(bytes(self.seg_syms[rng.choice(self.seg_syms.size, size=L, p=self.seg_probs)]))
            self.segments.append(segs)
        self.seg_w = zipf_weights(n_segments, 1.0)

    def draw_symbols(self, rng, n: int) -> np.ndarray:
        return self.seg_syms[rng.choice(self.seg_syms.size, size=n, p=self.seg_probs)]

    def urls(self, n: int, rng) -> list[bytes]:
        out: list[bytes] = []
        while len(out) < n:
            m = (n - len(out)) * 2 + 16
            hosts = rng.choice(len(self.hosts), size=m, p=self.host_w)
            https = rng.random(m) < 0.2
            nseg = rng.integers(2, 8, size=m)
            segs = rng.choice(len(self.seg_w), size=(m, 7), p=self.seg_w)
            suf = rng.integers(0, len(self.SUFFIXES), size=m)
            digits = rng.integers(0, 100000, size=m)
            for i in range(m):
                h = int(hosts[i])
                parts = [b"https://" if https[i] else b"http://", self.hosts[h]]
                sv = self.segments[h]
                for t in range(int(nseg[i])):
                    parts.append(b"/")
                    parts.append(sv[int(segs[i, t])])
                s = self.SUFFIXES[int(suf[i])]
                parts.append(s)
                if s.endswith(b"="):
                    parts.append(str(int(digits[i])).encode())
                u = b"".join(parts)
                if 20 <= len(u) <= 120:
                    out.append(u)
                    if len(out) == n:
                        break
        return out


def url_strings(n: int, seed: int, gen: UrlLike | None = None):
    g = gen or UrlLike(seed)
    rng = np.random.default_rng([seed, 0x72])
    return to_csr(g.urls(n, rng))


def distort(word: bytes, edits: int, rng, draw_symbols, min_len: int, max_len: int = 255) -> bytes:
    """Apply ``edits`` random edits: substitution (must change the symbol),
    insertion or deletion, equally likely, at a uniform position; deletions
    never go below ``min_len`` and insertions never above ``max_len``."""
    w = bytearray(word)
    for _ in range(edits):
        while True:
            op = int(rng.integers(3))
            if op == 0 and len(w) > 0:
                i = int(rng.integers(len(w)))
                c = int(draw_symbols(rng, 1)[0])
                while c == w[i]:
                    c = int(draw_symbols(rng, 1)[0])
                w[i] = c
                break
            if op == 1 and len(w) < max_len:
                i = int(rng.integers(len(w) + 1))
                w.insert(i, int(draw_symbols(rng, 1)[0]))
                break
            if op == 2 and len(w) > min_len:
                del w[int(rng.integers(len(w)))]
                break
    return bytes(w)


def make_queries(dictionary, n: int, seed: int, rho: float, edit_choices, fresh, draw_symbols, min_len: int):
    """``n`` queries: with probability ``rho`` a random dictionary word with
    ``rng.choice(edit_choices)`` edits, else a fresh string from ``fresh``."""
    rng = np.random.default_rng([seed, 0x51])
    words = dictionary
    nd = words[1].size - 1
    near = rng.random(n) < rho
    n_fresh = int((~near).sum())
    fresh_list = from_csr(fresh(n_fresh, rng)) if n_fresh else []
    out, fi = [], 0
    raw, offs = words[0].tobytes(), words[1]
    for i in range(n):
        if near[i]:
            j = int(rng.integers(nd))
            w = raw[int(offs[j]):int(offs[j + 1])]
            e = int(rng.choice(np.asarray(edit_choices)))
            out.append(distort(w, e, rng, draw_symbols, min_len))
        else:
            out.append(fresh_list[fi])
            fi += 1
    return to_csr(out)


# --------------------------------------------------------------------------
# Named workloads (sizes in the name; the queries-per-dictionary ratios and
# near-match rates are the ones the benchmarks use)
# --------------------------------------------------------------------------

def english_workload(n_words: int, n_queries: int, seed: int, law: str, rho: float, edit_choices=(1,),
                     query_seed: int | None = None):
    """Dictionary from `seed`; queries from `query_seed` (default: `seed`)."""
    qs = seed if query_seed is None else query_seed
    alpha = EnglishLike(seed)
    d = english_words(n_words, seed, law, alpha)

    def fresh(m, rng):
        r2 = np.random.default_rng([qs, 0x53, int(rng.integers(1 << 30))])
        return english_words(m, int(r2.integers(1 << 30)), law, alpha)

    q = make_queries(d, n_queries, qs, rho, edit_choices, fresh, alpha.draw, min_len=2 if law == "2-20" else 3)
    return d, q


def fixed_length_workload(n_words: int, n_queries: int, length: int, seed: int, rho: float = 0.5):
    """English-like words of one length (the single-length dictionaries of
    the paper's word-size experiment) and queries of the same length: with
    probability ``rho`` a dictionary word with one substitution, else a fresh
    word."""
    alpha = EnglishLike(seed)
    law = f"fixed:{length}"
    d = english_words(n_words, seed, law, alpha)
    rng = np.random.default_rng([seed, 0x5F, length])
    raw, offs = d[0], d[1]
    fresh = english_words(n_queries, seed + 7919, law, alpha)[0].reshape(n_queries, length) if length else None
    out = []
    for i in range(n_queries):
        if length and rng.random() < rho:
            j = int(rng.integers(n_words))
            w = bytearray(raw[int(offs[j]):int(offs[j + 1])].tobytes())
            pos = int(rng.integers(length))
            c = int(alpha.draw(rng, 1)[0])
            while c == w[pos]:
                c = int(alpha.draw(rng, 1)[0])
            w[pos] = c
            out.append(bytes(w))
        else:
            out.append(fresh[i].tobytes() if length else b"")
    return d, to_csr(out)


def url_workload(n_words: int, n_queries: int, seed: int, rho: float = 0.3, edit_choices=(1, 2),
                 query_seed: int | None = None):
    qs = seed if query_seed is None else query_seed
    gen = UrlLike(seed)
    d = url_strings(n_words, seed, gen)

    def fresh(m, rng):
        return to_csr(gen.urls(m, rng))

    q = make_queries(d, n_queries, qs, rho, edit_choices, fresh, gen.draw_symbols, min_len=20)
    return d, q


def mixed_workload(n_english: int, n_urls: int, n_queries: int, seed: int, rho: float = 0.3,
                   query_seed: int | None = None):
    """English-like (lengths 2-20) and URL-like (20-120) strings mixed 1:1 and
    shuffled; queries drawn the same way from both halves."""
    qs = seed if query_seed is None else query_seed
    alpha = EnglishLike(seed)
    gen = UrlLike(seed)
    de = english_words(n_english, seed, "2-20", alpha)
    du = url_strings(n_urls, seed, gen)
    rng = np.random.default_rng([seed, 0x4D])
    both = concat_csr(de, du)
    perm = rng.permutation(n_english + n_urls)
    d = take_csr(both, perm)
    qe = make_queries(de, n_queries // 2, qs + 11, rho, (1,),
                      lambda m, r: english_words(m, int(r.integers(1 << 30)), "2-20", alpha), alpha.draw, 2)
    qu = make_queries(du, n_queries - n_queries // 2, qs + 13, rho, (1,),
                      lambda m, r: to_csr(gen.urls(m, r)), gen.draw_symbols, 20)
    qb = concat_csr(qe, qu)
    qperm = np.random.default_rng([qs, 0x4E]).permutation(n_queries) if query_seed is not None \
        else rng.permutation(n_queries)
    return d, take_csr(qb, qperm)


WORKLOADS = {
    # 10,000 English-like words (lengths 3-15) x 1,000 queries, half near-matches
    "english_10k_q1k": (1, lambda seed, qs: english_workload(10_000, 1_000, seed, "3-15", 0.5, query_seed=qs)),
    # 1,000,000 English-like words (lengths 2-20) x 10,000 queries, 30% near-matches
    "english_1m_q10k": (2, lambda seed, qs: english_workload(1_000_000, 10_000, seed, "2-20", 0.3, query_seed=qs)),
    # 1,000,000 URL-like strings x 10,000 queries, 30% near-matches with 1 or 2 edits
    "url_1m_q10k": (3, lambda seed, qs: url_workload(1_000_000, 10_000, seed, 0.3, (1, 2), query_seed=qs)),
    # 2,000,000 mixed English/URL strings x 65,536 mixed queries
    "mixed_2m_q64k": (4, lambda seed, qs: mixed_workload(1_000_000, 1_000_000, 65_536, seed, query_seed=qs)),
}

TRAINING_QUERY_SEED_OFFSET = 1000


def workload(name: str, seed: int | None = None, query_seed: int | None = None):
    """(dictionary, queries) of a named workload."""
    default_seed, f = WORKLOADS[name]
    return f(default_seed if seed is None else seed, query_seed)


def training_queries(name: str):
    """Queries of workload `name` drawn with another seed (same dictionary,
    same query recipe): what a learned grouping is trained on, so the
    workload's own queries stay held out."""
    default_seed, f = WORKLOADS[name]
    return f(default_seed, default_seed + TRAINING_QUERY_SEED_OFFSET)[1]
