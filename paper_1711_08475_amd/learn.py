"""Driver of the learned symbol-to-field grouping.

Steps (all matching arithmetic runs in libfpm's kernels; this module only
samples indices and moves arrays):

1. sample (query, word) pairs uniformly among length-compatible pairs
   (|m - n| <= k) of a training query set against the dictionary;
2. label them with the library's exact verifier (``fpm_verify_pairs``) and
   add every true match of the training queries (``fpm_match``);
3. train the grouping model on the GPU (``fpm_learn_grouping``);
4. evaluate the hardened map against the paper's map on held-out queries --
   the filter's rejection rate over all length-compatible pairs, and the
   match list, which must be identical -- and fall back to the paper's map
   when the learned one does not reject more.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import datagen, fpm

HERE = os.path.dirname(os.path.abspath(__file__))
MAP_DIR = os.path.join(HERE, "maps")


def sample_compatible_pairs(dictionary, queries, n_pairs: int, k: int, seed: int) -> np.ndarray:
    """n_pairs (query, word) pairs, uniform over pairs with |m - n| <= k."""
    rng = np.random.default_rng([seed, 0x9A1])
    ld = datagen.csr_lengths(dictionary)
    lq = datagen.csr_lengths(queries)
    order = np.argsort(ld, kind="stable")
    cnt = np.bincount(ld, minlength=256 + k + 1)
    start = np.concatenate([[0], np.cumsum(cnt)])
    comp = np.zeros(lq.size, dtype=np.float64)
    for dl in range(-k, k + 1):
        L = lq + dl
        ok = (L >= 0) & (L < cnt.size)
        comp[ok] += cnt[L[ok]]
    if comp.sum() == 0:
        return np.zeros((0, 2), dtype=np.uint32)
    qi = rng.choice(lq.size, size=n_pairs, p=comp / comp.sum())
    # pick the word length with probability proportional to its bucket size
    m = lq[qi]
    u = rng.random(n_pairs) * comp[qi]
    L = np.full(n_pairs, -1, dtype=np.int64)
    acc = np.zeros(n_pairs)
    for dl in range(-k, k + 1):
        cand = m + dl
        ok = (cand >= 0) & (cand < cnt.size)
        c = np.where(ok, cnt[np.clip(cand, 0, cnt.size - 1)], 0)
        pick = (L < 0) & (u < acc + c) & (c > 0)
        L[pick] = cand[pick]
        acc += c
    r = (rng.random(n_pairs) * cnt[L]).astype(np.int64)
    w = order[start[L] + r]
    return np.stack([qi, w], axis=1).astype(np.uint32)


def label_pairs(index, queries, pairs: np.ndarray, k: int):
    """Exact Levenshtein distance <= k flags from the library verifier, with
    every true match of the queries appended."""
    dist = fpm.fpm_verify_pairs(index, queries, pairs, "lev", k)
    matches = fpm.fpm_match(index, queries, "lev", k)[:, :2]
    all_pairs = np.concatenate([pairs, matches]).astype(np.uint32)
    is_match = np.concatenate([dist <= k, np.ones(matches.shape[0], dtype=bool)])
    return all_pairs, is_match


def config(bits=16, k=1, epochs=40, batch=65536, lr=0.01, margin=0.5, beta=2.0, entropy_weight=0.05, hidden=64,
           seed=1):
    return fpm.LearnConfig(bits=bits, k=k, hidden=hidden, epochs=epochs, batch=batch, lr=lr, margin=margin,
                           beta=beta, entropy_weight=entropy_weight, seed=seed)


def rejection(index, queries, k: int):
    """(rejection rate over examined pairs, stats, match list) of a match."""
    res, st = fpm.fpm_match(index, queries, "lev", k, fpm.options(schedule=fpm.FPM_SCHED_BATCHED), with_stats=True)
    return 1.0 - st["survivors"] / max(st["pairs_examined"], 1), st, res


def learn_grouping(dictionary, train_queries, bits=16, k=1, n_pairs=2_000_000, seed=1, cfg=None):
    """Train a grouping for `dictionary`; returns (map, report)."""
    paper_ix = fpm.fpm_build_fingerprints(dictionary, "occ", bits, "common")
    pairs = sample_compatible_pairs(dictionary, train_queries, n_pairs, k, seed)
    all_pairs, is_match = label_pairs(paper_ix, train_queries, pairs, k)
    mp, rep = fpm.fpm_learn_grouping(dictionary, train_queries, all_pairs, is_match,
                                     cfg if cfg is not None else config(bits=bits, k=k, seed=seed))
    rep["labelled_pairs"] = int(all_pairs.shape[0])
    rep["labelled_matches"] = int(is_match.sum())
    return mp, rep


def evaluate(dictionary, heldout_queries, learned_map, bits=16, k=1):
    """Compare the learned map with the paper's common map on held-out
    queries.  Raises if the match lists differ (a grouping must never drop
    or add a match)."""
    paper_ix = fpm.fpm_build_fingerprints(dictionary, "occ", bits, "common")
    learned_ix = fpm.fpm_build_fingerprints(dictionary, "occ", bits, custom_map=learned_map)
    rp, sp, mp_ = rejection(paper_ix, heldout_queries, k)
    rl, sl, ml = rejection(learned_ix, heldout_queries, k)
    if not np.array_equal(mp_, ml):
        raise AssertionError("learned map changed the match list")
    return {"paper_rejection": rp, "learned_rejection": rl, "paper_survivors": sp["survivors"],
            "learned_survivors": sl["survivors"], "examined": sp["pairs_examined"], "matches": int(ml.shape[0])}


def choose_map(dictionary, heldout_queries, learned_map, bits=16, k=1):
    """The learned map when it rejects more held-out pairs, else the paper's
    common map (the fallback); returns (map, which, evaluation)."""
    ev = evaluate(dictionary, heldout_queries, learned_map, bits, k)
    if ev["learned_rejection"] > ev["paper_rejection"]:
        return learned_map, "learned", ev
    return fpm.fpm_get_map(fpm.fpm_build_fingerprints(dictionary, "occ", bits, "common")), "paper", ev


def save_map(name: str, mp: np.ndarray, meta: dict):
    os.makedirs(MAP_DIR, exist_ok=True)
    with open(os.path.join(MAP_DIR, name + ".json"), "w") as f:
        json.dump({"map": [int(x) for x in mp], **meta}, f, indent=1)


def load_map(name: str):
    path = os.path.join(MAP_DIR, name + ".json")
    if not os.path.exists(path):
        return None, None
    d = json.load(open(path))
    return np.array(d.pop("map"), dtype=np.uint8), d


def main(argv=None):
    """Train, evaluate and store the grouping of a named workload:
    ``python -m paper_1711_08475_amd.learn --workload english_1m_q10k --bits 16``."""
    import argparse
    import time

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--workload", default="english_1m_q10k")
    ap.add_argument("--bits", type=int, default=16)
    ap.add_argument("--k", type=int, default=1)
    ap.add_argument("--pairs", type=int, default=2_000_000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--lr", type=float, default=0.01)
    ap.add_argument("--entropy-weight", type=float, default=0.05)
    ap.add_argument("--margin", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default=None, help="map name (default: <workload>_occ<bits>_k<k>)")
    a = ap.parse_args(argv)
    d, q = datagen.workload(a.workload)
    tq = datagen.training_queries(a.workload)
    cfg = config(bits=a.bits, k=a.k, epochs=a.epochs, lr=a.lr, entropy_weight=a.entropy_weight, margin=a.margin,
                 seed=a.seed)
    t = time.time()
    mp, rep = learn_grouping(d, tq, bits=a.bits, k=a.k, n_pairs=a.pairs, seed=a.seed, cfg=cfg)
    chosen, which, ev = choose_map(d, q, mp, bits=a.bits, k=a.k)
    meta = {"workload": a.workload, "bits": a.bits, "k": a.k, "chosen": which, "training": rep, "evaluation": ev,
            "config": {f: getattr(cfg, f) for f, _ in cfg._fields_}, "pairs": a.pairs,
            "learned_map": [int(x) for x in mp], "seconds": time.time() - t,
            "heldout": f"the {a.workload} queries; training queries drawn with seed offset "
                       f"{datagen.TRAINING_QUERY_SEED_OFFSET}"}
    name = a.out or f"{a.workload}_occ{a.bits}_k{a.k}"
    save_map(name, chosen, meta)
    print(json.dumps({"name": name, "chosen": which, **ev, "train_ms": rep["ms"]}))


if __name__ == "__main__":
    main()
