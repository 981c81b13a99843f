"""Word-size sweep on the GPU: the axis of the paper's Fig. 1 (Hamming
comparison time against word size on synthetic English-like data, for the
occurrence, count and position fingerprints).

For each word length L, a dictionary of English-like words of that single
length and queries of the same length (half of them dictionary words with
one substitution) are matched under Hamming k = 1 twice on the GPU: by the
fingerprint filter (batched schedule, tiles picked by the autotuner) and by
the no-fingerprint brute force (every pair verified).  The speedup is the
paper's S = T_naive / T_filter; the rejection rate is 1 - survivors /
examined pairs.  Both runs must return the same match list.

    python -m paper_1711_08475_amd.lensweep [--words N] [--queries Q] [--lengths 4,6,...]

Prints one JSON object per (length, fingerprint) and a table at the end.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def time_plan(fpm, torch, plan, qb, qo, nq, steps, warmup):
    for _ in range(warmup):
        fpm.fpm_plan_run(plan, qb.data_ptr(), qo.data_ptr(), nq)
        fpm.fpm_plan_result(plan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fpm.fpm_plan_run(plan, qb.data_ptr(), qo.data_ptr(), nq)
    _, n, st = fpm.fpm_plan_result(plan)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, st


def parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--words", type=int, default=1_000_000)
    ap.add_argument("--queries", type=int, default=10_000)
    ap.add_argument("--lengths", default="4,6,8,10,12,14,16,18,20")
    ap.add_argument("--variants", default="occ,count,pos")
    ap.add_argument("--bits", type=int, default=16)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=41)
    ap.add_argument("--filter-unit", default="auto", choices=["auto", "valu", "matrix"],
                    help="where the filter test runs (fpm_options.filter_unit)")
    ap.add_argument("--pop-prune", default="off", choices=["off", "on"],
                    help="popcount pruning of the filtered form (fpm_options.pop_prune)")
    return ap.parse_args(argv)


def run(args, on_row=None):
    """The sweep: a list of (row, match list, symbol map) per (length,
    fingerprint); on_row(row) is called as each row is done."""
    import torch

    from paper_1711_08475_amd import datagen, fpm

    fpm.lib()
    out = []
    for L in [int(x) for x in args.lengths.split(",")]:
        d, q = datagen.fixed_length_workload(args.words, args.queries, L, args.seed + L)
        nq, qbytes = q[1].size - 1, int(q[1][-1])
        qb = torch.from_numpy(q[0].copy()).cuda()
        qo = torch.from_numpy(q[1].view(np.int64).copy()).cuda()
        torch.cuda.synchronize()
        brute_ms = None
        ref = None
        for variant in args.variants.split(","):
            ix = fpm.fpm_build_fingerprints(d, variant, args.bits, "common")
            if brute_ms is None:
                plan = fpm.fpm_plan_create(ix, nq, qbytes, "ham", 1, fpm.options(schedule=fpm.FPM_SCHED_BRUTE))
                brute_ms, _ = time_plan(fpm, torch, plan, qb, qo, nq, args.steps, args.warmup)
                ref = fpm.fpm_plan_copy_matches(plan)
                del plan
            best, _ = fpm.fpm_autotune(ix, qb.data_ptr(), qo.data_ptr(), nq, qbytes, "ham", 1, 2,
                                       base=fpm.options(filter_unit=args.filter_unit, pop_prune=args.pop_prune))
            plan = fpm.fpm_plan_create(ix, nq, qbytes, "ham", 1, best)
            ms, st = time_plan(fpm, torch, plan, qb, qo, nq, args.steps, args.warmup)
            got = fpm.fpm_plan_copy_matches(plan)
            del plan
            if not np.array_equal(got, ref):
                raise SystemExit(f"length {L} {variant}: filtered and brute-force match lists differ")
            row = {
                "length": L,
                "fingerprint": f"{variant}{args.bits}",
                "words": args.words,
                "queries": args.queries,
                "filtered_ms": ms,
                "brute_ms": brute_ms,
                "speedup": brute_ms / ms,
                "rejection_rate": 1.0 - st["survivors"] / max(st["pairs_examined"], 1),
                "filter_unit": {1: "valu", 2: "matrix"}.get(st.get("filter_unit"), "none"),
                "pairs_per_s": nq * args.words / (ms * 1e-3),
                "matches": int(got.shape[0]),
                "examined": st["pairs_examined"],
                "survivors": st["survivors"],
                "tested": st["pairs_filtered"],
                "tiles": [best.queries_per_item, best.slab, best.bucket_order, best.tail_split],
            }
            out.append((row, got, fpm.fpm_get_map(ix)))
            if on_row:
                on_row(row)
    return out


def main(argv=None):
    args = parse(argv)
    import torch

    if not torch.cuda.is_available():
        print("the sweep needs a GPU", file=sys.stderr)
        return 2
    rows = [r for r, _, _ in run(args, on_row=lambda row: print(json.dumps(row), flush=True))]
    variants = [f"{v}{args.bits}" for v in args.variants.split(",")]
    print("| length | brute ms | " + " | ".join(f"{v} ms (speedup, rejection)" for v in variants) + " |")
    print("|---|---|" + "---|" * len(variants))
    for L in sorted({r["length"] for r in rows}):
        rs = {r["fingerprint"]: r for r in rows if r["length"] == L}
        cells = [f"{rs[v]['filtered_ms']:.3f} ({rs[v]['speedup']:.1f}x, {100 * rs[v]['rejection_rate']:.1f}%)"
                 for v in variants if v in rs]
        print(f"| {L} | {next(iter(rs.values()))['brute_ms']:.3f} | " + " | ".join(cells) + " |")
    return 0


if __name__ == "__main__":
    sys.exit(main())
