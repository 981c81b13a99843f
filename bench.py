#!/usr/bin/env python3
"""Levenshtein k=1 query-word pairs per second on one MI355X.

Workload (default): 1,000,000 synthetic English-like words (lengths 2-20,
Zipf letter weights) against 10,000 queries (30% are dictionary words with
one random edit), 16-bit occurrence fingerprints.  One step is one full
match of the query batch with inputs resident in HBM: query fingerprints,
length bucketing, work list, the fused filter + verify kernel and the sorted
match list.

Forms timed on the same GPU:
  plain        paper's common-symbol map, host-built work list, one wave per
               work item, default tiles, no graph;
  batched      persistent kernel over a device-built work list in a hipGraph,
               tiles picked by the autotuner;
  brute        no fingerprints: every length-compatible pair is verified (the
               paper's naive comparison, giving its speedup S = T_n / T_f);
  learned      the batched form with the symbol grouping learned by the MLP
               (paper_1711_08475_amd/maps/<workload>_occ<bits>_k1.json, written by
               `python -m paper_1711_08475_amd.learn`; --train retrains it here);
  asym         the learned form under the asymmetric bound (a filter rule
               beyond the paper: both one-directional excesses <= k), with
               popcount-ordered blocks and popcount-range tile skipping.
The headline is the paper's rule (learned); asym is reported beside it.

Device-scheduled forms keep several batches in flight (two or three, chosen
with the tiles and stored in the tuning table; --inflight overrides): that
many plans, each with its own stream and buffers, take steps in turn, so one
batch's preparation and match-list sort overlap another batch's match
kernel.  Every step is still the whole pipeline over one batch; the kernel
time in `roofline` is measured inside that timed, overlapped region.

Prints one JSON line.  `value` is the headline form's logical pairs/s
(|Q| * |D| / step time).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD_TEXT = {
    "english_10k_q1k": "10,000 English-like words (lengths 3-15) x 1,000 queries",
    "english_1m_q10k": "1,000,000 English-like words (lengths 2-20) x 10,000 queries",
    "url_1m_q10k": "1,000,000 URL-like strings (lengths 20-120) x 10,000 queries",
    "mixed_2m_q64k": "2,000,000 mixed English-like/URL-like strings x 65,536 mixed queries",
}


def metric_name(metric: str, k: int) -> str:
    return f"{'Lev' if metric == 'lev' else 'Ham'} k={k} query-word pairs/sec (1 MI355X), learned+batched vs plain filter"
PEAK_INT_OPS = 256 * 64 * 2.4e9  # CUs x lanes x clock: one 32-bit VALU op per lane per clock
PEAK_INT8_MATRIX_OPS = 5.0e15  # MI355X dense int8 matrix-core peak (ops/s)
# matrix-core filter: per pair the vector ALUs shift one sign bit into a
# survivor mask, and the matrix cores run a 32-deep int8 contraction
# (v_mfma_i32_32x32x32_i8: 2 x 32 ops per output)
MATRIX_VALU_OPS_PER_PAIR = 1
MATRIX_INT8_OPS_PER_PAIR = 64
FPM_UNIT_MATRIX = 2
# VALU instructions per examined pair in the vector filter loop (see fpm_match.hip)
FILTER_OPS = {("occ", 16): 3, ("occ", 32): 3, ("occh", 16): 3, ("occh", 32): 3, ("count", 16): 3, ("count", 32): 5,
              ("pos", 16): 8, ("pos", 32): 8, ("qgram", 16): 3, ("qgram", 32): 3,
              ("combo", 16): 6, ("combo", 32): 6}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "match_kernel_traffic.json")
TUNING_FILE = os.path.join(ROOT, "paper_1711_08475_amd", "tuned.json")
MATCH_SRC = os.path.join(ROOT, "paper_1711_08475_amd", "csrc", "fpm_match.hip")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    return hashlib.sha256(open(MATCH_SRC, "rb").read()).hexdigest()


def load_traffic(form: str, workload: str):
    """HBM bytes per launch of the match kernel from the committed rocprofv3
    counter runs of this form and workload, only while the kernel source is
    unchanged since."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    if t.get("form") != form or t.get("workload_name") != workload:
        return None
    return t


def roofline_of(st: dict, kernel_ms, variant: str, bits: int, traffic, peaks=None) -> dict:
    """Roofline of the match kernel: algorithmic VALU work per launch (the
    filter unit's VALU ops per examined pair + band cells of the survivors)
    over the kernel's measured duration, against the published int-VALU
    peak; on the matrix cores the int8 contraction is reported beside it.
    `peaks` (fpm_measure_peaks) adds the peaks measured on this device."""
    matrix = st.get("filter_unit") == FPM_UNIT_MATRIX
    per_pair = MATRIX_VALU_OPS_PER_PAIR if matrix else FILTER_OPS[(variant, bits)]
    ops = per_pair * st["pairs_examined"] + st["verify_cells"]
    achieved = ops / (kernel_ms * 1e-3) if kernel_ms else None
    roofline = {
        "bound": "alu",
        "achieved": achieved / 1e12 if achieved else None,
        "peak": PEAK_INT_OPS / 1e12,
        "unit": "Tops/s",
        "frac": achieved / PEAK_INT_OPS if achieved else None,
        "traffic": traffic["bytes_per_launch"] if traffic else None,
        "kernel": "k_match (fused filter + LDS queue + verify)",
        "filter_unit": "matrix" if matrix else "valu",
        "valu_ops_per_pair": per_pair,
        "ops_per_launch": ops,
        "kernel_ms": kernel_ms,
    }
    if peaks:
        roofline["peak_measured"] = peaks["int_valu_ops_per_s"] / 1e12
    if matrix and kernel_ms:
        m_ops = MATRIX_INT8_OPS_PER_PAIR * st["pairs_examined"]
        roofline["matrix_cores"] = {"achieved": m_ops / (kernel_ms * 1e-3) / 1e12,
                                    "peak": PEAK_INT8_MATRIX_OPS / 1e12, "unit": "int8 Tops/s",
                                    "frac": m_ops / (kernel_ms * 1e-3) / PEAK_INT8_MATRIX_OPS}
        if peaks:
            roofline["matrix_cores"]["peak_measured"] = peaks["int8_matrix_ops_per_s"] / 1e12
    return roofline


def serving_refinement(fpm, torch, ix, qb, qo, nq, qbytes, metric, k, entry):
    """With several batches in flight the best slab shifts (the match kernel
    shares the GPU with the other batches' small kernels): time the autotuned
    tiles with 2 or 3 batches in flight and the slab or twice the slab, and
    keep the fastest.  The persistent kernel keeps its full-GPU size, so one
    launch still spans the whole GPU and its duration stays a measure of the
    kernel.  Returns (entry, batches in flight)."""
    best = None
    for inflight in (2, 3):
        for slab in sorted({entry["slab"], min(2 * entry["slab"], 1 << 22)}):
            e = dict(entry, slab=slab)
            plans = [fpm.fpm_plan_create(ix, nq, qbytes, metric, k, fpm.options(**e)) for _ in range(inflight)]
            ms, _, _ = time_plans(fpm, torch, plans, qb, qo, nq, 100, 2)
            del plans
            if best is None or ms < best[0]:
                best = (ms, e, inflight)
    log(f"serving refinement: {best[2]} in flight, slab {best[1]['slab']}, {best[0]:.3f} ms/step")
    return best[1], best[2]


def tuned_options(fpm, torch, key, ix, qb, qo, nq, qbytes, retune: bool, metric: str, k: int, bound: str = "fd"):
    """Autotuner result for `key`, from the tuning table when present (so a
    profiled run dispatches the match kernel with one configuration only),
    else measured now and stored: fpm_autotune's tiles, then the serving
    refinement (batches in flight, persistent waves, slab).  Returns
    (options, batches in flight, tuned now)."""
    table = {}
    if os.path.exists(TUNING_FILE):
        table = json.load(open(TUNING_FILE))
    if key in table and not retune:
        entry = dict(table[key])
        inflight = entry.pop("inflight", 2)
        return fpm.options(**entry), inflight, False
    t = time.perf_counter()
    best, rows = fpm.fpm_autotune(ix, qb.data_ptr(), qo.data_ptr(), nq, qbytes, metric, k, 2,
                                  base=fpm.options(bound=bound))
    log(f"autotune {len(rows)} configs in {time.perf_counter() - t:.1f} s; fastest (qt, slab, order, tail, ms): "
        f"{sorted(rows, key=lambda r: r[4])[:4]}")
    entry = {k: v for k, v in best.as_dict().items()
             if k in ("schedule", "queries_per_item", "slab", "bucket_order", "tail_split", "bound")}
    entry, inflight = serving_refinement(fpm, torch, ix, qb, qo, nq, qbytes, metric, k, entry)
    table[key] = dict(entry, inflight=inflight)
    with open(TUNING_FILE, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    return fpm.options(**entry), inflight, True


def time_plans(fpm, torch, plans, qb, qo, nq, steps, warmup):
    """Step i runs on plans[i % len(plans)].  Each plan owns a stream and its
    buffers, so with two plans consecutive steps overlap on the GPU: the
    preparation and match-list sort of one batch run beside the match kernel
    of the next (a serving loop with two batches in flight)."""
    for p in plans:
        for _ in range(warmup):
            fpm.fpm_plan_run(p, qb.data_ptr(), qo.data_ptr(), nq)
            fpm.fpm_plan_result(p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        fpm.fpm_plan_run(plans[i % len(plans)], qb.data_ptr(), qo.data_ptr(), nq)
    for p in plans:
        _, n, st = fpm.fpm_plan_result(p)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / steps, n, st


def cpu_baseline(oracle, d, q, target_s: float, metric: int, k: int):
    """The oracle (full DP on every pair, all host threads) on a bounded
    sample of the queries against the whole dictionary."""
    from paper_1711_08475_amd import datagen

    threads = oracle.host_threads()
    nq = q[1].size - 1
    nd = d[1].size - 1
    cal = min(nq, threads)
    t0 = time.perf_counter()
    oracle.match(d, datagen.take_csr(q, np.arange(cal)), metric, k, threads=threads)
    t_cal = time.perf_counter() - t0
    rounds = max(1, int(target_s / max(t_cal, 1e-3)))
    n_sample = int(min(nq, cal * rounds))
    idx = np.arange(n_sample)
    t0 = time.perf_counter()
    res = oracle.match(d, datagen.take_csr(q, idx), metric, k, threads=threads)
    el = time.perf_counter() - t0
    return {
        "value": n_sample * nd / el,
        "unit": "pairs/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {n_sample} queries x all {nd} words, "
                  f"{'full Wagner-Fischer table' if metric == oracle.LEV else 'full mismatch count'} on every pair, "
                  f"{el:.1f} s",
    }, idx, res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="english_1m_q10k")
    ap.add_argument("--variant", default="occ")
    ap.add_argument("--bits", type=int, default=16)
    ap.add_argument("--metric", default="lev", choices=["lev", "ham"])
    ap.add_argument("-k", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--modes", default="plain,brute,asym,learned",
                    help="forms to time, from plain, batched, brute, asym, learned; the last one named is the "
                         "headline")
    ap.add_argument("--train", action="store_true", help="train the learned grouping in this process")
    ap.add_argument("--no-autotune", action="store_true", help="default tiles for the batched form")
    ap.add_argument("--retune", action="store_true", help="run the autotuner even when the table has an entry")
    ap.add_argument("--inflight", type=int, default=0,
                    help="batches in flight for the device-scheduled forms (one plan and stream each; default: the "
                         "tuning table's choice for tuned forms, else 2); the plain form reads its work list on the "
                         "host every step and always runs one")
    ap.add_argument("--filter-unit", default="auto", choices=["auto", "valu", "matrix"],
                    help="where the filter test runs: auto (matrix cores for 16-bit occurrence, "
                         "occurrence-halved and bigram keys under the paper's rule, else vector ALUs), valu, "
                         "matrix (also 32-bit and 16-bit count keys)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (one process drives one "
              f"MI355X; sharding the query batch across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    import oracle
    from paper_1711_08475_amd import datagen, fpm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    fpm.lib()
    t = time.perf_counter()
    d, q = datagen.workload(args.workload)
    nd, nq = d[1].size - 1, q[1].size - 1
    log(f"workload {args.workload}: {nd} words, {nq} queries ({time.perf_counter() - t:.1f} s)")
    t = time.perf_counter()
    ix = fpm.fpm_build_fingerprints(d, args.variant, args.bits, "common")
    torch.cuda.synchronize()
    log(f"index built in {time.perf_counter() - t:.2f} s")
    qb = torch.from_numpy(q[0].copy()).cuda()
    qo = torch.from_numpy(q[1].view(np.int64).copy()).cuda()
    torch.cuda.synchronize()  # the plans run on their own streams
    qbytes = int(q[1][-1])

    if args.copy_mib:
        src = torch.ones(args.copy_mib << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_mib} MiB read + {args.copy_mib} MiB written")
        del src, dst

    modes = args.modes.split(",")
    results = {}
    hits = {}
    learned_meta = None
    indexes = {"paper": ix}
    if "learned" in modes or "asym" in modes:
        from paper_1711_08475_amd import learn

        name = f"{args.workload}_{args.variant}{args.bits}_k{args.k}"
        mp, learned_meta = learn.load_map(name)
        if mp is None or args.train:
            t = time.perf_counter()
            mp, rep = learn.learn_grouping(d, datagen.training_queries(args.workload), bits=args.bits, k=args.k)
            learned_meta = {"training": rep, "chosen": "learned (trained in this run)"}
            log(f"trained grouping in {time.perf_counter() - t:.1f} s")
        indexes["learned"] = fpm.fpm_build_fingerprints(d, args.variant, args.bits, custom_map=mp)
    for mode in modes:
        tuned_inflight = 2
        if mode == "plain":
            opts = fpm.options(schedule=fpm.FPM_SCHED_PLAIN, time_kernel=1)
        elif mode == "brute":
            opts = fpm.options(schedule=fpm.FPM_SCHED_BRUTE, time_kernel=1)
        elif mode in ("batched", "learned", "asym"):
            mix = indexes["paper" if mode == "batched" else "learned"]
            bound = "asym" if mode == "asym" else "fd"
            if args.no_autotune:
                opts = fpm.options(schedule=fpm.FPM_SCHED_BATCHED, time_kernel=1, bound=bound)
            else:
                key = (f"{args.workload}|{args.variant}{args.bits}|{args.metric}{args.k}|"
                       f"{'common' if mode == 'batched' else 'learned'}" + ("|asym" if mode == "asym" else ""))
                opts, tuned_inflight, fresh = tuned_options(fpm, torch, key, mix, qb, qo, nq, qbytes, args.retune,
                                                            args.metric, args.k, bound)
                log(f"{mode} tiles ({'autotuned now' if fresh else 'tuning table'}): {opts.as_dict()}, "
                    f"{tuned_inflight} in flight")
                opts.time_kernel = 1
        else:
            raise SystemExit(f"unknown mode {mode}")
        if not (args.filter_unit == "matrix" and mode in ("asym", "brute")):
            opts.filter_unit = fpm.UNITS[args.filter_unit]
        inflight = 1 if mode == "plain" else (args.inflight if args.inflight > 0 else tuned_inflight)
        plans = [fpm.fpm_plan_create(indexes["paper" if mode in ("plain", "brute", "batched") else "learned"], nq,
                                     qbytes, args.metric, args.k, opts) for _ in range(inflight)]
        ms, n, st = time_plans(fpm, torch, plans, qb, qo, nq, args.steps, args.warmup)
        per_plan = (args.steps + inflight - 1) // inflight
        kms = np.concatenate([fpm.fpm_plan_kernel_ms(p, per_plan) for p in plans])
        results[mode] = {
            "ms_per_step": ms,
            "pairs_per_s": nq * nd / (ms * 1e-3),
            "kernel_ms": float(np.mean(kms)) if kms.size else None,
            "stats": st,
            "options": opts.as_dict(),
            "inflight": inflight,
        }
        hits[mode] = fpm.fpm_plan_copy_matches(plans[0])
        for p in plans[1:]:
            if not np.array_equal(fpm.fpm_plan_copy_matches(p), hits[mode]):
                raise SystemExit(f"{mode}: plans in flight returned different match lists")
        log(f"{mode}: {ms:.3f} ms/step ({inflight} in flight), kernel {results[mode]['kernel_ms']:.3f} ms, "
            f"{results[mode]['pairs_per_s']:.3e} pairs/s, survivors {st['survivors']}, matches {n}")
        del plans

    # the forms must agree exactly
    names = list(hits)
    agree = all(np.array_equal(hits[names[0]], hits[m]) for m in names[1:])

    head = names[-1]
    r = results[head]
    st = r["stats"]
    traffic = load_traffic(head, args.workload)
    try:  # the device's own peak rates, reported beside the published ones
        peaks = fpm.fpm_measure_peaks()
        log(f"measured peaks: int VALU {peaks['int_valu_ops_per_s'] / 1e12:.2f} Tops/s, "
            f"int8 matrix {peaks['int8_matrix_ops_per_s'] / 1e12:.0f} Tops/s")
    except fpm.FpmError as e:  # auxiliary: the bench line does not depend on it
        peaks = None
        log(f"peak probes failed: {e}")
    roofline = roofline_of(st, r["kernel_ms"], args.variant, args.bits, traffic, peaks)

    cpu = None
    sampled_parity = None
    if not args.no_cpu_baseline:
        cpu, idx, ref = cpu_baseline(oracle, d, q, args.cpu_seconds, oracle.LEV if args.metric == "lev" else oracle.HAM,
                                     args.k)
        g = hits[head]
        g = g[np.isin(g[:, 0], idx)]
        sampled_parity = bool(np.array_equal(g, ref))
        log(f"cpu baseline {cpu['value']:.3e} pairs/s on {cpu['cores']} threads; sampled parity {sampled_parity}")

    out = {
        "metric": metric_name(args.metric, args.k),
        "value": r["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {WORKLOAD_TEXT.get(args.workload, args.workload)}, "
                        f"{'Levenshtein' if args.metric == 'lev' else 'Hamming'} k={args.k}",
            "fingerprint": f"{args.variant}{args.bits}",
            "form": head,
            "symbols": "learned grouping" if head in ("learned", "asym") else "common (paper map)",
            "filter_rule": "asymmetric bound" if head == "asym" else "F_D <= 2k (Eq. 1)",
            "batches_in_flight": r["inflight"],
            "options": r["options"],
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "forms": {m: {"pairs_per_s": v["pairs_per_s"], "ms_per_step": v["ms_per_step"], "in_flight": v["inflight"],
                      "kernel_ms": v["kernel_ms"], "examined": v["stats"]["pairs_examined"],
                      "survivors": v["stats"]["survivors"], "matches": v["stats"]["matches"]}
                  for m, v in results.items()},
        "rejection_rate": 1.0 - st["survivors"] / max(st["pairs_examined"], 1),
        "speedup_vs_brute": (results["brute"]["ms_per_step"] / r["ms_per_step"]) if "brute" in results else None,
        "speedup_vs_plain": (results["plain"]["ms_per_step"] / r["ms_per_step"]) if "plain" in results else None,
        "learned_map": ({"chosen": learned_meta.get("chosen"), "evaluation": learned_meta.get("evaluation"),
                         "train_ms": learned_meta.get("training", {}).get("ms")} if learned_meta else None),
        "forms_agree": agree,
        "sampled_oracle_parity": sampled_parity,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
