#!/usr/bin/env python3
"""Levenshtein k=1 query-word pairs per second on one MI355X.

Workload (default): the batched uneven workload -- 2,000,000 dictionary
strings (1,000,000 English-like words of lengths 2-20 and 1,000,000 URL-like
strings of lengths 20-120, shuffled) against 65,536 mixed queries (30% are
dictionary strings with one random edit), 32-bit occurrence fingerprints,
Levenshtein k = 1.  One step is one full match of the query batch with
inputs resident in HBM: query fingerprints, length bucketing, work list, the
fused filter + verify kernel and the sorted match list.

Forms timed on the same GPU (all return the same match list):
  plain        paper's common-symbol map, host-built work list, one wave per
               work item, default tiles, no graph;
  brute        no fingerprints: every length-compatible pair is verified (the
               paper's naive comparison, giving its speedup S = T_n / T_f);
  batched      paper's map, persistent kernel over a device-built work list,
               one captured hipGraph per step, tiles from the autotuner;
  learned      the batched form with the symbol grouping learned by the MLP
               (paper_1711_08475_amd/maps/<workload>_occ<bits>_k1.json, written
               by `python -m paper_1711_08475_amd.learn`; --train retrains it);
  learned_matrix  the learned form with the filter test on the matrix cores
               (an opt-in addition of this library; same survivors and matches);
  asym         (on request) the learned form under the asymmetric bound, a
               filter rule beyond the paper.
The headline is the last form named (default: learned, the paper's rule on
the vector ALUs).

Device-scheduled forms keep several batches in flight (the number is stored
with the tiles in the tuning table; --inflight overrides): that many plans,
each with its own stream and buffers, take steps in turn, so one batch's
preparation and match-list sort overlap another batch's match kernel.  Every
step is still the whole pipeline over one batch.  A graph form is timed
twice over the same number of steps: once as one captured graph per step
(`ms_per_step`, `value`), once with the graph split around an event-bracketed
launch of the match kernel (`kernel_ms`, the roofline's duration).

A secondary block times the 1,000,000 English-like words x 10,000 queries
workload with 16-bit occurrence fingerprints (plain, and the learned form on
the vector ALUs and, as an opt-in addition, on the matrix cores).

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
    "mixed_2m_q64k": "2,000,000 mixed English-like/URL-like strings x 65,536 mixed queries (lengths 2-120)",
}


def metric_name(metric: str, k: int) -> str:
    return f"{'Lev' if metric == 'lev' else 'Ham'} k={k} query-word pairs/sec (1 MI355X), learned+batched vs plain filter"


PEAK_INT_OPS = 256 * 64 * 2.4e9  # CUs x lanes x clock: one 32-bit VALU op per lane per clock
PEAK_INT8_MATRIX_OPS = 5.0e15  # MI355X dense int8 matrix-core peak (ops/s)
PEAK_HBM = 8.0e12  # bytes/s
MATRIX_INT8_OPS_PER_PAIR = 64  # v_mfma_i32_32x32x32_i8: 2 x 32 ops per output
FPM_UNIT_MATRIX = 2


def filter_ops(variant: str, bits: int) -> int:
    """Algorithmic integer ops of the filter test per examined pair (Eq. 1),
    whichever unit runs it: XOR, popcount and threshold compare for keys
    whose F_D is the popcount of their XOR (occurrence, occurrence-halved,
    bigram, 16-bit count as a 24-bit thermometer code); the 32-bit count
    thermometer spans two words (5); position fingerprints gather the fields
    of the XOR first (9); combined keys test two words (6)."""
    if variant == "count":
        return 3 if bits == 16 else 5
    return {"occ": 3, "occh": 3, "qgram": 3, "pos": 9, "combo": 6}[variant]


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "match_kernel_traffic.json")
TUNING_FILE = os.path.join(ROOT, "paper_1711_08475_amd", "tuned.json")
MATCH_SRC = os.path.join(ROOT, "paper_1711_08475_amd", "csrc", "fpm_match.hip")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    return hashlib.sha256(open(MATCH_SRC, "rb").read()).hexdigest()


def load_counters(form: str, workload: str):
    """Counter summary of the match kernel (HBM bytes per launch, VALU issue)
    from the committed rocprofv3 runs of this form and workload, only while
    the kernel source is unchanged since they were taken."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash():
        return None
    if t.get("form") != form or t.get("workload_name") != workload:
        return None
    return t


def roofline_of(st: dict, kernel_ms, variant: str, bits: int, counters, peaks=None, hbm_bytes=None) -> dict:
    """Roofline of the match kernel.  Algorithmic work per launch = filter
    ops per examined pair x examined pairs + band cells (2k+1) min(m, n) of
    the survivors, over the kernel's measured duration, against the
    published int-VALU peak -- whichever unit ran the filter test.  When
    popcount pruning skipped pairs (which fail the filter without a test),
    the same pricing over the pairs the filter tested is reported beside it
    as `frac_tested`.  Issued VALU utilisation (from the committed counters)
    and, when the matrix cores ran the filter, their int8 fraction are
    reported under their own names.  `peaks` (fpm_measure_peaks) adds the
    peaks measured on this device; `hbm_bytes` the kernel's algorithmic HBM
    bytes."""
    matrix = st.get("filter_unit") == FPM_UNIT_MATRIX
    per_pair = filter_ops(variant, bits)
    tested = st.get("pairs_filtered") or st["pairs_examined"]
    ops = per_pair * st["pairs_examined"] + st["verify_cells"]
    achieved = ops / (kernel_ms * 1e-3) if kernel_ms else None
    roofline = {
        "bound": "alu",
        "achieved": achieved / 1e12 if achieved else None,
        "peak": PEAK_INT_OPS / 1e12,
        "unit": "Tops/s",
        "frac": achieved / PEAK_INT_OPS if achieved else None,
        "traffic": counters["bytes_per_launch"] if counters else None,
        "kernel": "k_match (fused filter + LDS queue + verify)",
        "filter_unit": "matrix" if matrix else "valu",
        "filter_ops_per_pair": per_pair,
        "pairs_examined": st["pairs_examined"],
        "pairs_tested": tested,
        "ops_per_launch": ops,
        "kernel_ms": kernel_ms,
    }
    if tested < st["pairs_examined"] and kernel_ms:
        roofline["frac_tested"] = (per_pair * tested + st["verify_cells"]) / (kernel_ms * 1e-3) / PEAK_INT_OPS
    if peaks:
        roofline["peak_measured"] = peaks["int_valu_ops_per_s"] / 1e12
    if counters and counters.get("valu_insts_per_launch") and kernel_ms:
        # wave64 VALU instructions issued, one per SIMD per 4 clocks at most
        slots = 256 * 4 * 2.4e9 / 4 * kernel_ms * 1e-3
        roofline["valu_issue"] = {"insts_per_launch": counters["valu_insts_per_launch"],
                                  "utilisation": counters["valu_insts_per_launch"] / slots}
    if hbm_bytes and kernel_ms:
        roofline["hbm"] = {"algorithmic_bytes": hbm_bytes, "achieved_GBps": hbm_bytes / (kernel_ms * 1e-3) / 1e9,
                           "frac": hbm_bytes / (kernel_ms * 1e-3) / PEAK_HBM}
    if matrix and kernel_ms:
        m_ops = MATRIX_INT8_OPS_PER_PAIR * st["pairs_examined"]
        roofline["matrix_cores"] = {"achieved": m_ops / (kernel_ms * 1e-3) / 1e12,
                                    "peak": PEAK_INT8_MATRIX_OPS / 1e12, "unit": "int8 Tops/s",
                                    "frac": m_ops / (kernel_ms * 1e-3) / PEAK_INT8_MATRIX_OPS}
        if peaks:
            roofline["matrix_cores"]["peak_measured"] = peaks["int8_matrix_ops_per_s"] / 1e12
    return roofline


def match_kernel_bytes(d, q, bits: int, matches: int) -> int:
    """Compulsory HBM bytes of one match launch: dictionary keys and strings,
    query keys and strings (each read once), 8-byte match keys written."""
    nd, nq = d[1].size - 1, q[1].size - 1
    kb = 8 if bits > 32 else 4
    return int(nd * kb + int(d[1][-1]) + nq * kb + int(q[1][-1]) + 8 * matches)


def serving_refinement(fpm, torch, ix, qb, qo, nq, qbytes, metric, k, entry):
    """With several batches in flight the best slab shifts (the match kernel
    shares the GPU with the other batches' small kernels): time the autotuned
    tiles with 1, 2 or 3 batches in flight and the slab or twice the slab,
    and keep the fastest (one batch in flight unless more are at least 1%
    faster: the match kernel then runs alone and its timed duration is its
    own).  Returns (entry, batches in flight, ms per step)."""
    best = None
    for inflight in (1, 2, 3):
        for slab in sorted({entry["slab"], min(2 * entry["slab"], 1 << 22)}):
            e = dict(entry, slab=slab)
            plans = [fpm.fpm_plan_create(ix, nq, qbytes, metric, k, fpm.options(**e)) for _ in range(inflight)]
            ms, _, _ = time_plans(fpm, torch, plans, qb, qo, nq, 100, 2)
            del plans
            if best is None or ms < best[0] * (0.99 if inflight > best[2] else 1.0):
                best = (ms, e, inflight)
    log(f"serving refinement: {best[2]} in flight, slab {best[1]['slab']}, {best[0]:.3f} ms/step")
    return best[1], best[2], best[0]


def tuned_options(fpm, torch, key, ix, qb, qo, nq, qbytes, retune: bool, metric: str, k: int, bound: str = "fd",
                  unit: str = "auto"):
    """Autotuner result for `key`, from the tuning table when present (so a
    profiled run dispatches the match kernel with one configuration only),
    else measured now and stored.  Returns (options, batches in flight,
    tuned now)."""
    table = {}
    if os.path.exists(TUNING_FILE):
        table = json.load(open(TUNING_FILE))
    if key in table and not retune:
        entry = dict(table[key])
        inflight = entry.pop("inflight", 2)
        return fpm.options(**entry), inflight, False
    # popcount pruning is tried where it applies (the paper's rule on the
    # vector ALUs); the faster of the two refined configurations is kept
    prunes = (0, 1) if bound == "fd" and unit != "matrix" and key.split("|")[1][:-2] in (
        "occ", "occh", "count", "qgram") else (0,)
    chosen = None
    for prune in prunes:
        t = time.perf_counter()
        best, rows = fpm.fpm_autotune(ix, qb.data_ptr(), qo.data_ptr(), nq, qbytes, metric, k, 2,
                                      base=fpm.options(bound=bound, filter_unit=unit, pop_prune=prune))
        log(f"autotune (pop_prune {prune}) {len(rows)} configs in {time.perf_counter() - t:.1f} s; fastest "
            f"(qt, slab, order, tail, ms): {sorted(rows, key=lambda r: r[4])[:4]}")
        entry = {k: v for k, v in best.as_dict().items()
                 if k in ("schedule", "queries_per_item", "slab", "bucket_order", "tail_split", "bound", "pop_prune")}
        entry, inflight, ms = serving_refinement(fpm, torch, ix, qb, qo, nq, qbytes, metric, k,
                                                 dict(entry, filter_unit=fpm.UNITS[unit]))
        if chosen is None or ms < chosen[2]:
            chosen = (entry, inflight, ms)
    entry, inflight, _ = chosen
    entry.pop("filter_unit", None)
    if not entry.get("pop_prune"):
        entry.pop("pop_prune", None)
    table[key] = dict(entry, inflight=inflight)
    with open(TUNING_FILE, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    return fpm.options(**entry), inflight, True


def time_plans(fpm, torch, plans, qb, qo, nq, steps, warmup):
    """Step i runs on plans[i % len(plans)].  Each plan owns a stream and its
    buffers, so with two plans consecutive steps overlap on the GPU.
    Returns (mean ms per step, matches of the last run, its stats)."""
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


def host_cpu():
    """CPU model and clock from /proc/cpuinfo."""
    model, mhz = None, []
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name") and model is None:
                model = line.split(":", 1)[1].strip()
            elif line.startswith("cpu MHz"):
                mhz.append(float(line.split(":", 1)[1]))
    except OSError:
        pass
    return {"cpu_model": model, "cpu_mhz_max_reported": max(mhz) if mhz else None}


def cpu_baseline(oracle, d, q, target_s: float, metric: int, k: int):
    """The oracle (full DP on every pair) on bounded samples: all host
    threads over the first queries against the whole dictionary, and one
    thread over the first query against a prefix of the dictionary (the
    paper's protocol is single-threaded)."""
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
    # single thread: the calibration queries against a dictionary prefix
    # sized to about a third of the target time
    q1 = datagen.take_csr(q, np.arange(cal))
    n_pre = min(nd, 2_000)
    t0 = time.perf_counter()
    oracle.match(datagen.take_csr(d, np.arange(n_pre)), q1, metric, k, threads=1)
    t_pre = time.perf_counter() - t0
    n_words1 = int(min(nd, max(n_pre, n_pre * (target_s / 3) / max(t_pre, 1e-3))))
    t0 = time.perf_counter()
    oracle.match(datagen.take_csr(d, np.arange(n_words1)), q1, metric, k, threads=1)
    el1 = time.perf_counter() - t0
    kind = "full Wagner-Fischer table" if metric == oracle.LEV else "full mismatch count"
    return {
        "value": n_sample * nd / el,
        "unit": "pairs/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {n_sample} queries x all {nd} words, {kind} on every pair, {el:.1f} s on {threads} threads",
        "single_thread": {"value": cal * n_words1 / el1, "unit": "pairs/s",
                          "sample": f"first {cal} queries x first {n_words1} words, {kind}, {el1:.1f} s on one thread"},
        **host_cpu(),
    }, idx, res


def time_form(fpm, torch, mode, ix, qb, qo, nq, qbytes, args, opts, inflight):
    """Times one form.  Returns its result dict and the match list."""
    graph = mode in ("batched", "learned", "asym")
    entry = opts.as_dict()
    res = {"inflight": inflight, "options": entry}
    if graph:
        # one captured graph per step: the step time
        plans = [fpm.fpm_plan_create(ix, nq, qbytes, args.metric, args.k, fpm.options(**dict(entry, time_kernel=0)))
                 for _ in range(inflight)]
        ms, n, st = time_plans(fpm, torch, plans, qb, qo, nq, args.steps, args.warmup)
        hits = fpm.fpm_plan_copy_matches(plans[0])
        for p in plans[1:]:
            if not np.array_equal(fpm.fpm_plan_copy_matches(p), hits):
                raise SystemExit(f"{mode}: plans in flight returned different match lists")
        del plans
        res["ms_per_step"] = ms
    # the match kernel bracketed by HIP events on the plans' streams (a graph
    # form is split into prep graph + kernel + post graph for this)
    plans = [fpm.fpm_plan_create(ix, nq, qbytes, args.metric, args.k, fpm.options(**dict(entry, time_kernel=1)))
             for _ in range(inflight)]
    ms_t, n, st = time_plans(fpm, torch, plans, qb, qo, nq, args.steps, args.warmup)
    per_plan = (args.steps + inflight - 1) // inflight
    kms = np.concatenate([fpm.fpm_plan_kernel_ms(p, per_plan) for p in plans])
    h = fpm.fpm_plan_copy_matches(plans[0])
    for p in plans[1:]:
        if not np.array_equal(fpm.fpm_plan_copy_matches(p), h):
            raise SystemExit(f"{mode}: plans in flight returned different match lists")
    if graph and not np.array_equal(h, hits):
        raise SystemExit(f"{mode}: split and whole graphs returned different match lists")
    hits = h
    del plans
    if graph and inflight > 1:
        # the same kernel with one batch in flight: its duration without
        # the other batches' kernels beside it
        plan = fpm.fpm_plan_create(ix, nq, qbytes, args.metric, args.k, fpm.options(**dict(entry, time_kernel=1)))
        ms_a, _, _ = time_plans(fpm, torch, [plan], qb, qo, nq, args.steps, args.warmup)
        ka = fpm.fpm_plan_kernel_ms(plan, args.steps)
        if not np.array_equal(fpm.fpm_plan_copy_matches(plan), hits):
            raise SystemExit(f"{mode}: one batch in flight returned a different match list")
        del plan
        res["alone"] = {"ms_per_step": ms_a, "kernel_ms": float(np.mean(ka)) if ka.size else None}
    if graph:
        res["ms_per_step_kernel_timed"] = ms_t
    else:
        res["ms_per_step"] = ms_t
    res["kernel_ms"] = float(np.mean(kms)) if kms.size else None
    res["kernel_ms_median"] = float(np.median(kms)) if kms.size else None
    res["stats"] = st
    res["pairs_per_s"] = nq * (ix.n_words) / (res["ms_per_step"] * 1e-3)
    return res, hits


def learned_index(fpm, d, args, workload, variant, bits, k):
    from paper_1711_08475_amd import datagen, learn

    name = f"{workload}_{variant}{bits}_k{k}"
    mp, meta = learn.load_map(name)
    if mp is None or args.train:
        t = time.perf_counter()
        mp, rep = learn.learn_grouping(d, datagen.training_queries(workload), bits=bits, k=k)
        meta = {"training": rep, "chosen": "learned (trained in this run)"}
        log(f"trained grouping in {time.perf_counter() - t:.1f} s")
    return fpm.fpm_build_fingerprints(d, variant, bits, custom_map=mp), meta


def form_options(fpm, torch, mode, args, workload, variant, bits, ix, qb, qo, nq, qbytes, unit="auto"):
    if mode == "plain":
        return fpm.options(schedule=fpm.FPM_SCHED_PLAIN, filter_unit=unit), 1, "plain"
    if mode == "brute":
        return fpm.options(schedule=fpm.FPM_SCHED_BRUTE), (args.inflight or 2), "brute"
    bound = "asym" if mode == "asym" else "fd"
    if args.no_autotune:
        return fpm.options(schedule=fpm.FPM_SCHED_BATCHED, bound=bound, filter_unit=unit), (args.inflight or 2), \
            "default tiles"
    key = (f"{workload}|{variant}{bits}|{args.metric}{args.k}|{'common' if mode == 'batched' else 'learned'}"
           + ("|asym" if mode == "asym" else "") + ("|matrix" if unit == "matrix" else ""))
    opts, tuned_inflight, fresh = tuned_options(fpm, torch, key, ix, qb, qo, nq, qbytes, args.retune, args.metric,
                                                args.k, bound, unit)
    opts.filter_unit = fpm.UNITS[unit]
    return opts, (args.inflight or tuned_inflight), ("autotuned now" if fresh else "tuning table")


def run_block(fpm, torch, args, workload, variant, bits, modes, unit="auto", extra=None):
    """Times `modes` on one workload; returns (results, match lists, context)."""
    from paper_1711_08475_amd import datagen

    t = time.perf_counter()
    d, q = datagen.workload(workload)
    nd, nq = d[1].size - 1, q[1].size - 1
    log(f"workload {workload}: {nd} words, {nq} queries ({time.perf_counter() - t:.1f} s)")
    # index build, three times: its device time is the fingerprint
    # construction throughput (the analogue of the paper's Table 4)
    builds = []
    for _ in range(3):
        t = time.perf_counter()
        ix = fpm.fpm_build_fingerprints(d, variant, bits, "common")
        builds.append((time.perf_counter() - t,) + fpm.fpm_index_build_ms(ix))
    build_ms = float(np.median([b[1] for b in builds]))
    layout_ms = float(np.median([b[2] for b in builds]))
    dict_bytes = int(d[1][-1])
    fp_bytes = 4 if bits <= 16 or variant != "count" else 8
    alg = dict_bytes + 8 * (nd + 1) + 4 * nd + nd * fp_bytes
    fp_build = {"dictionary_bytes": dict_bytes, "words": nd, "device_ms": build_ms, "layout_fp_ms": layout_ms,
                "MB_per_s": dict_bytes / 1e6 / (build_ms * 1e-3),
                "algorithmic_bytes": alg, "hbm_frac": alg / (build_ms * 1e-3) / PEAK_HBM,
                "host_s_with_upload": float(np.median([b[0] for b in builds]))}
    log(f"index built: device {build_ms:.3f} ms ({fp_build['MB_per_s']:.0f} MB/s of dictionary text; "
        f"length sort + layout + fingerprints {layout_ms:.3f} ms)")
    qb = torch.from_numpy(q[0].copy()).cuda()
    qo = torch.from_numpy(q[1].view(np.int64).copy()).cuda()
    torch.cuda.synchronize()  # the plans run on their own streams
    qbytes = int(q[1][-1])
    indexes = {"paper": ix}
    meta = None
    if any(m.replace("_matrix", "") in ("learned", "asym") for m in modes):
        indexes["learned"], meta = learned_index(fpm, d, args, workload, variant, bits, args.k)
    results, hits = {}, {}
    for mode in modes:
        name, u = (mode[:-len("_matrix")], "matrix") if mode.endswith("_matrix") else (mode, unit)
        mix = indexes["learned" if name in ("learned", "asym") else "paper"]
        opts, inflight, src = form_options(fpm, torch, name, args, workload, variant, bits, mix, qb, qo, nq, qbytes,
                                           u)
        if name in ("batched", "learned", "asym"):
            log(f"{mode} tiles ({src}): {opts.as_dict()}, {inflight} in flight")
        r, h = time_form(fpm, torch, name, mix, qb, qo, nq, qbytes, args, opts, inflight)
        r["index"], r["opts"] = mix, opts
        results[mode], hits[mode] = r, h
        st = r["stats"]
        log(f"{mode}: {r['ms_per_step']:.3f} ms/step ({inflight} in flight), kernel {r['kernel_ms']:.3f} ms, "
            f"{r['pairs_per_s']:.3e} pairs/s, survivors {st['survivors']}, matches {h.shape[0]}, "
            f"filter unit {st['filter_unit']}, pairs tested {st['pairs_filtered']} of {st['pairs_examined']}")
    return results, hits, {"d": d, "q": q, "fp_build": fp_build, "learned_meta": meta}


def host_end_to_end(fpm, ix, q, opts, metric, k, ref, calls=5):
    """The host-buffer entry point (fpm_match) timed on the host clock, one
    warm-up and `calls` timed calls: query upload over PCIe, a temporary
    plan (its allocations, and a rerun when the default match buffer has to
    grow), the device pipeline, and the match list's download as (query,
    word, dist) rows.  Reported beside the device-resident value, never as
    it."""
    opts = fpm.options(**dict(opts.as_dict(), time_kernel=0))
    fpm.fpm_match(ix, q, metric, k, opts)
    ts = []
    got = None
    for _ in range(calls):
        t0 = time.perf_counter()
        got = fpm.fpm_match(ix, q, metric, k, opts)
        ts.append(time.perf_counter() - t0)
    if not np.array_equal(got, ref):
        raise SystemExit("host entry point returned a different match list")
    ms = 1e3 * float(np.median(ts))
    nq = q[1].size - 1
    return {"ms_median": ms, "pairs_per_s": nq * ix.n_words / (ms * 1e-3), "calls": calls,
            "query_bytes_up": int(q[1][-1]) + 8 * (nq + 1), "result_bytes_down": 12 * int(got.shape[0]),
            "includes": "query upload, temporary plan (allocations, buffer growth), device pipeline, "
                        "match-list download"}


def forms_summary(results):
    return {m: {"pairs_per_s": v["pairs_per_s"], "ms_per_step": v["ms_per_step"], "one_in_flight": v.get("alone"),
                "ms_per_step_kernel_timed": v.get("ms_per_step_kernel_timed"), "in_flight": v["inflight"],
                "kernel_ms": v["kernel_ms"], "kernel_ms_median": v["kernel_ms_median"],
                "examined": v["stats"]["pairs_examined"], "tested": v["stats"]["pairs_filtered"],
                "survivors": v["stats"]["survivors"], "matches": v["stats"]["matches"],
                "filter_unit": {0: "none", 1: "valu", 2: "matrix"}[v["stats"]["filter_unit"]]}
            for m, v in results.items()}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="mixed_2m_q64k")
    ap.add_argument("--variant", default="occ")
    ap.add_argument("--bits", type=int, default=32)
    ap.add_argument("--metric", default="lev", choices=["lev", "ham"])
    ap.add_argument("-k", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--modes", default="plain,brute,batched,learned_matrix,learned",
                    help="forms to time, from plain, batched, brute, asym, learned (and learned_matrix: the "
                         "learned form with the filter on the matrix cores); the last one named is the headline")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary block (english_1m_q10k, occ16, Lev k=1)")
    ap.add_argument("--train", action="store_true", help="train the learned grouping in this process")
    ap.add_argument("--no-autotune", action="store_true", help="default tiles for the batched form")
    ap.add_argument("--retune", action="store_true", help="run the autotuner even when the table has an entry")
    ap.add_argument("--inflight", type=int, default=0,
                    help="batches in flight for the device-scheduled forms (default: the tuning table's choice "
                         "for tuned forms, else 2); the plain form always runs one")
    ap.add_argument("--filter-unit", default="auto", choices=["auto", "valu", "matrix"],
                    help="where the filter test runs (auto = vector ALUs; matrix: the opt-in matrix-core filter)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (one process drives one "
              f"MI355X; sharding the query batch across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    import oracle
    from paper_1711_08475_amd import fpm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    fpm.lib()
    if args.copy_mib:
        src = torch.ones(args.copy_mib << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_mib} MiB read + {args.copy_mib} MiB written")
        del src, dst

    modes = args.modes.split(",")
    results, hits, ctx = run_block(fpm, torch, args, args.workload, args.variant, args.bits, modes,
                                   args.filter_unit)
    d, q = ctx["d"], ctx["q"]
    names = list(hits)
    agree = all(np.array_equal(hits[names[0]], hits[m]) for m in names[1:])
    head = names[-1]
    r = results[head]
    st = r["stats"]
    counters = load_counters(head, args.workload)
    try:  # the device's own peak rates, reported beside the published ones
        peaks = fpm.fpm_measure_peaks()
        log(f"measured peaks: int VALU {peaks['int_valu_ops_per_s'] / 1e12:.2f} Tops/s, "
            f"int8 matrix {peaks['int8_matrix_ops_per_s'] / 1e12:.0f} Tops/s")
    except fpm.FpmError as e:  # auxiliary: the bench line does not depend on it
        peaks = None
        log(f"peak probes failed: {e}")
    roofline = roofline_of(st, r["kernel_ms"], args.variant, args.bits, counters, peaks,
                           match_kernel_bytes(d, q, args.bits, int(st["matches"])))
    # with several batches in flight one launch shares the GPU with its
    # neighbours' kernels, so its duration is not its own: the same work
    # priced by the step time, and by the kernel's duration with one batch
    # in flight
    roofline["frac_step"] = roofline["ops_per_launch"] / (r["ms_per_step"] * 1e-3) / PEAK_INT_OPS
    if r.get("alone") and r["alone"]["kernel_ms"]:
        roofline["one_in_flight"] = {
            "kernel_ms": r["alone"]["kernel_ms"], "ms_per_step": r["alone"]["ms_per_step"],
            "frac": roofline["ops_per_launch"] / (r["alone"]["kernel_ms"] * 1e-3) / PEAK_INT_OPS}

    e2e = host_end_to_end(fpm, r["index"], q, r["opts"], args.metric, args.k, hits[head])
    log(f"host entry point (PCIe included): {e2e['ms_median']:.2f} ms per call, {e2e['pairs_per_s']:.3e} pairs/s")

    cpu = None
    sampled_parity = None
    if not args.no_cpu_baseline:
        cpu, idx, ref = cpu_baseline(oracle, d, q, args.cpu_seconds,
                                     oracle.LEV if args.metric == "lev" else oracle.HAM, args.k)
        g = hits[head]
        g = g[np.isin(g[:, 0], idx)]
        sampled_parity = bool(np.array_equal(g, ref))
        log(f"cpu baseline {cpu['value']:.3e} pairs/s on {cpu['cores']} threads, "
            f"{cpu['single_thread']['value']:.3e} on one; sampled parity {sampled_parity}")

    meta = ctx["learned_meta"]
    learned = None
    if meta is not None:
        learned = {"chosen": meta.get("chosen"),
                   "stored_evaluation": meta.get("evaluation"),
                   "stored_train_ms": meta.get("training", {}).get("ms")}
        paper_form = next((m for m in ("batched", "plain") if m in results), None)
        if paper_form and "learned" in results:
            ex = results["learned"]["stats"]["pairs_examined"]
            ps, ls = results[paper_form]["stats"]["survivors"], results["learned"]["stats"]["survivors"]
            learned["measured"] = {"examined": ex, "paper_survivors": ps, "learned_survivors": ls,
                                   "paper_rejection": 1 - ps / max(ex, 1), "learned_rejection": 1 - ls / max(ex, 1)}

    secondary = None
    if not args.no_secondary and args.workload != "english_1m_q10k":
        sargs = argparse.Namespace(**dict(vars(args), metric="lev", k=1, inflight=0))
        sres, shits, sctx = run_block(fpm, torch, sargs, "english_1m_q10k", "occ", 16,
                                      ["plain", "learned", "learned_matrix"], "auto")
        sn = list(shits)
        ls = sres["learned"]["stats"]
        secondary = {
            "workload": f"english_1m_q10k: {WORKLOAD_TEXT['english_1m_q10k']}, Levenshtein k=1",
            "fingerprint": "occ16",
            "forms": forms_summary(sres),
            "forms_agree": all(np.array_equal(shits[sn[0]], shits[m]) for m in sn[1:]),
            "speedup_vs_plain": sres["plain"]["ms_per_step"] / sres["learned"]["ms_per_step"],
            "roofline_learned_valu": roofline_of(ls, sres["learned"]["kernel_ms"], "occ", 16, None),
            "roofline_learned_matrix": roofline_of(sres["learned_matrix"]["stats"],
                                                   sres["learned_matrix"]["kernel_ms"], "occ", 16, None),
            "fp_build": sctx["fp_build"],
        }

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
            "timing": ("value / ms_per_step: mean over the timed steps, batches in flight, one captured graph per "
                       "step" if head in ("batched", "learned", "asym") else
                       "value / ms_per_step: mean over the timed steps") +
                      "; roofline kernel_ms: mean HIP-event duration of the match kernel over the same number of "
                      "steps, same batches in flight, with the graph split around it (roofline.frac_step prices the "
                      "kernel's work by the step time, roofline.one_in_flight by its duration with one batch in "
                      "flight)",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp_build": ctx["fp_build"],
        "host_end_to_end": e2e,
        "forms": forms_summary(results),
        "rejection_rate": 1.0 - st["survivors"] / max(st["pairs_examined"], 1),
        "speedup_vs_brute": (results["brute"]["ms_per_step"] / r["ms_per_step"]) if "brute" in results else None,
        "speedup_vs_plain": (results["plain"]["ms_per_step"] / r["ms_per_step"]) if "plain" in results else None,
        "learned_map": learned,
        "forms_agree": agree,
        "sampled_oracle_parity": sampled_parity,
        "secondary": secondary,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
