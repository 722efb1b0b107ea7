"""Benchmark: bulk build to 95% load, lookups, deletes and re-lookups on one MI355X.

Workload (one step): a FIXED-addressing table of 4,415,057 buckets x 16
slots (70,640,912 slots) is cleared, then
  insert   2^26 unique uniform keys (values = lo32(splitmix64(key)))  -> 95% load
  lookup   2^26 keys, 50% present
  delete   2^25 of the inserted keys
  lookup   the same 2^26 keys again (25% present)
= 3.5 * 2^26 = 234,881,024 operations.  Inputs sit in HBM before timing.

Prints one JSON line.  `value` is whole-step throughput in Mops/s; per-phase
rates, the roofline of the dominant kernel (the lookup kernel) and the CPU
oracle on a bounded sample are reported beside it.
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

METRIC = "Mops/s insert/lookup/mixed @95% LF vs plain launch; served p50/p99 latency"
HBM_PEAK_GBS = 8000.0
BUCKET_BYTES = 128  # 16 slots x 8 B: one line per bucket touch
N_KEYS = 1 << 26
LOAD = 0.95
S = 16


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=("suite", "bulk", "mixed", "resize", "served", "breakdown", "hashes",
                                           "gather"), default="suite",
                    help="suite (default): the bulk step as the headline, with the mixed and served "
                         "configurations as sub-records")
    ap.add_argument("--executor", choices=("plain", "persistent"), default="plain",
                    help="mixed: one launch sequence per batch, or the persistent executor")
    ap.add_argument("--no-mixed", action="store_true", help="suite: skip the mixed sub-record")
    ap.add_argument("--no-served", action="store_true", help="suite: skip the served sub-record")
    ap.add_argument("--mixed-steps", type=int, default=2, help="suite: timed passes over the mixed batches")
    ap.add_argument("--blocks-per-cu", type=int, default=-1,
                    help="persistent executor blocks per CU (0: as many as fit; -1: the autotuned value, else 1)")
    ap.add_argument("--tables", type=int, default=256, help="served: tables")
    ap.add_argument("--table-log2-max", type=float, default=24, help="served: largest table (log2 keys)")
    ap.add_argument("--requests", type=int, default=20000, help="served: requests")
    ap.add_argument("--request-log2", type=float, default=20, help="served: largest request (log2 ops)")
    ap.add_argument("--lambda-sweep", default="0.35,0.7,1.0",
                    help="served: Poisson rates as fractions of the plain-launch saturation rate")
    ap.add_argument("--validate", action="store_true",
                    help="mixed/served: also compare every output with the CPU dictionary (untimed, slow)")
    ap.add_argument("--keys-log2", type=int, default=26)
    ap.add_argument("--entry-bits", type=int, choices=(64, 32), default=64,
                    help="bulk: 64 = key/value pairs in 16-slot buckets; 32 = a key-only set of 32-bit entries in "
                         "32-slot buckets (one 128-byte line each)")
    ap.add_argument("--batches", type=int, default=64, help="mixed/resize: insert batches")
    ap.add_argument("--batch-log2", type=int, default=22, help="mixed/resize: operations per batch")
    ap.add_argument("--resize-k", type=int, default=0, help="0: the autotuned value if cached, else 1024")
    ap.add_argument("--autotune", action="store_true", help="run the autotuner first and use its picks")
    ap.add_argument("--probe-both", type=int, default=-1,
                    help="bulk: 1 = lookups/deletes probe both candidates in one round (-1: autotuned, else 0)")
    ap.add_argument("--probe-tuning", type=int, default=-1,
                    help="bulk/mixed: probe-kernel variant word (hive_config.probe_tuning; -1: autotuned, else 0)")
    ap.add_argument("--probe-grid", type=int, default=-1,
                    help="bulk/mixed: blocks per probe launch cap (0: 32768; -1: autotuned, else 0)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="bulk: first run one plain device copy of this many MiB (a known-size dispatch that "
                         "scales HBM byte counters read by a profiler)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-log2", type=int, default=23)
    return ap.parse_args()


def source_digest() -> str:
    h = hashlib.sha256()
    for f in ("hive.hip", "hive_device.hpp"):
        with open(os.path.join(ROOT, "paper_2510_15095_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(log2n: int) -> dict:
    """The CPU oracle (sequential Hive model, single thread) on the same
    sequence at 2^log2n keys."""
    import oracle
    from paper_2510_15095_amd import workload as wl
    n = 1 << log2n
    w = wl.bulk_workload(2, n)
    nb = int(np.ceil(n / (LOAD * S)))
    o = oracle.O2(S, 8, max(1024, nb * S // 100), oracle.ADDR_FIXED, nb)
    t0 = time.perf_counter()
    o.insert(w["ins_keys"], w["ins_vals"])
    o.lookup(w["query_keys"])
    o.delete(w["del_keys"])
    o.lookup(w["query_keys"])
    dt = time.perf_counter() - t0
    ops = 3.5 * n
    host_cores = os.cpu_count()
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else host_cores
    return {"value": round(ops / dt / 1e6, 3), "unit": "Mops/s", "cores": 1, "kind": "oracle",
            "sample": f"same sequence at 2^{log2n} keys ({nb} buckets, 95% load), {dt:.1f} s single-threaded",
            "host_cores": host_cores, "host_cores_usable": usable}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    tuned = {}
    if args.workload in ("suite", "bulk", "mixed", "resize", "served"):
        from paper_2510_15095_amd import autotune
        if args.autotune:
            autotune.tune({"suite": "all", "bulk": "probe"}.get(args.workload, args.workload))
        tuned = {sec: autotune.load(sec) for sec in ("resize", "executor", "probe", "probe_kernel")}
    if not args.resize_k:
        args.resize_k = (tuned.get("resize") or {}).get("resize_k", 1024)
    if args.blocks_per_cu < 0:
        args.blocks_per_cu = (tuned.get("executor") or {}).get("blocks_per_cu", 1)
    if args.probe_both < 0:
        args.probe_both = (tuned.get("probe") or {}).get("probe_both", 0)
    pk = tuned.get("probe_kernel") or {}
    if args.probe_tuning < 0:
        args.probe_tuning = 0 if args.probe_both else pk.get("probe_tuning", 0)
    if args.probe_grid < 0:
        args.probe_grid = pk.get("probe_grid", 0)
    run = {"suite": run_suite, "bulk": run_bulk, "mixed": run_mixed, "resize": run_resize, "served": run_served,
           "breakdown": run_breakdown, "hashes": run_hashes, "gather": run_gather}[args.workload]
    out = run(args)
    if tuned:
        out["autotuned"] = {k: v for k, v in tuned.items() if v}
    print(json.dumps(out), flush=True)


def run_suite(args):
    """The bulk step is the headline record; the mixed contended and served
    configurations are measured after it and reported as sub-records."""
    out = run_bulk(args)
    print("[bench] bulk done", file=sys.stderr, flush=True)
    if not args.no_mixed:
        out["mixed"] = mixed_subrecord(args)
        print("[bench] mixed done", file=sys.stderr, flush=True)
    if not args.no_served:
        rec = run_served(args)
        out["served"] = {"config": rec["config"], **rec["served"], "ms_per_step": rec["ms_per_step"]}
        print("[bench] served done", file=sys.stderr, flush=True)
    return out


def base_record(args, value, ms_step, workload, extra_config):
    return {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": workload, **extra_config},
    }


MIXED_UNIVERSE, MIXED_PRE, MIXED_NB0 = 1 << 26, 1 << 24, 1103765


def mixed_setup(args):
    """The mixed contended configuration's inputs, on the device: a 2^24-key
    prefill (uniform sample of a 2^26-key Zipf universe) and `batches`
    batches of 2^batch_log2 operations (40% insert incl. repeats, 40%
    delete, 20% lookup; Zipf(0.99); per-batch disjoint key sets per type)."""
    import torch
    from paper_2510_15095_amd import hive as H
    from paper_2510_15095_amd import workload as wl
    n_ops, nbat = 1 << args.batch_log2, args.batches
    ks = wl.KeyStream(3)
    gen = wl.mixed_batches([dict(seed=3, batch=b, n_ops=n_ops, universe=MIXED_UNIVERSE, stream=ks)
                            for b in range(nbat)])
    pre_keys = ks.keys(wl.DomainPerm(wl.batch_seed(3, 0xBEEF), MIXED_UNIVERSE).sample(MIXED_PRE))
    dev = torch.device("cuda:0")
    st = {
        "host": gen,
        "pre_keys": pre_keys,
        "pk": torch.from_numpy(pre_keys).to(dev),
        "pv": torch.from_numpy(wl.values_for(pre_keys)).to(dev),
        "batches": [tuple(torch.from_numpy(a).to(dev) for a in (mb["ops"], mb["keys"], mb["vals"])) for mb in gen],
        "vout": torch.empty(n_ops, dtype=torch.uint32, device=dev),
        "fout": torch.empty(n_ops, dtype=torch.uint8, device=dev),
        "table": H.Table(MIXED_NB0, addressing=H.HIVE_LINEAR, max_buckets=4 * MIXED_NB0, lf_expand_pct=95,
                         post_policy=1, resize_k=args.resize_k, max_batch=n_ops, probe_tuning=args.probe_tuning,
                         probe_grid=args.probe_grid),
    }
    print(f"[bench] mixed inputs ready: {nbat} batches of {n_ops} ops", file=sys.stderr, flush=True)
    return st


def mixed_prefill(st):
    import torch
    from paper_2510_15095_amd import hive as H
    t = st["table"]
    t.clear()
    t.insert(st["pk"], st["pv"], flags=H.HIVE_UNIQUE)
    torch.cuda.synchronize()


def mixed_time(args, st, executor, steps, warmup):
    """Per-batch times (ms) of `steps` passes over the batches, each after a
    fresh prefill: plain launches are timed per batch; the persistent
    executor drains all batches in one launch (its mean per batch is
    reported for every batch)."""
    import torch
    from paper_2510_15095_amd import hive as H
    t, batches, vout, fout = st["table"], st["batches"], st["vout"], st["fout"]
    nbat = len(batches)
    drain = H.hive_drain_create(16, args.blocks_per_cu, max(64, nbat), 4, 0) if executor == "persistent" else None

    def run(evs):
        if drain is not None:
            evs[0].record()
            for (o, k, v) in batches:
                H.hive_drain_submit(drain, t.h, H.HIVE_OP_MIXED, k, v, o, vout, fout)
            H.hive_drain_launch(drain, 0)
            evs[-1].record()
            return
        for j, (o, k, v) in enumerate(batches):
            evs[j].record()
            H.hive_mixed_batch(t.h, o, k, v, vout, fout)
        evs[-1].record()

    mk = lambda: [torch.cuda.Event(enable_timing=True) for _ in range(nbat + 1)]  # noqa: E731
    for _ in range(warmup):
        mixed_prefill(st)
        run(mk())
    times = []
    for step in range(steps):
        mixed_prefill(st)
        ev = mk()
        run(ev)
        torch.cuda.synchronize()
        print(f"[bench] mixed {executor} step {step} done", file=sys.stderr, flush=True)
        if drain is not None:
            times.append([ev[0].elapsed_time(ev[-1]) / nbat] * nbat)
        else:
            times.append([ev[j].elapsed_time(ev[j + 1]) for j in range(nbat)])
    if drain is not None:
        H.hive_drain_destroy(drain)
    return np.array(times)


def mixed_census(args, st):
    """One untimed plain pass: each batch's outcomes (lookups and deletes that
    found their key, new and replaced insert keys) and the fraction of
    entries in their second candidate after the prefill, from which the
    batch's algorithmic bytes follow; with --validate every output is also
    compared with the CPU dictionary."""
    import torch
    from paper_2510_15095_amd import hive as H
    from paper_2510_15095_amd import workload as wl
    t = st["table"]
    mixed_prefill(st)
    first, second, overflow = t.placement()
    f2 = second / max(1, first + second + overflow)
    o1 = None
    if args.validate:
        import oracle
        o1 = oracle.O1(1 << 25)
        o1.insert(st["pre_keys"], wl.values_for(st["pre_keys"]))
    live = t.stats()["live"]
    rows, mismatches = [], 0
    for (o, k, v), mb in zip(st["batches"], st["host"]):
        H.hive_mixed_batch(t.h, o, k, v, st["vout"], st["fout"])
        torch.cuda.synchronize()
        f = st["fout"][:mb["ops"].size].cpu().numpy()
        ops = mb["ops"]
        if o1 is not None:
            ov, of = o1.apply(ops, mb["keys"], mb["vals"])
            vo = st["vout"][:ops.size].cpu().numpy()
            mismatches += int(not (np.array_equal(f, of) and np.array_equal(vo, ov)))
        s2 = t.stats()
        lh = int(f[ops == wl.OP_LOOKUP].sum())
        dh = int(f[ops == wl.OP_DELETE].sum())
        u = int(np.unique(mb["keys"][ops == wl.OP_INSERT]).size)
        new = s2["live"] - live + dh
        rows.append({"n": int(ops.size), "look": int((ops == wl.OP_LOOKUP).sum()), "look_hit": lh,
                     "del": int((ops == wl.OP_DELETE).sum()), "del_hit": dh,
                     "ins": int((ops == wl.OP_INSERT).sum()), "ins_distinct": u, "ins_new": new,
                     "status": s2["status"]})
        live = s2["live"]
    final = t.stats()
    return {"f2": f2, "rows": rows, "mismatched_batches": mismatches if o1 is not None else None,
            "final": {k: final[k] for k in ("live", "n_buckets", "stash_count", "pending_count", "evictions",
                                            "evict_items", "status")}}


def mixed_bytes(row, f2):
    """Algorithmic bytes of one mixed batch (16-slot buckets, one touch =
    128 B): a lookup or delete that finds its key touches 1 + f2 buckets on
    average and a miss touches both candidates; an insert of a new key reads
    both candidates and claims a slot (8-byte CAS); a replace reads 1 + f2
    buckets and stores 8 bytes; a delete that finds its key stores 8 bytes;
    every insert and delete records itself in the dedupe set (one 128-byte
    line); every operation reads 9 B (op, key, value) and writes 5 B."""
    hit = BUCKET_BYTES * (1 + f2)
    miss = 2 * BUCKET_BYTES
    look = row["look_hit"] * hit + (row["look"] - row["look_hit"]) * miss
    dele = row["del_hit"] * (hit + 8) + (row["del"] - row["del_hit"]) * miss
    ins = row["ins_new"] * (miss + 8) + (row["ins_distinct"] - row["ins_new"]) * (hit + 8)
    dedupe = (row["ins"] + row["del"]) * BUCKET_BYTES
    return look + dele + ins + dedupe + 14 * row["n"]


def mixed_label(args):
    return (f"mixed contended: prefill 2^24 of a 2^26-key Zipf universe at 95% load (LINEAR, {MIXED_NB0} x "
            f"16-slot buckets, post-batch expansion at 95%), {args.batches} batches of 2^{args.batch_log2} ops "
            f"40/40/20 insert/delete/lookup, Zipf(0.99), per-type disjoint, dedupe on")


def run_mixed(args):
    """The mixed contended configuration through one executor (--executor)."""
    st = mixed_setup(args)
    ms = mixed_time(args, st, args.executor, args.steps, args.warmup)
    nbat, n_ops = args.batches, 1 << args.batch_log2
    ms_step = float(ms.sum(axis=1).mean())
    rec = base_record(args, nbat * n_ops / (ms_step * 1e-3) / 1e6, ms_step,
                      mixed_label(args) + f"; {args.executor} executor",
                      {"ops_per_step": nbat * n_ops, "batches": nbat, "resize_k": args.resize_k,
                       "probe_tuning": args.probe_tuning, "probe_grid": args.probe_grid})
    rec["batch_ms"] = {"mean": round(float(ms.mean()), 4), "p50": round(float(np.percentile(ms, 50)), 4),
                       "p99": round(float(np.percentile(ms, 99)), 4)}
    if args.validate:
        rec["census"] = mixed_census(args, st)
    st["table"].close()
    return rec


def mixed_subrecord(args):
    """Both executors on the mixed configuration, with the whole-batch
    roofline (algorithmic bytes of every batch over its time, against
    8 TB/s)."""
    st = mixed_setup(args)
    steps, warmup = max(1, args.mixed_steps), 1
    out = {"config": {"workload": mixed_label(args), "batches": args.batches,
                      "ops_per_batch": 1 << args.batch_log2, "resize_k": args.resize_k,
                      "persistent_blocks_per_cu": args.blocks_per_cu, "probe_tuning": args.probe_tuning,
                      "probe_grid": args.probe_grid, "steps": steps, "warmup": warmup}}
    times = {}
    for ex in ("plain", "persistent"):
        ms = mixed_time(args, st, ex, steps, warmup)
        times[ex] = ms
        total = ms.sum(axis=1).mean()
        out[ex] = {"mops": round(args.batches * (1 << args.batch_log2) / (total * 1e-3) / 1e6, 1),
                   "ms_per_batch": round(float(ms.mean()), 4),
                   "batch_ms_p50": round(float(np.percentile(ms, 50)), 4),
                   "batch_ms_p99": round(float(np.percentile(ms, 99)), 4)}
    cen = mixed_census(args, st)
    byts = np.array([mixed_bytes(r, cen["f2"]) for r in cen["rows"]])
    for ex in ("plain", "persistent"):
        per_batch_ms = times[ex].mean(axis=0)
        achieved = byts.sum() / (per_batch_ms.sum() * 1e-3) / 1e9
        out[ex]["roofline"] = {"kernel": "whole batch (all phases)", "bound": "hbm", "achieved": round(achieved, 1),
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                               "traffic": None, "algorithmic_bytes_per_batch": round(float(byts.mean()))}
    rows = cen["rows"]
    out["census"] = {"f2": round(cen["f2"], 4), "final": cen["final"],
                     "per_batch_mean": {k: round(float(np.mean([r[k] for r in rows])), 1)
                                        for k in ("look_hit", "del_hit", "ins", "ins_distinct", "ins_new")},
                     "statuses": sorted({r["status"] for r in rows})}
    if cen["mismatched_batches"] is not None:
        out["census"]["batches_differing_from_dictionary"] = cen["mismatched_batches"]
    st["table"].close()
    return out


def served_label(args):
    return (f"served multi-table loop: {args.tables} LINEAR tables of 2^U(12,{args.table_log2_max:g}) keys at 85% "
            f"load (HBM budget = reservations incl. 25% headroom), {args.requests} mixed requests (50% lookup, "
            f"25% insert, 25% delete; uniform or Zipf(0.99) keys) of 2^U(0,{args.request_log2:g}) ops on random "
            f"tables; persistent executor vs per-request launches on 8 streams; Poisson arrivals at "
            f"{args.lambda_sweep} x the plain-launch saturation rate")


def run_served(args):
    """Served multi-table loop: many LINEAR tables (log-uniform sizes,
    created at 85% load, 25% HBM headroom each), mixed requests of
    log-uniform sizes aimed at random tables.  First all requests arrive at
    once (saturation throughput of each mode), then Poisson arrivals at
    fractions of the plain-launch saturation rate (p50/p99 latency of each
    mode)."""
    import torch
    from paper_2510_15095_amd import serve as sv
    specs = sv.make_specs(args.tables, 5, log2_min=12, log2_max=args.table_log2_max)
    reqs = sv.make_requests(specs, args.requests, 5, rate=0, log2_max_size=args.request_log2)
    print(f"[bench] {len(reqs)} requests on {len(specs)} tables generated", file=sys.stderr, flush=True)
    budget = sv.footprint_bytes(specs)
    srv = sv.Server(specs, budget, max_request=1 << int(np.ceil(args.request_log2)), ring=1024, streams=8,
                    blocks_per_cu=args.blocks_per_cu)
    res = {}
    validate = {}
    expect = served_expectation(specs, reqs) if args.validate else None
    for mode in ("plain", "persistent"):
        srv.load()
        srv.run(reqs[: min(200, len(reqs))], mode)  # warm-up
        srv.load()
        r = srv.run(reqs, mode, outputs=expect is not None, timeout_s=600)
        if expect is not None:
            bad = sum(not (np.array_equal(f, of) and np.array_equal(v, ov))
                      for (v, f), (ov, of) in zip(r.pop("results"), expect))
            validate[mode] = {"requests_differing_from_dictionary": bad}
        res[mode + "_saturation"] = r
        print(f"[bench] served {mode} saturation run done", file=sys.stderr, flush=True)
    mean_ops = float(np.mean([r.n for r in reqs]))
    sat_rate = res["plain_saturation"]["mops"] * 1e6 / mean_ops
    for frac in [float(x) for x in args.lambda_sweep.split(",") if x]:
        rate = frac * sat_rate
        gaps = np.random.default_rng(55).exponential(1.0 / rate, len(reqs))
        arrivals = np.cumsum(gaps) - gaps[0]
        for r, a in zip(reqs, arrivals):
            r.arrival = float(a)
        for mode in ("plain", "persistent"):
            srv.load()
            res[f"{mode}_poisson_{frac:g}"] = srv.run(reqs, mode, timeout_s=600)
            res[f"{mode}_poisson_{frac:g}"]["rate_req_per_s"] = round(rate, 1)
            print(f"[bench] served {mode} at {frac:g} x saturation done", file=sys.stderr, flush=True)
    srv.close()
    torch.cuda.synchronize()
    p = res["persistent_saturation"]
    rec = base_record(args, p["mops"], p["span_s"] * 1e3, served_label(args),
                      {"ops_per_step": p["ops"], "tables": args.tables, "requests": args.requests,
                       "mean_request_ops": round(mean_ops, 1),
                       "plain_saturation_req_per_s": round(sat_rate, 1)})
    rec["served"] = {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                     for k, v in res.items()}
    if validate:
        rec["served"]["validate"] = validate
    return rec


def served_expectation(specs, reqs):
    """Every request's outputs from the CPU dictionary: each table's
    requests replayed in submission order through a dictionary loaded with
    that table's keys."""
    import oracle
    from paper_2510_15095_amd import workload as wl
    dicts, out = {}, []
    for r in reqs:
        if r.table not in dicts:
            sp = specs[r.table]
            keys = wl.KeyStream(sp.seed).range(0, sp.n_keys)
            dicts[r.table] = oracle.O1(2 * sp.n_keys)
            dicts[r.table].insert(keys, wl.values_for(keys))
        out.append(dicts[r.table].apply(r.ops, r.keys, r.vals))
    print("[bench] served: dictionary answers ready", file=sys.stderr, flush=True)
    return out


BREAKDOWN_LF = (0.55, 0.65, 0.75, 0.85, 0.90, 0.95, 0.97)


def run_breakdown(args):
    """Insert time by step against load factor (the insertion step breakdown
    of Section V-D: steps 1 and 2 dominate at moderate load, the later steps
    grow near full).  A FIXED table of the bulk geometry (4,415,057 x 16-slot
    buckets) is built in slices, from empty to 55% load and then to 65, 75,
    85, 90, 95 and 97%, one hive_insert_batch of unique uniform keys per
    slice, with phase timing on: steps 1 and 2 (replace, claim-then-commit)
    run in the probe launch, step 3 (bounded cuckoo chains) in the eviction
    launch and step 4 (stash or pending) in a launch of its own.  Per slice:
    the three times and their shares, items sent to eviction, displacements
    and stash placements; medians over the timed builds."""
    import torch
    from paper_2510_15095_amd import hive as H
    from paper_2510_15095_amd import workload as wl
    nb = 4415057
    slots = nb * S
    bounds = [0] + [int(round(f * slots)) for f in BREAKDOWN_LF]
    ks = wl.KeyStream(6)
    keys = ks.range(0, bounds[-1])
    dk = torch.from_numpy(keys).cuda()
    dv = torch.from_numpy(wl.values_for(keys)).cuda()
    del keys
    widest = max(b - a for a, b in zip(bounds, bounds[1:]))
    t = H.Table(nb, slots_per_bucket=S, max_evictions=8, max_batch=widest)
    H.hive_phase_timing(t.h, True)
    fields = ("evictions", "evict_items", "stash_inserts", "pending_inserts")

    def build():
        t.clear()
        torch.cuda.synchronize()
        H.hive_phase_times(t.h)
        prev = t.stats()
        rows = []
        for a, b in zip(bounds, bounds[1:]):
            t.insert(dk[a:b], dv[a:b], flags=H.HIVE_UNIQUE)
            ph = H.hive_phase_times(t.h)
            st = t.stats()
            rows.append({"inserts": b - a, **{k: ph[k] for k in ("probe", "evict", "stash", "finish")},
                         **{f: st[f] - prev[f] for f in fields}})
            prev = st
        assert st["status"] in (H.HIVE_OK, H.HIVE_WARN_PENDING) and st["live"] == bounds[-1], st
        return rows

    for _ in range(args.warmup):
        build()
    runs = [build() for _ in range(args.steps)]
    out_rows = []
    lo = 0.0
    for i, hi in enumerate(BREAKDOWN_LF):
        probe = float(np.median([r[i]["probe"] for r in runs]))
        evict = float(np.median([r[i]["evict"] for r in runs]))
        stash = float(np.median([r[i]["stash"] for r in runs]))
        fin = float(np.median([r[i]["finish"] for r in runs]))
        last = runs[-1][i]
        steps = probe + evict + stash
        out_rows.append({"load_from": lo, "load_to": hi, "inserts": last["inserts"],
                         "steps12_ms": round(probe, 4), "step3_ms": round(evict, 4), "step4_ms": round(stash, 4),
                         "finish_ms": round(fin, 4), "steps12_share": round(probe / steps, 4),
                         "step3_share": round(evict / steps, 4), "step4_share": round(stash / steps, 4),
                         "to_eviction": last["evict_items"], "displacements": last["evictions"],
                         "stash": last["stash_inserts"], "pending": last["pending_inserts"],
                         "mops": round(last["inserts"] / ((steps + fin) * 1e-3) / 1e6, 1)})
        lo = hi
    total_ms = sum(r["steps12_ms"] + r["step3_ms"] + r["step4_ms"] + r["finish_ms"] for r in out_rows)
    rec = base_record(args, bounds[-1] / (total_ms * 1e-3) / 1e6, total_ms,
                      f"insert time by step: FIXED {nb} x {S}-slot buckets built from empty to 97% load in "
                      f"{len(BREAKDOWN_LF)} slices of unique uniform keys, probe launch (steps 1-2), eviction "
                      f"launch (step 3) and stash launch (step 4) timed apart",
                      {"slices": len(BREAKDOWN_LF), "max_evictions": 8})
    rec["breakdown"] = out_rows
    t.close()
    return rec


def run_hashes(args):
    """Hash-function study (Section III-C): the collision speedup ratio
    CSR = E[Y] / Y of BitHash1/2, CRC-32, CRC-64, MurmurHash3 and CityHash32
    over m = 512^2 buckets for n = 512 ... 2048^2 keys (E[Y] from the
    uniform-hashing theorem), for unique uniform keys and for the sequential
    keys 1..n (the paper does not say which keys it hashed); then each hash's
    rate over 2^26 keys (key in, bucket out, timed with HIP events); then the
    bulk insert rate of a 95%-load table under each hash pair."""
    import torch
    from paper_2510_15095_amd import hash_study as hs
    from paper_2510_15095_amd import hive as H
    from paper_2510_15095_amd import workload as wl
    m = 512 * 512
    ns = [512 << k for k in range(14)]  # 512 ... 4,194,304 = 2048^2
    uniform = torch.from_numpy(wl.KeyStream(7).range(0, ns[-1])).cuda()
    sequential = torch.arange(1, ns[-1] + 1, dtype=torch.int64).to(torch.uint32).cuda()
    scratch = torch.empty(2 + m // 32, dtype=torch.uint32, device="cuda")
    csr = {}
    for name, keys in (("uniform", uniform), ("sequential", sequential)):
        csr[name] = {}
        for kind in H.HASH_KINDS:
            row = []
            for n in ns:
                y = H.hive_hash_collisions(kind, keys[:n], m, scratch)
                row.append(round(hs.csr(n, m, y), 4))
            csr[name][kind] = row
    big = torch.from_numpy(wl.KeyStream(8).range(0, 1 << args.keys_log2)).cuda()
    out = torch.empty_like(big)
    rates = {}
    reps = max(args.steps, 1)
    for kind in H.HASH_KINDS:
        for _ in range(max(args.warmup, 1)):
            H.hive_hash_buckets(kind, big, m, out)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            H.hive_hash_buckets(kind, big, m, out)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        rates[kind] = {"ms": round(ms, 4), "mops": round(big.numel() / (ms * 1e-3) / 1e6, 1),
                       "gb_s": round(8 * big.numel() / (ms * 1e-3) / 1e9, 1)}
    del big, out
    # insert throughput of the table under each hash pair (the paper's
    # figure of hash-pair insertion throughput, 2^20 .. 2^25 unique keys):
    # a FIXED 16-slot table sized for 95% load, cleared and built per rep
    pairs = {"bithash1+bithash2": H.HIVE_PAIR_BITHASH, "crc32+crc64": H.HIVE_PAIR_CRC,
             "murmur3+city32": H.HIVE_PAIR_MURMUR, "bithash1+bithash2+city32 (three candidates)": H.HIVE_PAIR_TRIPLE}
    host_keys = wl.KeyStream(9).range(0, 1 << 25)
    ik = torch.from_numpy(host_keys).cuda()
    iv = torch.from_numpy(wl.values_for(host_keys)).cuda()
    insert = {name: {} for name in pairs}
    for log2n in (20, 22, 24, 25):
        n = 1 << log2n
        nb = int(np.ceil(n / (LOAD * S)))
        for name, pair in pairs.items():
            t = H.Table(nb, hash_pair=pair, max_batch=n)
            times = []
            for rep in range(max(args.warmup, 1) + reps):
                t.clear()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                t.insert(ik[:n], iv[:n], flags=H.HIVE_UNIQUE)
                b.record()
                torch.cuda.synchronize()
                if rep >= max(args.warmup, 1):
                    times.append(a.elapsed_time(b))
            st = t.stats()
            assert st["live"] == n and st["status"] in (H.HIVE_OK, H.HIVE_WARN_PENDING), st
            insert[name][str(log2n)] = round(n / (float(np.median(times)) * 1e-3) / 1e6, 1)
            t.close()
    rec = base_record(args, rates["bithash1"]["mops"], rates["bithash1"]["ms"],
                      f"hash study: CSR of 6 hashes over 512^2 buckets for 512..2048^2 uniform and sequential keys; "
                      f"hash rate over 2^{args.keys_log2} keys (value: BitHash1); insert Mops/s of a 95% table per "
                      f"hash pair at 2^20..2^25 keys", {"buckets": m, "n": ns})
    rec["csr"] = csr
    rec["rates"] = rates
    rec["insert_mops_by_pair"] = insert
    rec["roofline"] = {"kernel": "hash_study bucket_kernel (BitHash1)", "bound": "hbm",
                       "achieved": rates["bithash1"]["gb_s"], "peak": 8000.0, "unit": "GB/s",
                       "frac": round(rates["bithash1"]["gb_s"] / 8000.0, 4), "traffic": None}
    return rec


def run_gather(args):
    """Gather ceiling: random 128-byte line reads (the access pattern of
    bucket probing, with the probe kernel's shape) over a table of the bulk
    geometry (4,415,057 lines, 565 MB, larger than the 256 MB last-level
    cache) and of the mixed geometry (1,103,765 lines, 141 MB, which fits
    it); 2^26 uniform random line indices, HIP-event timing."""
    import torch
    from paper_2510_15095_amd import hive as H
    n = 1 << args.keys_log2
    res = {}
    for name, lines in (("bulk_565MB", 4415057), ("mixed_141MB", 1103765)):
        table = torch.randint(0, 2 ** 62, (lines * 16,), dtype=torch.int64, device="cuda").view(torch.uint64)
        idx = torch.randint(0, lines, (n,), dtype=torch.int64, device="cuda").to(torch.uint32)
        out = torch.empty(n, dtype=torch.uint64, device="cuda")
        for _ in range(max(args.warmup, 1)):
            H.hive_gather_lines(table, idx, out)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(max(args.steps, 1)):
            H.hive_gather_lines(table, idx, out)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / max(args.steps, 1)
        res[name] = {"ms": round(ms, 4), "line_gb_s": round(128 * n / (ms * 1e-3) / 1e9, 1),
                     "all_gb_s": round(140 * n / (ms * 1e-3) / 1e9, 1)}
        del table, idx, out
    bulk = res["bulk_565MB"]
    rec = base_record(args, n / (bulk["ms"] * 1e-3) / 1e6, bulk["ms"],
                      f"gather ceiling: 2^{args.keys_log2} random 128-byte line reads over 565 MB and 141 MB "
                      f"tables (value: lines per second over 565 MB, in millions)", {"lines_read": n})
    rec["gather"] = res
    rec["roofline"] = {"kernel": "gather_kernel (565 MB)", "bound": "hbm", "achieved": bulk["all_gb_s"],
                       "peak": 8000.0, "unit": "GB/s", "frac": round(bulk["all_gb_s"] / 8000.0, 4), "traffic": None}
    return rec


def resize_geometry(nb, live, extra, initial, max_b, K, lf_e=90):
    """Bucket count after the expansion rule of Section IV-C (K pairs at a
    time while live + extra exceeds lf_e% of the slots)."""
    while (live + extra) * 100 > lf_e * nb * S and nb < max_b:
        nb = min(nb + K, max_b)
    return nb


def resize_validate(args, t, keys, vals, dkeys, ks, nb0, max_b):
    """Untimed validation of the resize cycle: after every insert and delete
    batch the table is dumped, every stored key is mapped back to its
    generator index and checked against a bitmap of the indices that must be
    live (each exactly once, with its value); the geometry after each insert
    batch equals the expansion rule's, and after each delete batch the table
    is not over the expansion threshold and stops contracting only at its
    initial size or at a merge pair that does not fit (Section IV-C-2)."""
    import torch
    from paper_2510_15095_amd import hive as H
    from paper_2510_15095_amd import workload as wl
    nbat, nb_ops = args.batches, 1 << args.batch_log2
    n = nbat * nb_ops
    n_del = dkeys.numel()
    didx = ks.index_of(dkeys.cpu().numpy())
    words = torch.empty(n + 1, dtype=torch.uint64, device="cuda")
    where = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    live_bm = np.zeros(n, bool)
    t.clear()
    t0 = time.perf_counter()
    nb, failures, checks = nb0, [], 0

    def check(label, want_geometry=None):
        nonlocal checks
        st = t.stats()
        cnt = H.hive_dump(t.h, words, where)
        w = words[:cnt].cpu().numpy()
        k = (w & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        idx = ks.index_of(k)
        seen = np.zeros(n, bool)
        seen[idx] = True
        ok = (cnt == st["live"] and int(seen.sum()) == cnt and np.array_equal(seen, live_bm)
              and np.array_equal((w >> np.uint64(32)).astype(np.uint32), wl.values_for(k)))
        if want_geometry is not None:
            ok = ok and st["n_buckets"] == want_geometry
        else:
            ok = ok and st["live"] * 100 <= 90 * st["n_buckets"] * S
            if ok and st["live"] * 100 < 25 * st["n_buckets"] * S and st["n_buckets"] > nb0:
                im, sp = st["index_mask"], st["split_ptr"]
                if sp == 0:
                    im, sp = im >> 1, (im >> 1) + 1
                lo, hi = sp - 1, sp + im
                wh = where[:cnt].cpu().numpy()
                ok = int((wh == hi).sum()) > S - int((wh == lo).sum())
        checks += 1
        if not ok:
            failures.append(label)
        return st

    for b in range(nbat):
        st0 = t.stats()
        want = resize_geometry(st0["n_buckets"], st0["live"], nb_ops, nb0, max_b, args.resize_k)
        t.insert(keys[b * nb_ops:(b + 1) * nb_ops], vals[b * nb_ops:(b + 1) * nb_ops], flags=H.HIVE_UNIQUE)
        live_bm[b * nb_ops:(b + 1) * nb_ops] = True
        want = resize_geometry(want, (b + 1) * nb_ops, 0, nb0, max_b, args.resize_k)
        check(f"insert batch {b}", want)
        print(f"[bench] resize validation: insert batch {b} checked", file=sys.stderr, flush=True)
    dout = torch.empty(nb_ops, dtype=torch.uint8, device="cuda")
    for b in range((n_del + nb_ops - 1) // nb_ops):
        lo_, hi_ = b * nb_ops, min(n_del, (b + 1) * nb_ops)
        H.hive_delete_batch(t.h, dkeys[lo_:hi_], dout[:hi_ - lo_], H.HIVE_UNIQUE)
        if not bool(dout[:hi_ - lo_].all()):
            failures.append(f"delete batch {b}: a delete missed its key")
        live_bm[didx[lo_:hi_]] = False
        check(f"delete batch {b}")
        print(f"[bench] resize validation: delete batch {b} checked", file=sys.stderr, flush=True)
    return {"batches_checked": checks, "failures": failures, "seconds": round(time.perf_counter() - t0, 1)}


def run_resize(args):
    """Dynamic resize cycle: a LINEAR table of 2^16 buckets (2^20 slots)
    takes `batches` batches of 2^22 unique uniform inserts with pre-batch
    expansion at 90% load, then 90% of the keys are deleted in random order
    in 2^22-op batches with post-batch contraction under 25% load."""
    import torch
    from paper_2510_15095_amd import hive as H
    from paper_2510_15095_amd import workload as wl
    nbat, nb_ops = args.batches, 1 << args.batch_log2
    n = nbat * nb_ops
    n_del = int(n * 0.9)
    ks = wl.KeyStream(4)
    dev = torch.device("cuda:0")
    keys = torch.from_numpy(ks.range(0, n)).to(dev)
    vals = torch.from_numpy(wl.values_for(keys.cpu().numpy())).to(dev)
    dkeys = torch.from_numpy(ks.keys(wl.DomainPerm(wl.batch_seed(4, 0xDE1), n).sample(n_del))).to(dev)
    print(f"[bench] resize inputs ready: {n} inserts, {n_del} deletes", file=sys.stderr, flush=True)
    nb0 = 1 << 16
    max_b = 1
    while max_b * 16 * 0.9 < n * 1.05:
        max_b *= 2
    t = H.Table(nb0, addressing=H.HIVE_LINEAR, max_buckets=max_b, pre_expand=1, post_policy=1, lf_expand_pct=90,
                lf_contract_pct=25, resize_k=args.resize_k, max_batch=nb_ops)
    dout = torch.empty(nb_ops, dtype=torch.uint8, device=dev)
    n_del_batches = (n_del + nb_ops - 1) // nb_ops
    validation = resize_validate(args, t, keys, vals, dkeys, ks, nb0, max_b) if args.validate else None

    def run(ev):
        t.clear()
        ev[0].record()
        for b in range(nbat):
            t.insert(keys[b * nb_ops:(b + 1) * nb_ops], vals[b * nb_ops:(b + 1) * nb_ops], flags=H.HIVE_UNIQUE)
        ev[1].record()
        peak = t.stats()["n_buckets"]  # synchronises between the two timed intervals
        ev[2].record()
        for b in range(n_del_batches):
            dk = dkeys[b * nb_ops:min(n_del, (b + 1) * nb_ops)]
            H.hive_delete_batch(t.h, dk, dout[:dk.numel()], H.HIVE_UNIQUE)
        ev[3].record()
        return peak

    mk = lambda: [torch.cuda.Event(enable_timing=True) for _ in range(4)]  # noqa: E731
    for _ in range(args.warmup):
        run(mk())
    res = []
    peak = 0
    for step in range(args.steps):
        ev = mk()
        peak = run(ev)
        print(f"[bench] resize step {step} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        res.append((ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])))
    ms = np.array(res)
    st = t.stats()
    ms_step = float(ms.sum(axis=1).mean())
    rec = base_record(args, (n + n_del) / (ms_step * 1e-3) / 1e6, ms_step,
                      f"dynamic resize cycle: LINEAR from 2^16 x 16-slot buckets, {nbat} batches of 2^{args.batch_log2} "
                      f"unique uniform inserts with pre-batch expansion at 90%, then delete 90% in random order with "
                      f"contraction under 25%, K={args.resize_k}",
                      {"ops_per_step": n + n_del, "resize_k": args.resize_k})
    rec["phase_mops"] = {"insert_with_growth": round(n / (ms[:, 0].mean() * 1e-3) / 1e6, 1),
                         "delete_with_contraction": round(n_del / (ms[:, 1].mean() * 1e-3) / 1e6, 1)}
    rec["peak_buckets"] = peak
    rec["final_stats"] = {k: st[k] for k in ("live", "n_buckets", "stash_count", "pending_count", "status")}
    if validation is not None:
        rec["validation"] = validation
    t.close()
    return rec


def run_bulk(args):
    import torch
    from paper_2510_15095_amd import hive as H
    from paper_2510_15095_amd import workload as wl

    n = 1 << args.keys_log2
    set32 = args.entry_bits == 32
    slots = 32 if set32 else S
    nb = int(np.ceil(n / (LOAD * slots)))
    w = wl.bulk_workload(2, n)
    dev = torch.device("cuda:0")
    keys = torch.from_numpy(w["ins_keys"]).to(dev)
    vals = torch.from_numpy(w["ins_vals"]).to(dev)
    qk = torch.from_numpy(w["query_keys"]).to(dev)
    dk = torch.from_numpy(w["del_keys"]).to(dev)
    vout = torch.empty(n, dtype=torch.uint32, device=dev)
    fout = torch.empty(n, dtype=torch.uint8, device=dev)
    dout = torch.empty(dk.numel(), dtype=torch.uint8, device=dev)
    t = (H.Table(nb, slots_per_bucket=32, entry_bits=32, max_evictions=8, max_batch=n, probe_grid=args.probe_grid)
         if set32 else
         H.Table(nb, slots_per_bucket=S, max_evictions=8, max_batch=n, probe_both=args.probe_both,
                 probe_tuning=args.probe_tuning, probe_grid=args.probe_grid))
    if set32:
        vals = None
    n_present = int((w["query_idx"] < n).sum())
    deleted = np.zeros(n, bool)
    deleted[w["del_idx"]] = True
    qi = w["query_idx"]
    n_present2 = int(((qi < n) & ~deleted[np.minimum(qi, n - 1)]).sum())
    del w

    if args.copy_calibration_mib:
        src = torch.empty(args.copy_calibration_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    phases = ("clear", "insert", "lookup", "delete", "lookup2")

    def step(ev):
        ev[0].record()
        t.clear()
        ev[1].record()
        t.insert(keys, vals, flags=H.HIVE_UNIQUE)
        ev[2].record()
        H.hive_lookup_batch(t.h, qk, vout, fout)
        ev[3].record()
        H.hive_delete_batch(t.h, dk, dout, H.HIVE_UNIQUE)
        ev[4].record()
        H.hive_lookup_batch(t.h, qk, vout, fout)
        ev[5].record()

    mk = lambda: [torch.cuda.Event(enable_timing=True) for _ in range(6)]  # noqa: E731
    for _ in range(args.warmup):
        step(mk())
    torch.cuda.synchronize()
    # placement census after a full build (untimed): lookups of present keys
    # touch one bucket when the key sits in its first candidate, two otherwise
    t.clear()
    t.insert(keys, vals, flags=H.HIVE_UNIQUE)
    first, second, overflow = t.placement()
    st_build = t.stats()
    frac_second = second / max(1, first + second + overflow)

    evs = [mk() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ev in evs:
        step(ev)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([[ev[j].elapsed_time(ev[j + 1]) for j in range(5)] for ev in evs])
    st = t.stats()
    ops_step = n + n + dk.numel() + n
    ms_step = float(ms.sum(axis=1).mean())

    # roofline of the lookup kernel: algorithmic bytes per launch =
    # hits * 128 * (1 + f_second) + misses * 256 (both candidates) + 9 B of I/O
    # per operation (key in, value and found flag out)
    def lookup_bytes(hits):
        misses = n - hits
        io = 5 if set32 else 9  # key in, (value and) found flag out
        return hits * BUCKET_BYTES * (1 + frac_second) + misses * 2 * BUCKET_BYTES + io * n
    lk_ms = (ms[:, 2].mean() + ms[:, 4].mean()) / 2
    lk_bytes = (lookup_bytes(n_present) + lookup_bytes(n_present2)) / 2
    achieved = lk_bytes / (lk_ms * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "lookup_bulk95_traffic.json")
    if os.path.exists(tfile) and not set32:
        rec = json.load(open(tfile))
        if rec.get("source_digest") == source_digest():
            traffic = rec.get("bytes_per_launch")

    phase_mops = {
        "insert": n / (ms[:, 1].mean() * 1e-3) / 1e6,
        "lookup": n / (ms[:, 2].mean() * 1e-3) / 1e6,
        "delete": dk.numel() / (ms[:, 3].mean() * 1e-3) / 1e6,
        "lookup2": n / (ms[:, 4].mean() * 1e-3) / 1e6,
    }
    out = {
        "metric": METRIC,
        "value": round(ops_step / (ms_step * 1e-3) / 1e6, 1),
        "unit": "Mops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "probe_both": args.probe_both,
            "probe_tuning": 0 if set32 else args.probe_tuning,
            "probe_grid": args.probe_grid,
            "workload": f"bulk build to 95% load, plain launch: 2^{args.keys_log2} unique uniform keys into "
                        f"{nb} x {slots}-slot buckets (FIXED"
                        f"{', key-only set of 32-bit entries' if set32 else ''}), 2^{args.keys_log2} lookups at "
                        f"50% hits, delete 2^{args.keys_log2 - 1}, re-lookup",
            "ops_per_step": ops_step,
            "load_factor": round(n / (nb * slots), 6),
        },
        "phase_mops": {k: round(v, 1) for k, v in phase_mops.items()},
        "phase_ms": {p: round(float(ms[:, j].mean()), 4) for j, p in enumerate(phases)},
        "wall_ms_per_step": round(wall / args.steps * 1e3, 4),
        "build_stats": {k: st_build[k] for k in ("evictions", "evict_items", "stash_count", "pending_count",
                                                 "full_chains")},
        "placement": {"first": first, "second": second, "overflow": overflow},
        "roofline": {
            "kernel": "set_ops_kernel<lookup>" if set32 else "ops_kernel<16, lookup>",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": round(lk_bytes),
            "avg_launch_ms": round(float(lk_ms), 4),
            "one_touch_frac": round(n / (lk_ms * 1e-3) / (HBM_PEAK_GBS * 1e9 / BUCKET_BYTES), 4),
        },
        "status": st["status"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_log2)
    t.close()
    return out


if __name__ == "__main__":
    main()
