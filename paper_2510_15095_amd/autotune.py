"""Autotuner: the table's tunable sizes, picked by measurement on this GPU.

* bucket width S (16, 32 or 64 slots): a bulk build to 95% load followed by
  lookups (50% hits), scored by operations per second;
* resize step K (pairs per split/merge step): growth of a LINEAR table from
  a small start under pre-batch expansion, then contraction, scored by
  operations per second including the resize work;
* resident blocks per CU of the persistent executor: a queue of small mixed
  batches, scored by operations per second;
* the probe kernel (16-slot BitHash tables): per operation kind (insert,
  delete, lookup, mixed) the variant -- occupancy target in waves per SIMD
  and bucket loads in flight per wave -- on the bulk workload at 95% load,
  then the cap on blocks per probe launch (how many 256-operation tiles each
  block strides over).

Each candidate runs once to warm up and is then timed `reps` times with HIP
events around the measured work only (table clears and prefills run outside
the timed region); the median decides.  A candidate replaces the default
only when it beats it by more than MARGIN, so run-to-run noise does not
flip the choice.  Winners are cached per (GPU architecture, workload) in a
JSON file ($HIVE_TUNE_CACHE, default ~/.cache/hive_mi355x/tuned.json) and
returned by `load()`, which falls back to the values measured for the
architecture shipped with the package (tuned_<arch>.json) when the cache
has none.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from . import hive as H
from . import workload as wl

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "hive_mi355x", "tuned.json")
SHIPPED_DIR = os.path.dirname(os.path.abspath(__file__))
MARGIN = 0.02  # a candidate must beat the default by 2% to replace it


def cache_path() -> str:
    return os.environ.get("HIVE_TUNE_CACHE", DEFAULT_CACHE)


def gpu_arch() -> str:
    import torch
    return getattr(torch.cuda.get_device_properties(0), "gcnArchName", "unknown").split(":")[0]


def _timed(fn, reps: int, prep=None) -> float:
    """Median milliseconds of fn() over `reps` runs after one warm-up; prep()
    (untimed) runs before each."""
    import torch
    if prep:
        prep()
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        if prep:
            prep()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b))
    return float(np.median(out))


def _pick(scores: dict, default):
    """The best-scoring candidate if it beats the default by more than
    MARGIN, else the default."""
    best = max(scores, key=scores.get)
    return best if scores[best] > scores[default] * (1 + MARGIN) else default


def tune_bucket_width(n_keys: int = 1 << 22, reps: int = 3) -> dict:
    import torch
    w = wl.bulk_workload(12, n_keys)
    k = torch.from_numpy(w["ins_keys"]).cuda()
    v = torch.from_numpy(w["ins_vals"]).cuda()
    q = torch.from_numpy(w["query_keys"]).cuda()
    vo = torch.empty(q.numel(), dtype=torch.uint32, device="cuda")
    fo = torch.empty(q.numel(), dtype=torch.uint8, device="cuda")
    scores = {}
    for S in (16, 32, 64):
        nb = int(np.ceil(n_keys / (0.95 * S)))
        t = H.Table(nb, slots_per_bucket=S, max_batch=n_keys)

        def step():
            t.insert(k, v, flags=H.HIVE_UNIQUE)
            H.hive_lookup_batch(t.h, q, vo, fo)
        ms = _timed(step, reps, prep=t.clear)
        scores[S] = 2 * n_keys / (ms * 1e-3) / 1e6
        t.close()
    best = _pick(scores, 16)
    return {"slots_per_bucket": int(best), "scores_mops": {str(s): round(x, 1) for s, x in scores.items()}}


def tune_probe_both(n_keys: int = 1 << 24, reps: int = 3) -> dict:
    """Lookups (50% hits) and deletes after a 95% build, with the second
    candidate probed only after a miss (0) or together with the first (1)."""
    import torch
    w = wl.bulk_workload(15, n_keys)
    k = torch.from_numpy(w["ins_keys"]).cuda()
    v = torch.from_numpy(w["ins_vals"]).cuda()
    q = torch.from_numpy(w["query_keys"]).cuda()
    dk = torch.from_numpy(w["del_keys"]).cuda()
    vo = torch.empty(q.numel(), dtype=torch.uint32, device="cuda")
    fo = torch.empty(q.numel(), dtype=torch.uint8, device="cuda")
    nb = int(np.ceil(n_keys / (0.95 * 16)))
    scores = {}
    for pb in (0, 1):
        t = H.Table(nb, max_batch=n_keys, probe_both=pb)
        t.insert(k, v, flags=H.HIVE_UNIQUE)

        def step():
            H.hive_lookup_batch(t.h, q, vo, fo)
        ms_l = _timed(step, reps)

        def rebuild():
            t.clear()
            t.insert(k, v, flags=H.HIVE_UNIQUE)
        ms_d = _timed(lambda: H.hive_delete_batch(t.h, dk, None, H.HIVE_UNIQUE), max(1, reps // 2), prep=rebuild)
        scores[pb] = (q.numel() + dk.numel()) / ((ms_l + ms_d) * 1e-3) / 1e6
        t.close()
    best = _pick(scores, 0)
    return {"probe_both": int(best), "scores_mops": {str(k): round(x, 1) for k, x in scores.items()}}


def tune_probe_kernel(n_keys: int = 1 << 26, reps: int = 5, mixed_ops: int = 1 << 22,
                      grids=(0, 4096, 8192, 131072, 1 << 20)) -> dict:
    """Probe-kernel variant per operation kind, then the probe grid cap, on
    the bulk workload: 2^26 unique keys built to 95% load in 16-slot buckets
    (inserts), lookups with 50% hits, deletes of half the keys, and Zipf(0.99)
    mixed batches (40/40/20) of 2^22 operations on the built table."""
    import torch
    w = wl.bulk_workload(2, n_keys)
    k = torch.from_numpy(w["ins_keys"]).cuda()
    v = torch.from_numpy(w["ins_vals"]).cuda()
    q = torch.from_numpy(w["query_keys"]).cuda()
    dk = torch.from_numpy(w["del_keys"]).cuda()
    mb = wl.mixed_batch(16, 0, mixed_ops, 2 * n_keys, stream=w["stream"], value_salt=1)
    mo, mk, mv = (torch.from_numpy(mb[f]).cuda() for f in ("ops", "keys", "vals"))
    del w, mb
    vo = torch.empty(q.numel(), dtype=torch.uint32, device="cuda")
    fo = torch.empty(q.numel(), dtype=torch.uint8, device="cuda")
    nb = int(np.ceil(n_keys / (0.95 * 16)))
    kinds = H.PROBE_KINDS
    ms = {kind: {} for kind in kinds}

    def measure(tuning: int, grid: int) -> dict:
        t = H.Table(nb, max_batch=max(n_keys, mixed_ops), probe_tuning=tuning, probe_grid=grid)

        def build():
            t.clear()
            t.insert(k, v, flags=H.HIVE_UNIQUE)
        out = {"insert": _timed(lambda: t.insert(k, v, flags=H.HIVE_UNIQUE), reps, prep=t.clear)}
        build()
        out["lookup"] = _timed(lambda: H.hive_lookup_batch(t.h, q, vo, fo), reps)
        out["delete"] = _timed(lambda: H.hive_delete_batch(t.h, dk, None, H.HIVE_UNIQUE), reps, prep=build)
        out["mixed"] = _timed(lambda: H.hive_mixed_batch(t.h, mo, mk, mv, vo, fo), reps, prep=build)
        t.close()
        return out

    for var in range(len(H.PROBE_VARIANTS)):
        ins = var if var in H.PROBE_INSERT_VARIANTS else 0
        got = measure(H.probe_tuning(ins, var, var, var), 0)
        _progress(f"probe variant {var} {H.PROBE_VARIANTS[var]}: " +
                  ", ".join(f"{kk} {x:.3f} ms" for kk, x in got.items()))
        for kind in kinds:
            if kind != "insert" or var == ins:
                ms[kind][var] = got[kind]
    n_ops = {"insert": n_keys, "lookup": n_keys, "delete": dk.numel(), "mixed": mixed_ops}
    scores = {kind: {var: n_ops[kind] / (m * 1e-3) / 1e6 for var, m in ms[kind].items()} for kind in kinds}
    pick = {kind: int(_pick(scores[kind], 0)) for kind in kinds}
    tuning = H.probe_tuning(*(pick[kind] for kind in kinds))
    # the grid cap, scored on the whole bulk step with the chosen variants
    step_ops = 2 * n_keys + dk.numel()
    gscores = {}
    for grid in grids:
        got = measure(tuning, grid)
        _progress(f"probe grid {grid}: " + ", ".join(f"{kk} {x:.3f} ms" for kk, x in got.items()))
        gscores[grid] = step_ops / ((got["insert"] + got["lookup"] + got["delete"]) * 1e-3) / 1e6
    grid = int(_pick(gscores, 0))
    return {"probe_tuning": int(tuning), "probe_grid": grid,
            "variants": {kind: H.PROBE_VARIANTS[pick[kind]] for kind in kinds},
            "scores_mops": {kind: {str(var): round(x, 1) for var, x in scores[kind].items()} for kind in kinds},
            "grid_scores_mops": {str(g): round(x, 1) for g, x in gscores.items()}}


def tune_resize_k(n_keys: int = 1 << 22, batch: int = 1 << 18, reps: int = 3,
                  candidates=(64, 256, 1024, 4096)) -> dict:
    import torch
    ks = wl.KeyStream(13)
    keys = torch.from_numpy(ks.range(0, n_keys)).cuda()
    vals = torch.from_numpy(wl.values_for(keys.cpu().numpy())).cuda()
    scores = {}
    max_b = 1
    while max_b * 16 * 0.9 < n_keys * 1.1:
        max_b *= 2
    for K in candidates:
        t = H.Table(1024, addressing=H.HIVE_LINEAR, max_buckets=max_b, pre_expand=1, post_policy=1,
                    resize_k=K, max_batch=batch)

        def step():
            for b in range(0, n_keys, batch):
                t.insert(keys[b:b + batch], vals[b:b + batch], flags=H.HIVE_UNIQUE)
            for b in range(0, int(n_keys * 0.9), batch):
                H.hive_delete_batch(t.h, keys[b:min(b + batch, int(n_keys * 0.9))], None, H.HIVE_UNIQUE)
        ms = _timed(step, reps, prep=t.clear)
        scores[K] = 1.9 * n_keys / (ms * 1e-3) / 1e6
        t.close()
    best = _pick(scores, 1024) if 1024 in scores else max(scores, key=scores.get)
    return {"resize_k": int(best), "scores_mops": {str(k): round(x, 1) for k, x in scores.items()}}


def tune_executor_blocks(n_batches: int = 256, batch: int = 1 << 12, reps: int = 3) -> dict:
    import torch
    universe, nb = 1 << 20, 1 << 16
    ks = wl.KeyStream(14)
    pre = ks.range(0, int(0.8 * nb * 16))
    batches = [wl.mixed_batch(14, b, batch, universe, zipf_s=None, stream=ks) for b in range(n_batches)]
    dev = [tuple(torch.from_numpy(x[f]).cuda() for f in ("ops", "keys", "vals")) for x in batches]
    vo = torch.empty(batch, dtype=torch.uint32, device="cuda")
    fo = torch.empty(batch, dtype=torch.uint8, device="cuda")
    pk, pv = torch.from_numpy(pre).cuda(), torch.from_numpy(wl.values_for(pre)).cuda()
    t = H.Table(nb, max_batch=batch)
    scores = {}
    for bpc in (1, 2, 3, 0):
        d = H.hive_drain_create(16, bpc, n_batches, 4, 0)

        def prefill():
            t.clear()
            t.insert(pk, pv, flags=H.HIVE_UNIQUE)

        def step():
            for o, k, v in dev:
                H.hive_drain_submit(d, t.h, H.HIVE_OP_MIXED, k, v, o, vo, fo)
            H.hive_drain_launch(d, 0)
        ms = _timed(step, reps, prep=prefill)
        scores[bpc] = n_batches * batch / (ms * 1e-3) / 1e6
        H.hive_drain_destroy(d)
    t.close()
    best = _pick(scores, 1)
    return {"blocks_per_cu": int(best), "scores_mops": {str(k): round(x, 1) for k, x in scores.items()}}


def _progress(msg: str) -> None:
    print(f"[autotune] {msg}", file=sys.stderr, flush=True)


def tune(workload: str = "all", reps: int = 10, save: bool = True) -> dict:
    """Run the tuners a workload needs and cache the winners."""
    t0 = time.time()
    res = {}
    if workload in ("all", "bulk", "probe"):
        res["bulk"] = tune_bucket_width(reps=reps)
        _progress(f"bucket width: {res['bulk']}")
        res["probe"] = tune_probe_both(reps=reps)
        _progress(f"probe_both: {res['probe']}")
        if res["probe"]["probe_both"] == 0:  # the variants exist for second-after-miss probing
            res["probe_kernel"] = tune_probe_kernel(reps=max(3, reps // 2))
            _progress(f"probe kernel: {res['probe_kernel']}")
    if workload in ("all", "resize", "mixed"):
        res["resize"] = tune_resize_k(reps=reps)
        _progress(f"resize: {res['resize']}")
    if workload in ("all", "served", "mixed"):
        res["executor"] = tune_executor_blocks(reps=reps)
        _progress(f"executor: {res['executor']}")
    res["seconds"] = round(time.time() - t0, 1)
    if save:
        path = cache_path()
        os.makedirs(os.path.dirname(path), exist_ok=True)
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        cache.setdefault(gpu_arch(), {}).update({k: v for k, v in res.items() if k != "seconds"})
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return res


def shipped_path(arch: str) -> str:
    return os.path.join(SHIPPED_DIR, f"tuned_{arch}.json")


def load(section: str) -> dict | None:
    """Winners of one tuner section for this GPU: this machine's cache, else
    the values shipped for its architecture, else None."""
    arch = gpu_arch()
    for path in (cache_path(), shipped_path(arch)):
        try:
            got = json.load(open(path)).get(arch, {}).get(section)
        except (OSError, ValueError):
            continue
        if got:
            return got
    return None


if __name__ == "__main__":
    import sys
    print(json.dumps(tune(sys.argv[1] if len(sys.argv) > 1 else "all"), indent=1))
