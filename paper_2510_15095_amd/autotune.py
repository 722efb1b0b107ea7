"""Autotuner: the table's tunable sizes, picked by measurement on this GPU.

* bucket width S (16, 32 or 64 slots): a bulk build to 95% load followed by
  lookups (50% hits), scored by operations per second;
* resize step K (pairs per split/merge step): growth of a LINEAR table from
  a small start under pre-batch expansion, then contraction, scored by
  operations per second including the resize work;
* resident blocks per CU of the persistent executor: a queue of small mixed
  batches, scored by operations per second.

Each candidate runs once to warm up and is then timed `reps` times with HIP
events; the median decides.  Winners are cached per (GPU architecture,
workload) in a JSON file ($HIVE_TUNE_CACHE, default
~/.cache/hive_mi355x/tuned.json) and returned by `load()`.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import hive as H
from . import workload as wl

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "hive_mi355x", "tuned.json")


def cache_path() -> str:
    return os.environ.get("HIVE_TUNE_CACHE", DEFAULT_CACHE)


def gpu_arch() -> str:
    import torch
    return getattr(torch.cuda.get_device_properties(0), "gcnArchName", "unknown").split(":")[0]


def _timed(fn, reps: int) -> float:
    """Median milliseconds of fn() over `reps` runs after one warm-up."""
    import torch
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b))
    return float(np.median(out))


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
            t.clear()
            t.insert(k, v, flags=H.HIVE_UNIQUE)
            H.hive_lookup_batch(t.h, q, vo, fo)
        ms = _timed(step, reps)
        scores[S] = 2 * n_keys / (ms * 1e-3) / 1e6
        t.close()
    best = max(scores, key=scores.get)
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
        ms_d = _timed(lambda: H.hive_delete_batch(t.h, dk, None, H.HIVE_UNIQUE), 1)
        scores[pb] = (q.numel() + dk.numel()) / ((ms_l + ms_d) * 1e-3) / 1e6
        t.close()
    best = max(scores, key=scores.get)
    return {"probe_both": int(best), "scores_mops": {str(k): round(x, 1) for k, x in scores.items()}}


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
            t.clear()
            for b in range(0, n_keys, batch):
                t.insert(keys[b:b + batch], vals[b:b + batch], flags=H.HIVE_UNIQUE)
            for b in range(0, int(n_keys * 0.9), batch):
                H.hive_delete_batch(t.h, keys[b:min(b + batch, int(n_keys * 0.9))], None, H.HIVE_UNIQUE)
        ms = _timed(step, reps)
        scores[K] = 1.9 * n_keys / (ms * 1e-3) / 1e6
        t.close()
    best = max(scores, key=scores.get)
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

        def step():
            t.clear()
            t.insert(pk, pv, flags=H.HIVE_UNIQUE)
            for o, k, v in dev:
                H.hive_drain_submit(d, t.h, H.HIVE_OP_MIXED, k, v, o, vo, fo)
            H.hive_drain_launch(d, 0)
        ms = _timed(step, reps)
        scores[bpc] = n_batches * batch / (ms * 1e-3) / 1e6
        H.hive_drain_destroy(d)
    t.close()
    best = max(scores, key=scores.get)
    return {"blocks_per_cu": int(best), "scores_mops": {str(k): round(x, 1) for k, x in scores.items()}}


def tune(workload: str = "all", reps: int = 10, save: bool = True) -> dict:
    """Run the tuners a workload needs and cache the winners."""
    t0 = time.time()
    res = {}
    if workload in ("all", "bulk"):
        res["bulk"] = tune_bucket_width(reps=reps)
        res["probe"] = tune_probe_both(reps=reps)
    if workload in ("all", "resize", "mixed"):
        res["resize"] = tune_resize_k(reps=reps)
    if workload in ("all", "served", "mixed"):
        res["executor"] = tune_executor_blocks(reps=reps)
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


def load(section: str) -> dict | None:
    """Cached winners of one tuner section for this GPU, or None."""
    try:
        return json.load(open(cache_path())).get(gpu_arch(), {}).get(section)
    except (OSError, ValueError):
        return None


if __name__ == "__main__":
    import sys
    print(json.dumps(tune(sys.argv[1] if len(sys.argv) > 1 else "all"), indent=1))
