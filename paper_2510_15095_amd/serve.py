"""Serving loop: uneven batches against many device-resident tables.

Requests (mixed insert/delete/lookup batches) arrive over time, each aimed at
one of many tables.  The server admits a request when a slot is free and its
table has room for the request's inserts inside the table's HBM reservation
(its bucket arena, resize headroom included), then runs it

* on the persistent executor (`hive_drain_*`): one resident grid, launched
  once, takes each request as it is admitted (continuous batching: requests
  on different tables overlap on the device, no launch per request); or
* with plain per-request launches (`hive_mixed_batch`) spread over a pool of
  streams (a table always maps to the same stream, so its requests stay in
  order).

It records each request's latency from arrival to the moment its results
are visible on the host, and the aggregate operation rate.  Everything here
is host logic; all table work runs in the HIP kernels behind the C ABI.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass

import numpy as np

from . import workload as wl


def _binding():
    """The C-ABI binding, imported on first use (request generation needs
    neither it nor the GPU)."""
    from . import hive
    return hive

BYTES_PER_BUCKET = 128  # 16 slots x 8 B


@dataclass
class TableSpec:
    tid: int
    n_keys: int     # keys loaded before serving
    universe: int   # key universe of its requests (about 50% of uniform keys hit)
    buckets: int    # initial buckets
    arena: int      # reserved buckets (growth headroom included)
    seed: int


def make_specs(n_tables: int, seed: int, log2_min: float = 12, log2_max: float = 24, load: float = 0.85,
               headroom: float = 1.25) -> list[TableSpec]:
    """Table sizes log-uniform in [2^log2_min, 2^log2_max] keys, created at
    `load`, each reserving `headroom` x its initial buckets."""
    rng = np.random.default_rng(wl.batch_seed(seed, 0x7AB))
    specs = []
    for t in range(n_tables):
        n = int(2.0 ** rng.uniform(log2_min, log2_max))
        nb = max(1, math.ceil(n / (load * 16)))
        specs.append(TableSpec(t, n, 2 * n, nb, max(nb + 1, math.ceil(nb * headroom)), seed * 1000 + t))
    return specs


def footprint_bytes(specs) -> int:
    return sum(s.arena for s in specs) * BYTES_PER_BUCKET


@dataclass
class Request:
    rid: int
    table: int
    arrival: float   # seconds after the start
    n: int
    n_ins: int
    ops: np.ndarray
    keys: np.ndarray
    vals: np.ndarray


def make_requests(specs, n_req: int, seed: int, rate: float, log2_max_size: float = 16):
    """Poisson arrivals at `rate` requests/s (rate <= 0: all at time 0);
    sizes floor(2^U(0, log2_max_size)), at most the table's initial key count;
    50% lookup / 25% insert / 25% delete; uniform or Zipf(0.99) keys by a
    per-request coin; tables uniform.  Request r on table t is mixed batch r
    of t's seed over t's key universe (the native generator, many requests
    at once)."""
    rng = np.random.default_rng(wl.batch_seed(seed, 0x5E5))
    tables = rng.integers(0, len(specs), n_req)
    sizes = np.floor(2.0 ** rng.uniform(0, log2_max_size, n_req)).astype(np.int64)
    zipf = rng.random(n_req) < 0.5
    gaps = rng.exponential(1.0 / rate, n_req) if rate > 0 else np.zeros(n_req)
    arrivals = np.cumsum(gaps) - (gaps[0] if n_req else 0)
    sizes = np.minimum(sizes, [specs[t].n_keys for t in tables])
    streams = {}
    jobs = []
    for r in range(n_req):
        sp = specs[tables[r]]
        if sp.seed not in streams:
            streams[sp.seed] = wl.KeyStream(sp.seed)
        jobs.append(dict(seed=sp.seed, batch=r, n_ops=int(sizes[r]), universe=sp.universe, frac_insert=0.25,
                         frac_delete=0.25, zipf_s=0.99 if zipf[r] else None, stream=streams[sp.seed],
                         value_salt=r + 1))
    gen = wl.mixed_batches(jobs)
    out = []
    for r, mb in enumerate(gen):
        out.append(Request(r, int(tables[r]), float(arrivals[r]), int(sizes[r]),
                           int((mb["ops"] == wl.OP_INSERT).sum()), mb["ops"], mb["keys"], mb["vals"]))
    return out


class Server:
    """Owns the tables (created and loaded once) and runs request streams.

    blocks_per_cu: resident blocks per compute unit of the persistent
    executor.  One is the default: small requests on many tables are bound
    by the handoffs between phases, and every block's agent-scope acquire
    invalidates its XCD's L2, so fewer blocks serve faster (3,000 requests on
    256 tables: 583 Mops/s at one block per CU against 418 at full
    occupancy)."""

    def __init__(self, specs, budget_bytes: int, max_request: int, ring: int = 1024, streams: int = 8,
                 blocks_per_cu: int = 1):
        import torch
        H = _binding()
        self.specs = specs
        need = footprint_bytes(specs)
        if need > budget_bytes:
            raise ValueError(f"tables need {need} B of buckets, budget is {budget_bytes} B")
        self.budget = budget_bytes
        self.ring = ring
        self.blocks_per_cu = blocks_per_cu
        self.max_request = max_request
        self.tables = []
        for s in specs:
            self.tables.append(H.Table(s.buckets, addressing=H.HIVE_LINEAR, max_buckets=s.arena, pre_expand=1,
                                       lf_expand_pct=90, max_batch=max_request))
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.live_host = torch.zeros(len(specs), dtype=torch.int64).pin_memory()

    def load(self):
        """Insert each table's initial keys (indices 0..n-1 of its stream)."""
        import torch
        H = _binding()
        for s, t in zip(self.specs, self.tables):
            t.clear()
            ks = wl.KeyStream(s.seed)
            keys = ks.range(0, s.n_keys)
            t.insert(torch.from_numpy(keys).cuda(), torch.from_numpy(wl.values_for(keys)).cuda(),
                     flags=H.HIVE_UNIQUE)
        torch.cuda.synchronize()
        self.live = [s.n_keys for s in self.specs]

    def capacity(self, tid: int) -> int:
        """Keys table `tid` may hold inside its reservation (90% of its arena)."""
        return int(0.9 * self.specs[tid].arena * 16)

    def run(self, requests, mode: str, outputs: bool = False, timeout_s: float = 120.0) -> dict:
        """Serve `requests` (device copies made beforehand) and return latency
        and throughput figures; with outputs=True also the per-request results."""
        import torch
        H = _binding()
        dev = [(torch.from_numpy(r.ops).cuda(), torch.from_numpy(r.keys).cuda(), torch.from_numpy(r.vals).cuda())
               for r in requests]
        vout = [torch.empty(r.n, dtype=torch.uint32, device="cuda") for r in requests]
        fout = [torch.empty(r.n, dtype=torch.uint8, device="cuda") for r in requests]
        torch.cuda.synchronize()
        n = len(requests)
        done_at = np.full(n, np.nan)
        admitted_at = np.full(n, np.nan)
        inflight_ins = [0] * len(self.specs)
        live = list(self.live)
        pending = []       # arrived, not yet admitted (FIFO)
        inflight = {}      # rid -> completion handle (persistent: ticket)
        nxt = 0
        deferred = 0
        if mode == "persistent":
            drain = H.hive_drain_create(16, self.blocks_per_cu, self.ring, len(self.specs), 0)
            side = torch.cuda.Stream()
            H.hive_drain_launch(drain, 1, side)
            # a ticket's result stays readable until its ring slot is reused,
            # i.e. until `ring` later submissions: keep new tickets within
            # `ring` of the oldest unread one
            unread = collections.deque()
            read = set()
            n_submitted = 0
        elif mode == "plain":
            # per stream, requests complete in submission order: a turn checks
            # only the oldest event of each stream
            fifo = [collections.deque() for _ in self.streams]
            live_pinned = torch.zeros(n, dtype=torch.int64).pin_memory()
        else:
            raise ValueError(mode)
        t0 = time.perf_counter()
        try:
            while nxt < n or pending or inflight:
                now = time.perf_counter() - t0
                if now > timeout_s:
                    raise TimeoutError(f"{mode}: {len(inflight)} requests still in flight after {timeout_s} s")
                while nxt < n and requests[nxt].arrival <= now:
                    pending.append(nxt)
                    nxt += 1
                # admit in arrival order while slots and table room allow
                while pending and len(inflight) < self.ring:
                    r = requests[pending[0]]
                    if live[r.table] + inflight_ins[r.table] + r.n_ins > self.capacity(r.table):
                        if not inflight:
                            raise RuntimeError(f"request {r.rid} can never fit table {r.table}")
                        deferred += 1
                        break
                    o_, k_, v_ = dev[r.rid]
                    h = self.tables[r.table].h
                    if mode == "persistent":
                        while unread and unread[0] in read:
                            read.discard(unread.popleft())
                        if unread and n_submitted - unread[0] >= self.ring:
                            break
                        tk = H.hive_drain_submit(drain, h, H.HIVE_OP_MIXED, k_, v_, o_, vout[r.rid], fout[r.rid])
                        if tk is None:
                            break
                        n_submitted += 1
                        unread.append(tk)
                        inflight[r.rid] = tk
                    else:
                        si = r.table % len(self.streams)
                        st = self.streams[si]
                        H.hive_mixed_batch(h, o_, k_, v_, vout[r.rid], fout[r.rid], stream=st)
                        H.hive_live_async(h, live_pinned.data_ptr() + 8 * r.rid, stream=st)
                        ev = torch.cuda.Event()
                        ev.record(st)
                        fifo[si].append((r.rid, ev))
                        inflight[r.rid] = r.rid
                    admitted_at[r.rid] = time.perf_counter() - t0
                    inflight_ins[r.table] += r.n_ins
                    pending.pop(0)
                # completions: one call for every ticket in flight, or the
                # heads of the stream queues
                finished = []
                if mode == "persistent" and inflight:
                    rids = list(inflight)
                    ok, lv = H.hive_drain_results(drain, [inflight[i] for i in rids])
                    for j in np.flatnonzero(ok):
                        read.add(inflight[rids[j]])
                        finished.append((rids[j], int(lv[j])))
                elif mode == "plain":
                    for q in fifo:
                        while q and q[0][1].query():
                            rid = q.popleft()[0]
                            finished.append((rid, int(live_pinned[rid])))
                t_done = time.perf_counter() - t0
                for rid, lv in finished:
                    r = requests[rid]
                    done_at[rid] = t_done
                    inflight_ins[r.table] -= r.n_ins
                    live[r.table] = lv
                    del inflight[rid]
        finally:
            if mode == "persistent":
                H.hive_drain_stop(drain, side)
                H.hive_drain_destroy(drain)
        torch.cuda.synchronize()
        self.live = live
        arrival = np.array([r.arrival for r in requests])
        lat = (done_at - arrival) * 1e3
        total_ops = sum(r.n for r in requests)
        span = np.nanmax(done_at) - arrival.min()
        out = {
            "mode": mode,
            "requests": n,
            "ops": int(total_ops),
            "mops": total_ops / span / 1e6,
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()),
            "deferred_admissions": deferred,
            "span_s": float(span),
        }
        if outputs:
            out["results"] = [(vout[i].cpu().numpy(), fout[i].cpu().numpy()) for i in range(n)]
        return out

    def run_alone(self, requests):
        """Each request by itself, in submission order, one at a time: the
        reference for "the same result alone and in the mix"."""
        import torch
        res = []
        for r in requests:
            t = self.tables[r.table]
            v, f = t.mixed(torch.from_numpy(r.ops).cuda(), torch.from_numpy(r.keys).cuda(),
                           torch.from_numpy(r.vals).cuda())
            torch.cuda.synchronize()
            res.append((v.cpu().numpy(), f.cpu().numpy()))
        return res

    def close(self):
        for t in self.tables:
            t.close()
        self.tables = []

