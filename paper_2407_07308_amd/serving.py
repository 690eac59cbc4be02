"""Continuous-batching server for encrypted comparison requests.

A request carries two encrypted operands as digit planes (one batch of
`groups` ciphertexts per plane, 128 integers per ciphertext group) and asks
for LT, MAX or ARGMAX (the LT bit: 1 where the second operand is larger).  The
server keeps keys resident per ring size, admits arrived requests while the
device-memory estimate of the work in flight stays under a budget, coalesces
admitted requests of one ring size into a single batch (their planes are
concatenated on the device), and launches batched comparisons on every free
stream -- batches of different ring sizes side by side, the oldest waiting
ring size first -- so they overlap on the GPU.  Each batch in flight has a
waiter thread blocked on its completion event (the HIP event wait releases
the interpreter lock), which hands the finished batch to the loop through a
queue; the loop sleeps on that queue until a batch finishes or the next
request arrives, and never polls.  Latency = completion time - arrival time.
Everything the batch computes runs in the library's kernels; this loop only
schedules.
"""
from __future__ import annotations

import collections
import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import BC_ERR_OOM, BC_TUNE_POOL_LIMIT_BYTES, Batch, BoostcomError, Context, Keys


@dataclass
class Request:
    rid: int
    kind: str  # "lt", "max" or "argmax"
    N: int
    groups: int
    arrival: float  # seconds from the start of the run
    a: list = field(default_factory=list)  # digit planes (Batch, count = groups), most significant first
    b: list = field(default_factory=list)
    result: object = None  # (lt Batch slice, max planes or None)
    done_at: float = None


class _InFlight:
    def __init__(self, reqs, event, outs, offsets, bytes_):
        self.reqs, self.event, self.outs, self.offsets, self.bytes = reqs, event, outs, offsets, bytes_


def _concat(planes_per_req, ctx: Context):
    """Concatenate the requests' plane d into one batch per plane."""
    import torch

    nd = len(planes_per_req[0])
    out = []
    for d in range(nd):
        ts = [pl[d].tensor for pl in planes_per_req]
        lv = planes_per_req[0][d].level
        cnt = sum(pl[d].count for pl in planes_per_req)
        out.append(Batch(torch.cat(ts), cnt, lv, 2))
    return out


def _slice(b: Batch, ctx: Context, first: int, n: int) -> Batch:
    w = ctx.ct_words(b.level, b.ncomp)
    return Batch(b.tensor[first * w:(first + n) * w], n, b.level, b.ncomp)


class Server:
    def __init__(self, members: dict, max_batch_groups: int = 64, mem_budget_bytes: int | None = None,
                 streams: int = 2, bytes_per_group: dict | None = None, headroom: float = 0.1):
        """members: {N: (Context, Keys)}.  mem_budget_bytes: device memory the
        batches in flight may use (default: the free device memory less
        `headroom` of the total).  bytes_per_group: {(N, planes): bytes} of one
        group's comparison at its peak; measured on first use of a shape
        otherwise (see _group_bytes)."""
        import torch

        self.members = members
        self.max_batch_groups = max_batch_groups
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        if mem_budget_bytes is None:
            free, total = torch.cuda.mem_get_info()
            mem_budget_bytes = int(free - headroom * total)
        self.budget = mem_budget_bytes
        self.bpg = dict(bytes_per_group or {})
        # Each context's workspace pool may hold its share of the budget (by
        # ciphertext size): blocks of finished batches stay cached for the
        # next ones up to that bound, and the pools together never take the
        # memory the operands and the runtime need.
        words = {N: ctx.ct_words(ctx.nQ - 1) for N, (ctx, _) in members.items()}
        for N, (ctx, _) in members.items():
            ctx.set_tuning(BC_TUNE_POOL_LIMIT_BYTES, max(1, self.budget * words[N] // sum(words.values())))
        self.stats = {"batches": 0, "max_inflight_bytes": 0, "groups": 0}

    def _group_bytes(self, N: int, planes: int) -> int:
        """Peak workspace of one group of an LT + max batch with `planes`
        digit planes: measured once per shape on a 4-group batch of zero
        ciphertexts (the pool, emptied first, then holds exactly the blocks
        the call needed)."""
        import torch

        key = (N, planes)
        if key not in self.bpg:
            ctx, keys = self.members[N]
            G = 4
            torch.cuda.synchronize()
            ctx.trim()
            zero = lambda: [Batch(torch.zeros(G * ctx.ct_words(ctx.nQ - 1), dtype=torch.int64, device="cuda"),
                                  G, ctx.nQ - 1, 2) for _ in range(planes)]
            ctx.compare_max_min(keys, zero(), zero(), True, True, False)
            torch.cuda.synchronize()
            self.bpg[key] = -(-ctx.pool_bytes() // G)
            ctx.trim()
        return self.bpg[key]

    def _release_cached(self):
        import torch

        torch.cuda.synchronize()
        for ctx, _ in self.members.values():
            ctx.trim()
        torch.cuda.empty_cache()

    def _launch(self, reqs, stream_idx):
        import torch

        N = reqs[0].N
        ctx, keys = self.members[N]
        s = self.streams[stream_idx]
        want_max = any(r.kind == "max" for r in reqs)
        for attempt in range(2):
            try:
                with torch.cuda.stream(s):
                    A = _concat([r.a for r in reqs], ctx)
                    B = _concat([r.b for r in reqs], ctx)
                    outs = ctx.compare_max_min(keys, A, B, True, want_max, False)
                    ev = torch.cuda.Event()
                    ev.record(s)
                break
            except (torch.OutOfMemoryError, BoostcomError) as err:
                # device memory held in the caches (the library's workspace
                # blocks of earlier batch shapes, or torch's): wait for the
                # device, give it all back once and retry
                if attempt or (isinstance(err, BoostcomError) and err.code != BC_ERR_OOM):
                    raise
                self.stats["oom_retries"] = self.stats.get("oom_retries", 0) + 1
                self._release_cached()
        offsets, o = [], 0
        for r in reqs:
            offsets.append(o)
            o += r.groups
        self.stats["batches"] += 1
        self.stats["groups"] += o
        # keep the concatenated inputs alive until the batch completes
        return _InFlight(reqs, ev, (outs, A, B), offsets, sum(self._group_bytes(N, len(r.a)) * r.groups for r in reqs))

    def _next_batch(self, ready, used: int, any_inflight: bool):
        """The next admissible batch: requests of one ring size, taken in
        arrival order, ring sizes tried in the order of their oldest waiting
        request; at most max_batch_groups groups and within the memory budget
        (a single request is admitted over budget only when nothing is in
        flight).  Returns (requests, bytes) or None."""
        sizes = []
        for r in ready:
            if r.N not in sizes:
                sizes.append(r.N)
        for N in sizes:
            batch, nbytes, g = [], 0, 0
            for r in ready:
                if r.N != N:
                    continue
                need = self._group_bytes(N, len(r.a)) * r.groups
                if batch and (g + r.groups > self.max_batch_groups or used + nbytes + need > self.budget):
                    break
                if not batch and used + need > self.budget and (any_inflight or nbytes):
                    break  # wait for memory to free up
                batch.append(r)
                nbytes += need
                g += r.groups
            if batch:
                return batch, nbytes
        return None

    def run(self, requests: list, clock=time.perf_counter, progress=None, on_complete=None):
        """Serves `requests` (sorted by arrival) against their arrival times;
        returns them completed, with latencies filled in.  `progress(done,
        total)` is called as batches complete; `on_complete(request)` as each
        request completes (its result set: a caller that hands results on can
        drop them there, so that finished batches free their memory)."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        ready = collections.deque()
        inflight: list[_InFlight] = []
        free = list(range(len(self.streams)))
        finished: queue.Queue = queue.Queue()
        t0 = clock()
        used = 0
        done = 0

        def wait_for(f):
            f.event.synchronize()
            finished.put(f)

        def complete(f):
            nonlocal used, done
            t = clock() - t0
            f.waiter.join()
            (lt, mx, _), _, _ = f.outs
            for r, off in zip(f.reqs, f.offsets):
                ctx = self.members[r.N][0]
                r.result = (_slice(lt, ctx, off, r.groups),
                            [_slice(m, ctx, off, r.groups) for m in mx] if (mx and r.kind == "max") else None)
                r.done_at = t
                if on_complete:
                    on_complete(r)
            used -= f.bytes
            free.append(f.stream)
            inflight.remove(f)
            done += len(f.reqs)
            held = sum(c.pool_bytes() for c, _ in self.members.values())
            self.stats["max_pool_bytes"] = max(self.stats.get("max_pool_bytes", 0), held)
            if progress:
                progress(done, len(requests))

        while pending or ready or inflight:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                ready.append(pending.popleft())
            while True:  # batches that finished meanwhile
                try:
                    complete(finished.get_nowait())
                except queue.Empty:
                    break
            # fill every free stream with an admissible batch
            while ready and free:
                nb = self._next_batch(ready, used, bool(inflight))
                if nb is None:
                    break
                batch, nbytes = nb
                for r in batch:
                    ready.remove(r)
                si = free.pop(0)
                f = self._launch(batch, si)
                f.stream = si
                used += nbytes
                self.stats["max_inflight_bytes"] = max(self.stats["max_inflight_bytes"], used)
                self.stats["max_concurrent_batches"] = max(self.stats.get("max_concurrent_batches", 0),
                                                           len(inflight) + 1)
                f.waiter = threading.Thread(target=wait_for, args=(f,), daemon=True)
                inflight.append(f)
                f.waiter.start()
            # sleep until a batch finishes or the next request arrives
            if pending or inflight:
                timeout = max(0.0, pending[0].arrival - (clock() - t0)) if pending else None
                if inflight:
                    try:
                        complete(finished.get(timeout=timeout))
                    except queue.Empty:
                        pass
                elif timeout:
                    time.sleep(timeout)
        return requests


def latency_summary(reqs):
    lat = np.array([r.done_at - r.arrival for r in reqs])
    span = max(r.done_at for r in reqs) - min(r.arrival for r in reqs)
    return {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "throughput_req_s": len(reqs) / span if span > 0 else None}
