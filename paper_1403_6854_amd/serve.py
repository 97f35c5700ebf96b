"""Continuous-batching scan server over ss_scan_batch.

Scan requests -- iHS over one region, or XPEHH over a pair of populations on
one region -- arrive over time.  The server

  * admits waiting requests first come, first served, while the device memory
    they need (their haplotype matrices, kept resident until the request is
    done, plus workspace and outputs) fits the budget;
  * gathers every request admitted at one admission point into one batch: one
    ss_scan_batch call, whose EHH walks for all regions share one persistent
    launch, enqueued on a free stream;
  * keeps one batch per stream of the backend on the device at once, so
    requests that arrive while others run are admitted as soon as a stream
    and memory free up, and their work overlaps on the GPU;
  * completes each request as soon as its own results are ready: the torch
    backend enqueues a batch as up to two ss_scan_batch calls, the requests
    walked by the register-bitmask kernel (1,024 haplotypes or fewer in the
    walk) first, each followed by an event, so that small requests do not wait
    for the longest walk of a large one; the batch's memory and stream are
    released when its last event has fired;
  * survives backend failures: a batch whose launch or completion raises is
    dropped, its memory released, and its unfinished requests queued again at
    the front to run alone; a request that fails ``max_attempts`` times
    completes with an error entry (``Completion.error``) instead of results.

Latency of a request is completion time minus arrival time.  The per-request
results are exactly those of the request run alone (every walk kernel gives the
same answer, and standardization is per region).

``run_back_to_back`` is the reference point: the same requests one at a time in
arrival order, each a plain single-region scan waited for before the next.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, List, Optional

import numpy as np


@dataclasses.dataclass
class ServeRequest:
    rid: int
    arrival_s: float
    kind: str                    # "ihs" or "xpehh"
    nbytes: int                  # device memory held while admitted
    make: Callable               # () -> (HapMat a, HapMat b or None), enqueued on the current stream
    n_sites: int = 0
    work: float = 0.0            # estimated walk work (request_work); 0 = unknown


@dataclasses.dataclass
class Completion:
    rid: int
    arrival_s: float
    admit_s: float
    finish_s: float
    batch: int
    out: Optional[dict] = None
    error: Optional[str] = None   # set when the request failed every attempt

    @property
    def latency_s(self) -> float:
        return self.finish_s - self.arrival_s


def words(n: int) -> int:
    return (int(n) + 63) // 64


def request_bytes(kind: str, n_a: int, n_b: int, n_sites: int, steps: bool = False) -> int:
    """Device memory of one request while it is admitted (an upper estimate):
    0/1 alleles during packing, packed matrices, positions, haplotype-major
    copies, per-site workspace and outputs."""
    m = int(n_sites)
    n_tot = n_a + (n_b if kind == "xpehh" else 0)
    alleles = m * n_tot
    bits = 8 * m * (words(n_a) + (words(n_b) if kind == "xpehh" else 0))
    hapmajor = 8 * n_tot * (m // 64 + 3)
    per_site = 16 + 1 + 4 + 32 + 16 + 16 + 8 + 8 + 8 + 8   # positions, flags, bins, walk records, segments, redo
    outputs = m * (5 * 8 + 1 + (16 if steps else 0))
    return alleles + bits + hapmajor + per_site * m + outputs + (1 << 16)


def request_work(kind: str, n_a: int, n_b: int, n_sites: int) -> float:
    """Estimated walk work of a request: sites times haplotypes walked (a
    proxy for the marker steps of its walks times the haplotypes each
    refines)."""
    return float(n_sites) * float(n_a + (n_b if kind == "xpehh" else 0))


# Haplotypes in a walk up to which the register-bitmask kernel takes a request.
SMALL_WALK_HAPS = 1024


class TorchBackend:
    """Runs batches through ss_scan_batch on a pool of streams.  A batch is
    enqueued as one ss_scan_batch call for the requests of at most 1,024
    haplotypes in the walk (the bitmask kernel, one launch per scan), then one
    for the others (one persistent launch), each followed by an event; the
    requests of a call are complete when its event has fired."""

    def __init__(self, n_streams: int = 2, params=None, keep=("status",), steps: bool = False):
        import torch
        import paper_1403_6854_amd as ss
        self.ss = ss
        self.torch = torch
        self.params = params
        self.keep = keep
        self.steps = steps
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.free = list(range(n_streams))

    def slots(self) -> int:
        return len(self.free)

    def launch(self, reqs: List[ServeRequest]):
        torch, ss = self.torch, self.ss
        si = self.free.pop()
        s = self.streams[si]
        try:
            with torch.cuda.stream(s):
                srs = []
                for r in reqs:
                    a, b = r.make()
                    sr = ss.ScanRequest(a, b)
                    ss.alloc_outputs(sr, steps=self.steps)
                    srs.append(sr)
                small = [i for i, sr in enumerate(srs)
                         if sr.a.n_haps + (sr.b.n_haps if sr.b is not None else 0) <= SMALL_WALK_HAPS]
                in_small = set(small)
                large = [i for i in range(len(srs)) if i not in in_small]
                groups = []
                for pos in (small, large):
                    if not pos:
                        continue
                    ss.scan_batch([srs[i] for i in pos], self.params, stream=s, validate=False)
                    ev = torch.cuda.Event()
                    ev.record(s)
                    groups.append([pos, ev, False])
        except Exception:
            self.free.append(si)
            raise
        return (si, groups, srs)

    def _out(self, sr) -> dict:
        return {k: v for k, v in sr.out.items() if self.keep is None or k in self.keep}

    def partial(self, handle):
        """Members whose call's event has fired since the last query:
        [(position in the batch, outputs)]."""
        _, groups, srs = handle
        got = []
        for g in groups:
            if not g[2] and g[1].query():
                g[2] = True
                got.extend((i, self._out(srs[i])) for i in g[0])
        return got

    def done(self, handle) -> bool:
        return handle[1][-1][1].query()

    def retire(self, handle) -> List[dict]:
        si, _, srs = handle
        self.free.append(si)
        return [self._out(sr) for sr in srs]

    def release(self, handle):
        """Gives back the stream of a batch the server abandons."""
        if handle[1]:
            handle[1][-1][1].synchronize()   # its work may still be running
        self.free.append(handle[0])


class Server:
    """Admission by memory budget, continuous batching, completion polling.

    ``backend`` provides slots() (free streams), launch(list) -> handle,
    done(handle) -> bool and retire(handle) -> per-request outputs, and
    optionally partial(handle) -> [(position, outputs)] for members complete
    before the whole batch, and release(handle) to give back the stream of a
    batch dropped after an error; ``clock`` and ``sleep`` are injectable so the
    policy can be exercised off the GPU.

    ``work_ratio`` > 0 closes a batch at the first waiting request whose
    estimated work differs from the batch's first request's by more than
    that factor (first come, first served is kept: that request opens the
    next batch), so that small requests do not wait for the longest walk of
    a large one in the same batch.
    """

    def __init__(self, backend, budget_bytes: int, max_batch: int = 64,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, poll_s: float = 1e-4,
                 work_ratio: float = 0.0, max_attempts: int = 2):
        if budget_bytes <= 0 or max_batch < 1 or max_attempts < 1:
            raise ValueError("budget_bytes, max_batch and max_attempts must be positive")
        self.max_attempts = int(max_attempts)
        self.failures = 0                 # batches dropped after a backend error
        self.errors: List[str] = []
        if work_ratio < 0.0 or (0.0 < work_ratio < 1.0):
            raise ValueError("work_ratio must be 0 or at least 1")
        self.work_ratio = float(work_ratio)
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.clock = clock
        self.sleep = sleep
        self.poll_s = poll_s
        self.peak_bytes = 0
        self.batches = 0
        self.batch_sizes: List[int] = []

    def _apart(self, first: ServeRequest, r: ServeRequest) -> bool:
        if self.work_ratio <= 0.0 or first.work <= 0.0 or r.work <= 0.0:
            return False
        q = r.work / first.work
        return q > self.work_ratio or q * self.work_ratio < 1.0

    def run(self, requests: List[ServeRequest]) -> List[Completion]:
        reqs = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
        t0 = self.clock()
        nxt = 0
        pending = collections.deque()   # (request, alone): alone after a failed attempt
        attempts = collections.Counter()
        inflight = []          # [handle, [(req, admit_s)], bytes, batch id, set of positions done]
        used = 0
        done: List[Completion] = []
        partial = getattr(self.backend, "partial", None)

        def requeue(members, bid, err):
            # a failed attempt: each unfinished request goes back to the front
            # of the queue, to run alone, or completes with the error once it
            # has failed max_attempts times
            self.failures += 1
            self.errors.append(err)
            now_s = self.clock() - t0
            for r, adm in reversed(members):
                attempts[r.rid] += 1
                if attempts[r.rid] >= self.max_attempts:
                    done.append(Completion(r.rid, r.arrival_s, adm, now_s, bid, None, err))
                else:
                    pending.appendleft((r, True))

        def drop(item, err):
            # the batch failed after its launch: release its memory and stream
            nonlocal used
            handle, members, nbytes, bid, got = item
            inflight.remove(item)
            used -= nbytes
            release = getattr(self.backend, "release", None)
            if release is not None:
                try:
                    release(handle)
                except Exception as e:   # the stream is lost; keep serving on the others
                    self.errors.append("release: %r" % (e,))
            requeue([m for pos, m in enumerate(members) if pos not in got], bid, err)

        while nxt < len(reqs) or pending or inflight:
            now = self.clock() - t0
            while nxt < len(reqs) and reqs[nxt].arrival_s <= now:
                pending.append((reqs[nxt], False))
                nxt += 1
            progressed = False
            for item in list(inflight):
                handle, members, nbytes, bid, got = item
                try:
                    if partial is not None:
                        early = partial(handle)
                        if early:
                            fin = self.clock() - t0
                            for pos, o in early:
                                if pos not in got:
                                    got.add(pos)
                                    r, adm = members[pos]
                                    done.append(Completion(r.rid, r.arrival_s, adm, fin, bid, o))
                            progressed = True
                    if self.backend.done(handle):
                        fin = self.clock() - t0
                        outs = self.backend.retire(handle)
                        for pos, ((r, adm), o) in enumerate(zip(members, outs)):
                            if pos not in got:
                                done.append(Completion(r.rid, r.arrival_s, adm, fin, bid, o))
                        used -= nbytes
                        inflight.remove(item)
                        progressed = True
                except Exception as e:
                    drop(item, "batch %d: %r" % (bid, e))
                    progressed = True
            if pending and self.backend.slots() > 0:
                batch, nbytes = [], 0
                while pending and len(batch) < self.max_batch:
                    r, alone = pending[0]
                    if batch and (alone or batch[0][1] or self._apart(batch[0][0], r)):
                        break
                    if used + nbytes + r.nbytes > self.budget:
                        # a request larger than the whole budget runs alone
                        if not (r.nbytes > self.budget and not batch and not inflight):
                            break
                    batch.append(pending.popleft())
                    nbytes += r.nbytes
                if batch:
                    adm = self.clock() - t0
                    bid = self.batches
                    self.batch_sizes.append(len(batch))
                    self.batches += 1
                    progressed = True
                    try:
                        handle = self.backend.launch([r for r, _ in batch])
                    except Exception as e:   # nothing was admitted
                        requeue([(r, adm) for r, _ in batch], bid, "batch %d launch: %r" % (bid, e))
                    else:
                        used += nbytes
                        self.peak_bytes = max(self.peak_bytes, used)
                        inflight.append([handle, [(r, adm) for r, _ in batch], nbytes, bid, set()])
            if not progressed:
                if not inflight and not pending and nxt < len(reqs):
                    wait = reqs[nxt].arrival_s - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(min(wait, 0.01))
                else:
                    self.sleep(self.poll_s)
        return done


def run_back_to_back(requests: List[ServeRequest], run_one: Callable,
                     clock: Callable[[], float] = time.perf_counter,
                     sleep: Callable[[float], None] = time.sleep) -> List[Completion]:
    """Each request in arrival order, alone: ``run_one(request)`` runs the
    scan and returns when its results are complete."""
    reqs = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
    t0 = clock()
    out = []
    for i, r in enumerate(reqs):
        while clock() - t0 < r.arrival_s:
            sleep(min(0.01, r.arrival_s - (clock() - t0)))
        adm = clock() - t0
        o = run_one(r)
        out.append(Completion(r.rid, r.arrival_s, adm, clock() - t0, i, o))
    return out


def summarize(done: List[Completion]) -> dict:
    lat = np.array([c.latency_s for c in done])
    if lat.size == 0:
        return {"requests": 0}
    first = min(c.arrival_s for c in done)
    last = max(c.finish_s for c in done)
    return {
        "requests": int(lat.size),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "makespan_s": float(last - first),
        "requests_per_s": float(lat.size / max(last - first, 1e-9)),
    }
