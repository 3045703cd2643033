"""Continuous-batching search server over a resident bank (the serving path).

A resident bank is indexed once and its index stays in HBM.  Query banks
(requests) arrive over time.  The server keeps up to ``slots`` searches in
flight, each on its own HIP stream (default priority) with device and pinned
host buffers allocated once, so admission is by memory: a request joins the
batch being formed for a free slot while the batch's query sequences, padded
codes and expected hits fit that slot's buffers.  A batch is the concatenation
of its requests' query banks (one padded bank); the library searches it
against the resident index with no host round trip (``plast_search_enqueue``),
and its matches (hits that pass the gapped filter, with both scores) are split
back per request by query sequence id.  Searches of different slots overlap on
the device.  A batch whose hits overflow its slot (``PLAST_E_CAPACITY``) is
split in two and requeued at the head of the queue.

Every pair (query occurrence, resident occurrence) is scored independently,
so a request's matches do not depend on the other requests of its batch: the
tests check that each result is identical alone and in the mix.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np
import torch

from . import binding as B
from . import params as P

PAD_LEN = B.PAD_LEN
PAD_CODE = B.PAD_CODE


@dataclasses.dataclass
class Request:
    rid: int
    codes: np.ndarray        # padded layout, uint8
    seq_start: np.ndarray    # int64[n + 1]
    arrival: float = 0.0     # seconds after the start of the run
    done: float = -1.0       # completion time, same clock
    n_ext: int = 0           # pairs scored for this request (its share of the batch)
    matches: np.ndarray = None  # int32[m, 6]: seq1 (request-local), pos1, seq2, pos2, score, gscore
    batch_size: int = 0      # requests in the batch that served it

    @property
    def n_seqs(self):
        return int(self.seq_start.shape[0] - 1)

    @property
    def n_padded(self):
        return int(self.codes.shape[0])


def merge(reqs):
    """One padded bank from several: the runs between banks are shared.
    Returns codes, seq_start, and the first merged sequence id of each bank."""
    parts, starts, first = [reqs[0].codes], [reqs[0].seq_start[:-1]], [0]
    off, nseq = reqs[0].n_padded - PAD_LEN, reqs[0].n_seqs
    for r in reqs[1:]:
        parts.append(r.codes[PAD_LEN:])
        starts.append(r.seq_start[:-1] + off)
        first.append(nseq)
        off += r.n_padded - PAD_LEN
        nseq += r.n_seqs
    codes = np.concatenate(parts)
    seq_start = np.concatenate(starts + [np.array([codes.shape[0]], dtype=np.int64)])
    return codes, seq_start, first


class Resident:
    """The resident bank and its index on the device."""

    def __init__(self, codes, seq_start, device="cuda"):
        self.codes_t = torch.from_numpy(np.ascontiguousarray(codes, dtype=np.uint8)).to(device)
        self.starts_t = torch.from_numpy(np.ascontiguousarray(seq_start, dtype=np.int64)).to(device)
        self.index = B.build_index(self.codes_t, self.starts_t)
        key_off = self.index.key_off().cpu().numpy()
        self.n2 = np.diff(key_off).astype(np.int64)
        n_words = max(1, int(key_off[-1]))
        # expected candidate pairs per query word, with the resident bank's own key
        # frequencies as the query's: sum_k n2(k)^2 / N2
        self.ext_per_word = float((self.n2.astype(np.float64) ** 2).sum() / n_words)

    @property
    def view(self):
        return self.index.view

    def items_bound(self, max_words, tuning):
        """Upper bound of the work-list length for a query of at most max_words
        words: sum_k ceil(n1/32) ceil(n2/W) <= (max_words / 32) max_k c_k + sum_k c_k."""
        t = tuning if tuning is not None else B.tuning_default()
        lo, cols = np.asarray(list(t.class_min_n2)), np.asarray(list(t.item_cols))
        cls = np.clip(np.searchsorted(lo, self.n2, side="right") - 1, 0, len(lo) - 1)
        chunks = np.where(self.n2 > 0, (self.n2 + cols[cls] - 1) // cols[cls], 0)
        return int((max_words + 31) // 32 * chunks.max(initial=0) + chunks.sum())


class Slot:
    def __init__(self, resident, max_seqs, max_padded, capacity, tuning, s1, s2):
        self.stream = torch.cuda.Stream()
        max_items = resident.items_bound(max_padded, tuning)
        self.search = B.Searcher(resident.index, max_padded, max_seqs, max_items, capacity, s1, s2, tuning=tuning)
        self.codes_h = torch.empty(max_padded, dtype=torch.uint8, pin_memory=True)
        self.starts_h = torch.empty(max_seqs + 1, dtype=torch.int64, pin_memory=True)
        self.seg_h = torch.empty(max_seqs + 2, dtype=torch.int32, pin_memory=True)
        self.off_h = torch.empty(max_seqs + 2, dtype=torch.int64, pin_memory=True)
        # pinned landing area for matches (larger results fall back to a pageable copy)
        self.matches_h = torch.empty((min(capacity, 1 << 25), 6), dtype=torch.int32, pin_memory=True)
        self.start = torch.cuda.Event(enable_timing=True)
        self.event = torch.cuda.Event(enable_timing=True)
        self.batch = None
        self.first = None


class Server:
    """``slots`` searches in flight; each slot holds a batch of at most
    ``max_seqs`` query sequences, ``max_padded`` codes and ``capacity`` hits."""

    def __init__(self, resident, slots=3, max_seqs=2500, max_padded=2_600_000, capacity=150_000_000,
                 hit_rate=0.002, tuning=None, s1=P.S1, s2=P.S2):
        self.resident = resident
        self.max_seqs, self.max_padded, self.capacity = max_seqs, max_padded, capacity
        self.hit_rate = hit_rate
        self.slots = [Slot(resident, max_seqs, max_padded, capacity, tuning, s1, s2) for _ in range(slots)]
        self.forced = collections.deque()  # batches split after an overflow, served first
        self.batches = 0
        self.splits = 0
        self.total_ext = 0
        self.batch_hits = []  # ungapped hits of every batch served
        # per batch: requests, pairs, hits, matches, device ms (copy-in to compaction), host ms to split
        self.batch_log = []

    def expected_hits(self, r):
        words = max(0, r.n_padded - PAD_LEN * (r.n_seqs + 1))
        return words * self.resident.ext_per_word * self.hit_rate

    def _launch(self, slot, queue):
        if self.forced:
            self._start(slot, self.forced.popleft())
            return
        batch, seqs, padded, hits = [], 0, PAD_LEN, 0.0
        while queue:
            r = queue[0]
            s, p, h = r.n_seqs, r.n_padded - PAD_LEN, self.expected_hits(r)
            if batch and (seqs + s > self.max_seqs or padded + p > self.max_padded or hits + h > 0.6 * self.capacity):
                break
            if not batch and (s > self.max_seqs or p + PAD_LEN > self.max_padded):
                raise ValueError("request %d does not fit a slot (%d sequences, %d codes)" % (r.rid, s, r.n_padded))
            batch.append(queue.popleft())
            seqs, padded, hits = seqs + s, padded + p, hits + h
        self._start(slot, batch)

    def _start(self, slot, batch):
        codes, starts, first = merge(batch)
        n, ns, k = codes.shape[0], starts.shape[0], len(batch)
        slot.codes_h[:n].copy_(torch.from_numpy(codes))
        slot.starts_h[:ns].copy_(torch.from_numpy(starts))
        slot.seg_h[:k].copy_(torch.tensor(first, dtype=torch.int32))
        slot.seg_h[k] = ns - 1
        with torch.cuda.stream(slot.stream):
            slot.start.record(slot.stream)
            slot.search.codes[:n].copy_(slot.codes_h[:n], non_blocking=True)
            slot.search.starts[:ns].copy_(slot.starts_h[:ns], non_blocking=True)
            slot.search.seg_first[:k + 1].copy_(slot.seg_h[:k + 1], non_blocking=True)
        # matches come back grouped by request
        slot.search.enqueue(n, ns - 1, n_seg=k, stream=slot.stream)
        slot.event.record(slot.stream)
        slot.batch, slot.first = batch, first
        self.batches += 1

    def _collect(self, slot, queue, now):
        t_host = time.perf_counter()
        res = slot.search.result(stream=slot.stream)
        gpu_ms = slot.start.elapsed_time(slot.event)
        batch, first = slot.batch, slot.first
        slot.batch = None
        if res["status"] == B.E_CAPACITY and len(batch) > 1:
            half = len(batch) // 2
            self.forced.appendleft(batch[half:])
            self.forced.appendleft(batch[:half])
            self.splits += 1
            return 0
        if res["status"] != B.OK:
            raise B.PlastError(res["status"], "search of batch %s" % [r.rid for r in batch], "")
        self.total_ext += res["n_ext"]
        self.batch_hits.append(res["n_hits"])
        nm, k = res["n_matches"], len(batch)
        slot.off_h[:k + 1].copy_(slot.search.seg_off[:k + 1])
        bounds = slot.off_h[:k + 1].numpy().copy()
        if nm <= slot.matches_h.shape[0]:
            slot.matches_h[:nm].copy_(slot.search.matches[:nm])
            m = slot.matches_h[:nm].numpy().copy()
        else:
            m = slot.search.matches[:nm].cpu().numpy()
        words = np.array([max(0, r.n_padded - PAD_LEN * (r.n_seqs + 1)) for r in batch], dtype=np.float64)
        for j, r in enumerate(batch):
            mr = m[bounds[j]:bounds[j + 1]]
            mr[:, 0] -= first[j]
            r.matches = mr
            r.done = now
            r.batch_size = len(batch)
            r.n_ext = int(round(res["n_ext"] * words[j] / max(1.0, words.sum())))
        self.batch_log.append((len(batch), res["n_ext"], res["n_hits"], res["n_matches"], gpu_ms,
                               1e3 * (time.perf_counter() - t_host)))
        return len(batch)

    def run(self, requests, poll_s=0.0001, progress=None, every_s=10.0):
        """Serve ``requests`` (arrival times relative to the start); returns the
        wall time from the start to the last completion.  ``progress(done, n)``
        is called every ``every_s`` seconds."""
        order = sorted(requests, key=lambda r: r.arrival)
        queue = collections.deque()
        i, done, n = 0, 0, len(order)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_report = every_s
        while done < n:
            now = time.perf_counter() - t0
            if progress is not None and now >= t_report:
                progress(done, n)
                t_report = now + every_s
            while i < n and order[i].arrival <= now:
                queue.append(order[i])
                i += 1
            progressed = False
            for slot in self.slots:
                if slot.batch is not None and slot.event.query():
                    done += self._collect(slot, queue, time.perf_counter() - t0)
                    progressed = True
            for slot in self.slots:
                if slot.batch is None and (queue or self.forced):
                    self._launch(slot, queue)
                    progressed = True
            if not progressed:
                time.sleep(poll_s)
        return time.perf_counter() - t0


def canonical(m):
    """Matches sorted lexicographically (the order inside a result is unspecified)."""
    m = np.asarray(m, dtype=np.int64).reshape(-1, 6)
    return m[np.lexsort(m.T[::-1])] if len(m) else m


def latency_stats(requests):
    lat = np.array([r.done - r.arrival for r in requests], dtype=np.float64) * 1e3
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max())}
