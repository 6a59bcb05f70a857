"""Continuous-batching serving loop over the risrt C ABI.

A query names a *deployment* (scene, RIS, receiver grid, reflection order,
transmitter) and carries a batch of RIS configurations Gamma [M x C]; its
answer is the received power map P [R x C] (eqs. (9)-(10)).

* The scene's BVH and the deployment's channel (H, E_env) stay on the device
  in an LRU cache charged to the context's memory budget; a query whose
  channel is missing first traces it (every other query keeps running).
* A scheduler admits queued work into `n_slots` slots, each with its own HIP
  stream, as slots and memory free up (continuous batching: requests that
  arrive while others run join at the next free slot).
* Queued queries for the same deployment and precision are merged into one
  RIS sum: their configuration columns are concatenated, summed in one
  matrix-core launch, and split again.  Every output column depends only on
  its own column of Gamma, so a result is bit-identical alone and in a mix.
* A query that does not fit the budget waits; one that cannot fit even alone
  fails with the library's RT_ENOMEM instead of blocking the queue.
* Batches whose channel is not cached (they trace first, for milliseconds)
  hold at most n_slots - 1 slots; queued cache hits may pass queued misses,
  so a hit never waits behind traces occupying every slot.
* Latency = completion time - submission time (host clock), per query, kept
  apart for cache hits and misses (a miss: the deployment's channel was not
  cached when its batch started, so the batch traced it or waited for the
  slot that did).
* With ``log`` (a path or a text stream) every answered query adds one JSON
  line: latency, queueing time, columns, its batch, hit or miss, the segments
  its batch traced and the bytes of its answer.
* A channel can be exported to an ``.npz`` file and imported into another
  server's cache (a warm start: the deployment is then served without
  tracing).
"""
from __future__ import annotations

import collections
import dataclasses
import hashlib
import io
import json
import queue
import threading
import time
from concurrent.futures import Future
from typing import Dict, List, Optional

import numpy as np

from . import risrt


@dataclasses.dataclass
class Deployment:
    key: str
    scene_key: str
    ris_key: str
    tx_pos: np.ndarray
    tx_axis: np.ndarray
    tx_power_w: float
    tx_gain: float
    tx_pattern: int
    tx_param: float
    rx_pos: np.ndarray
    rx_axis: np.ndarray
    rx_gain: float
    rx_pattern: int
    rx_param: float
    freq_hz: float
    order: int
    n_rays: int


@dataclasses.dataclass
class _Query:
    qid: int
    dep: str
    gamma: np.ndarray          # complex64 [M, C]
    real: bool                 # Gamma has no imaginary part (checked at submission)
    scale: float
    precision: int
    t_submit: float
    future: Future


def deployment_from_problem(key: str, scene_key: str, ris_key: str, prob) -> Deployment:
    return Deployment(key, scene_key, ris_key, prob.tx_pos, prob.tx_ant.axis, prob.tx_power_w, prob.tx_ant.gain,
                      prob.tx_ant.pattern, prob.tx_ant.param, prob.rx_pos, prob.rx_ant.axis, prob.rx_ant.gain,
                      prob.rx_ant.pattern, prob.rx_ant.param, prob.freq, prob.order, prob.n_rays)


class Server:
    def __init__(self, ctx: risrt.Context, n_slots: int = 4, max_cols: int = 4096, cache_frac: float = 0.6,
                 cache_bytes: Optional[int] = None, log=None):
        import torch
        # per-query JSON lines: a path (appended to) or an open text stream
        self._log_own = isinstance(log, str)
        self._log: Optional[io.TextIOBase] = open(log, "a") if self._log_own else log
        self._log_lock = threading.Lock()
        self.ctx = ctx
        self.n_slots = n_slots
        self.max_cols = max_cols
        self._torch = torch
        self._budget = ctx.mem_info()[1]
        # channels are evicted (least recently used first) beyond this many bytes
        self._cache_limit = int(cache_bytes) if cache_bytes is not None else int(cache_frac * self._budget)
        self._scenes_host: Dict[str, object] = {}
        self._ris_host: Dict[str, object] = {}
        self._deps: Dict[str, Deployment] = {}
        self._scene_h: Dict[str, int] = {}
        self._ris_h: Dict[str, int] = {}
        self._chan: "collections.OrderedDict[str, int]" = collections.OrderedDict()
        self._chan_bytes: Dict[str, int] = {}
        self._in_use: Dict[str, int] = collections.Counter()
        self._key_locks: Dict[str, threading.Lock] = collections.defaultdict(threading.Lock)
        self._lock = threading.Condition()
        self._queue: List[_Query] = []
        self._free_slots = list(range(n_slots))
        torch.cuda.init()   # creating a stream does not initialise torch's device state by itself
        self._streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self._reserved = 0
        self._misses_running = 0   # admitted batches whose channel was not cached at admission
        self._next_id = 0
        self._running = True
        self.latencies: List[float] = []
        self.missed: List[bool] = []   # per latency: the query's batch found no cached channel
        self.n_traces = 0
        self.n_evictions = 0
        self.n_batches = 0
        self.n_cols = 0
        self.cache_hits = 0
        self.admission_waits = 0
        self._errors = 0
        self._work = [queue.Queue() for _ in range(n_slots)]
        self._workers = [threading.Thread(target=self._worker, args=(i,), name="risrt-slot%d" % i, daemon=True)
                         for i in range(n_slots)]
        for t in self._workers:
            t.start()
        self._sched = threading.Thread(target=self._scheduler, name="risrt-scheduler", daemon=True)
        self._sched.start()

    # ---------------- registration ----------------
    def add_scene(self, key: str, scene) -> None:
        self._scenes_host[key] = scene

    def add_ris(self, key: str, ris) -> None:
        self._ris_host[key] = ris

    def add_deployment(self, dep: Deployment) -> None:
        self._deps[dep.key] = dep

    # ---------------- client API ----------------
    def submit(self, dep_key: str, gamma: np.ndarray, scale: float = 1.0,
               precision: int = risrt.PREC_MFMA_BF16X2) -> Future:
        if dep_key not in self._deps:
            raise KeyError(dep_key)
        f: Future = Future()
        g = np.ascontiguousarray(gamma, np.complex64)
        real = not np.any(g.imag)   # on the caller's thread, off the device workers' path
        with self._lock:
            q = _Query(self._next_id, dep_key, g, real, float(scale), int(precision), time.perf_counter(), f)
            self._next_id += 1
            self._queue.append(q)
            self._lock.notify_all()
        return f

    def drain(self, timeout: Optional[float] = None) -> None:
        t0 = time.perf_counter()
        with self._lock:
            while self._queue or len(self._free_slots) < self.n_slots:
                if timeout is not None and time.perf_counter() - t0 > timeout:
                    raise TimeoutError("serving queue did not drain")
                self._lock.wait(0.05)

    def close(self) -> None:
        self.drain()
        with self._lock:
            self._running = False
            self._lock.notify_all()
        self._sched.join()
        for q in self._work:
            q.put(None)
        for t in self._workers:
            t.join()
        for h in list(self._chan.values()):
            self.ctx.destroy(h)
        for h in list(self._scene_h.values()) + list(self._ris_h.values()):
            self.ctx.destroy(h)
        self._chan.clear()
        self._scene_h.clear()
        self._ris_h.clear()
        if self._log is not None:
            self._log.flush()
            if self._log_own:
                self._log.close()
            self._log = None

    # ---------------- channel export / import ----------------
    def export_channel(self, dep_key: str, path: str) -> str:
        """Write the deployment's channel (traced first if it is not cached)
        to an ``.npz`` file with the deployment's parameters as metadata.
        Returns the path written."""
        dep = self._deps[dep_key]
        stream = self._torch.cuda.Stream()
        ch, _, _ = self._channel(dep, stream)
        try:
            return risrt.channel_save(self.ctx, ch, path, **_dep_meta(dep))
        finally:
            with self._lock:
                self._in_use[dep_key] -= 1

    def import_channel(self, dep_key: str, path: str) -> None:
        """Put a channel file written by export_channel (or
        risrt.channel_save) into the cache as the deployment's channel.  Its R
        and M must be the deployment's; if its metadata names deployment
        parameters, they must be the deployment's too."""
        dep = self._deps[dep_key]
        E, H, meta = risrt.read_channel_file(path)
        M = self._ris_host[dep.ris_key].elems.shape[0]
        if H.shape != (dep.rx_pos.shape[0], M):
            raise ValueError("channel %s is %s, deployment %s needs (%d, %d)"
                             % (path, H.shape, dep_key, dep.rx_pos.shape[0], M))
        mine = _dep_meta(dep)
        for k, v in meta.items():
            if k in mine and mine[k] != v:
                raise ValueError("channel %s was traced for %s = %r, deployment %s has %r"
                                 % (path, k, v, dep_key, mine[k]))
        with self._key_locks["chan:" + dep_key]:
            ch = self.ctx.channel_create(E, H)
            old = None
            with self._lock:
                if self._in_use[dep_key]:
                    self.ctx.destroy(ch)
                    raise RuntimeError("deployment %s has queries in flight" % dep_key)
                old = self._chan.pop(dep_key, None)
                self._chan_bytes.pop(dep_key, None)
                self._chan[dep_key] = ch
                self._chan_bytes[dep_key] = _channel_bytes(*H.shape)
            if old is not None:
                self.ctx.destroy(old)
            self._evict(dep_key)

    def clear_latencies(self) -> None:
        with self._lock:
            self.latencies.clear()
            self.missed.clear()

    def stats(self) -> dict:
        with self._lock:
            lat = np.asarray(self.latencies) * 1e3
            miss = np.asarray(self.missed, bool)

        def pct(x, q):
            return float(np.percentile(x, q)) if x.size else None
        return {"queries": int(lat.size), "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                "mean_ms": float(lat.mean()) if lat.size else None,
                "hits": int((~miss).sum()), "hit_p50_ms": pct(lat[~miss], 50), "hit_p99_ms": pct(lat[~miss], 99),
                "misses": int(miss.sum()), "miss_p50_ms": pct(lat[miss], 50), "miss_p99_ms": pct(lat[miss], 99),
                "traces": self.n_traces, "evictions": self.n_evictions,
                "batches": self.n_batches, "columns": self.n_cols, "channel_cache_hits": self.cache_hits,
                "admission_waits": self.admission_waits, "errors": self._errors}

    # ---------------- scheduling ----------------
    def _estimate(self, dep: Deployment, cols: int, cached: bool) -> int:
        ris = self._ris_host[dep.ris_key]
        R, M = dep.rx_pos.shape[0], ris.elems.shape[0]
        out = R * cols * 4 + M * cols * 8 * 3
        split = 2 * 2 * (2 * R + 128) * (2 * M + 32) + (cols + 128) * (2 * M + 32) * 4
        if cached:
            return out + split
        chan = R * M * 8 + R * 8
        trace_scratch = 64 * R * 300 + 64 * dep.n_rays * max(1, dep.order) + R * M * 4
        return out + split + chan + trace_scratch

    def _scheduler(self) -> None:
        while True:
            with self._lock:
                while self._running and (not self._queue or not self._free_slots):
                    self._lock.wait(0.05)
                if not self._running:
                    return
                # the oldest query, except that misses may not take the last free slot
                # (with one slot there is no such limit)
                head = None
                for q in self._queue:
                    if q.dep in self._chan or self.n_slots == 1 or self._misses_running < self.n_slots - 1:
                        head = q
                        break
                if head is None:
                    self._lock.wait(0.01)
                    continue
                batch = [head]
                cols = head.gamma.shape[1]
                for q in self._queue:
                    if q is not head and q.dep == head.dep and q.precision == head.precision and q.scale == head.scale \
                            and cols + q.gamma.shape[1] <= self.max_cols:
                        batch.append(q)
                        cols += q.gamma.shape[1]
                dep = self._deps[head.dep]
                est = self._estimate(dep, cols, head.dep in self._chan)
                in_use = self.ctx.mem_info()[0]
                busy = len(self._free_slots) < self.n_slots
                if busy and in_use + self._reserved + est > self._budget:
                    self.admission_waits += 1
                    self._lock.wait(0.01)
                    continue
                for q in batch:
                    self._queue.remove(q)
                slot = self._free_slots.pop()
                self._reserved += est
                miss = head.dep not in self._chan
                self._misses_running += miss
            self._work[slot].put((batch, est, miss))

    def _worker(self, slot: int) -> None:
        while True:
            item = self._work[slot].get()
            if item is None:
                return
            self._run_batch(slot, *item)

    # ---------------- device work ----------------
    def _scene(self, key: str, stream) -> int:
        with self._key_locks["scene:" + key]:
            if key not in self._scene_h:
                sc = self._scenes_host[key]
                self._scene_h[key] = self.ctx.scene_create(sc.V, sc.T, sc.surf, sc.refl_re, sc.refl_im,
                                                           stream=stream)
            return self._scene_h[key]

    def _ris(self, key: str) -> int:
        with self._key_locks["ris:" + key]:
            if key not in self._ris_h:
                r = self._ris_host[key]
                self._ris_h[key] = self.ctx.ris_create(r.elems, r.centre, r.normal, r.dy, r.dz, r.gain, r.q)
            return self._ris_h[key]

    def _channel(self, dep: Deployment, stream):
        """(channel handle, missed, segments traced): missed when the channel
        was not cached as the call began (this call traced it, or waited for
        the one that did)."""
        with self._lock:
            missed = dep.key not in self._chan
        with self._key_locks["chan:" + dep.key]:
            with self._lock:
                if dep.key in self._chan:
                    self._chan.move_to_end(dep.key)
                    self._in_use[dep.key] += 1
                    self.cache_hits += 1
                    return self._chan[dep.key], missed, 0
            self._evict(dep.key)
            scene = self._scene(dep.scene_key, stream)
            ris = self._ris(dep.ris_key)
            ch, st = self.ctx.trace(scene, ris, dep.tx_pos, dep.tx_axis, dep.tx_power_w, dep.tx_gain,
                                    dep.tx_pattern, dep.tx_param, dep.rx_pos, dep.rx_axis, dep.rx_gain,
                                    dep.rx_pattern, dep.rx_param, dep.freq_hz, dep.order, dep.n_rays,
                                    stream=stream)
            R, M, _, _ = self.ctx.channel_info(ch)
            with self._lock:
                self._chan[dep.key] = ch
                self._chan_bytes[dep.key] = _channel_bytes(R, M)
                self._in_use[dep.key] += 1
                self.n_traces += 1
            return ch, True, int(st["segments"])

    def _evict(self, keep: str) -> None:
        with self._lock:
            total = sum(self._chan_bytes.values())
            victims = []
            for k in list(self._chan.keys()):
                if total <= self._cache_limit:
                    break
                if k != keep and self._in_use[k] == 0:
                    victims.append((k, self._chan.pop(k)))
                    total -= self._chan_bytes.pop(k)
                    self.n_evictions += 1
        for _, h in victims:
            self.ctx.destroy(h)

    def _run_batch(self, slot: int, batch: List[_Query], est: int, miss: bool = False) -> None:
        torch = self._torch
        stream = self._streams[slot]
        dep = self._deps[batch[0].dep]
        held = False
        try:
            t_start = time.perf_counter()
            with torch.cuda.stream(stream):
                ch, missed, segments = self._channel(dep, stream)
                held = True
                # the batch's columns are gathered straight into pinned memory and uploaded on the slot's stream
                M = batch[0].gamma.shape[0]
                cols = sum(q.gamma.shape[1] for q in batch)
                gt = torch.empty((M, cols), dtype=torch.complex64, pin_memory=True)
                gv = gt.numpy()
                c0 = 0
                for q in batch:
                    gv[:, c0:c0 + q.gamma.shape[1]] = q.gamma
                    c0 += q.gamma.shape[1]
                gd = gt.to("cuda", non_blocking=True)
                _, P = self.ctx.ris_sum(ch, gd, scale=batch[0].scale, gamma_is_real=all(q.real for q in batch),
                                        precision=batch[0].precision, want_P=True, stream=stream)
                # the answer goes to pinned host memory (pageable copies of tens of MB dominate
                # a large query's latency otherwise); torch's host allocator reuses the blocks
                Pt = torch.empty(P.shape, dtype=P.dtype, pin_memory=True)
                Pt.copy_(P, non_blocking=True)
                stream.synchronize()
                Ph = Pt.numpy()
            t = time.perf_counter()
            c0 = 0
            lats = []
            for q in batch:
                c = q.gamma.shape[1]
                q.future.set_result(Ph[:, c0:c0 + c])
                c0 += c
                lats.append(t - q.t_submit)
            with self._lock:
                self.latencies.extend(lats)
                self.missed.extend([missed] * len(lats))
                self.n_batches += 1
                self.n_cols += cols
            if self._log is not None:
                R = P.shape[0]
                lines = [json.dumps({"qid": q.qid, "deployment": q.dep, "columns": int(q.gamma.shape[1]),
                                     "precision": q.precision, "cache": "miss" if missed else "hit",
                                     "latency_ms": 1e3 * lat, "queue_ms": 1e3 * (t_start - q.t_submit),
                                     "batch_queries": len(batch), "batch_columns": cols, "slot": slot,
                                     "segments_traced": segments, "bytes_out": R * int(q.gamma.shape[1]) * 4})
                         for q, lat in zip(batch, lats)]
                with self._log_lock:
                    self._log.write("\n".join(lines) + "\n")
                    self._log.flush()   # a batch's lines survive a crash of the process
        except risrt.RtError as e:
            requeue = False
            with self._lock:
                # out of budget while other work holds memory: wait for it instead of failing
                if e.status == risrt.RT_ENOMEM and len(self._free_slots) < self.n_slots - 1:
                    self._queue[0:0] = batch
                    self.admission_waits += 1
                    requeue = True
                else:
                    self._errors += 1
            if not requeue:
                for q in batch:
                    if not q.future.done():
                        q.future.set_exception(e)
        except Exception as e:   # surfaced to the callers; the loop keeps serving
            with self._lock:
                self._errors += 1
            for q in batch:
                if not q.future.done():
                    q.future.set_exception(e)
        finally:
            with self._lock:
                if held:
                    self._in_use[dep.key] -= 1
                self._reserved -= est
                self._misses_running -= miss
                self._free_slots.append(slot)
                self._lock.notify_all()


def _channel_bytes(R: int, M: int) -> int:
    # H, its cached two-part split and E_env
    return R * M * 8 * 3 + R * 8


def _dep_meta(dep: Deployment) -> dict:
    """The deployment parameters a channel depends on, JSON-ready."""
    d = dataclasses.asdict(dep)
    d.pop("key")
    d.pop("rx_pos")
    out = {k: np.asarray(v).tolist() for k, v in d.items()}   # numpy scalars and arrays to plain numbers
    out["rx_pos_sha1"] = hashlib.sha1(np.ascontiguousarray(dep.rx_pos, np.float64)).hexdigest()
    return out


def run_poisson(server: Server, queries, rate_hz: float, seed: int = 0):
    """Submit (dep_key, gamma) pairs with exponential inter-arrival times and
    wait for all answers.  Returns the futures in submission order."""
    rng = np.random.default_rng(seed)
    futs = []
    t_next = time.perf_counter()
    for dep_key, gamma in queries:
        t_next += rng.exponential(1.0 / rate_hz)
        d = t_next - time.perf_counter()
        if d > 0:
            time.sleep(d)
        futs.append(server.submit(dep_key, gamma))
    for f in futs:
        f.exception()
    return futs
