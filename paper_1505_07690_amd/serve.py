"""Serving: continuous batching of orientation-score jobs on one GPU.

A job is one volume f (float32, on the device) with a bank key
(shape, N_o, L).  Its work is either forward + reconstruction (the score
U of N^3 N_o complex values is materialised in HBM between the two calls) or
processing via scores (Eq. 23, fused: U never reaches memory).

A scheduler thread:

* admits pending jobs while an execution slot (a HIP stream) and enough of
  the HBM budget are free; the footprint of a job is its score, its input
  and output volumes and the library workspace of its launch;
* groups pending jobs with the same bank key and operation into one batched
  launch (the batch dimension of the C ABI);
* keeps wavelet banks cached on the device per key, counts their bytes
  against the same budget, and drops the least recently used idle bank when
  a new one needs the room; a missing bank is built by a thread of its own,
  so that launches keep being reaped and admitted meanwhile;
* lets jobs run concurrently on different streams and resolves each job's
  Future as soon as its launch has finished on the device, handing the
  output over to the stream the job was submitted from (the allocator does
  not reuse its memory before that stream's work on it is done);
* rejects a job that cannot fit even on an idle server (AdmissionError),
  fails only the affected jobs when a bank build or a launch raises, honours
  Future.cancel() before admission and a per-job timeout while pending, and
  stops admitting younger jobs while the oldest one has waited too long.

The scheduling logic only talks to an executor object (``GpuExecutor`` on
the device; tests substitute their own), so it runs unchanged on the CPU.
"""
from __future__ import annotations

import collections
import itertools
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np

__all__ = ["AdmissionError", "JobTimeout", "Server", "GpuExecutor", "bank_key"]

ORIENT_LEVEL = {12: 0, 42: 1, 162: 2}


class AdmissionError(RuntimeError):
    """The job's footprint exceeds the HBM budget even on an idle server."""


class JobTimeout(TimeoutError):
    """The job was still pending when its timeout expired."""


def bank_key(shape, n_orients, L):
    shape = tuple(int(s) for s in shape)
    if len(shape) != 3:
        raise ValueError(f"shape must have three dims, got {shape}")
    return (shape, int(n_orients), int(L))


@dataclass(eq=False)
class _Job:
    id: int
    key: tuple
    volume: object
    op: str
    dtype: str
    phi: str
    power: float
    future: Future
    t_submit: float
    deadline: float | None
    ready: object = None          # device event: the input volume is complete
    consumer: object = None       # the submitting thread's stream (where the result is used)
    t_admit: float | None = None
    t_done: float | None = None
    batch: int = 0
    state: str = "pending"        # pending -> running -> done

    @property
    def group(self):
        return (self.key, self.op, self.dtype, self.phi, self.power)


@dataclass(eq=False)
class _BankEntry:
    bank: object
    nbytes: int
    refs: int = 0
    last_used: float = 0.0
    launches: int = 0             # launches that have used it
    building: bool = False        # a builder thread is synthesising it
    error: object = None          # the build's exception, if it failed


@dataclass(eq=False)
class _Launch:
    slot: int
    jobs: list
    handle: object
    nbytes: int
    entry: _BankEntry


@dataclass
class _Record:
    key: tuple
    op: str
    vo: int
    t_submit: float
    t_admit: float
    t_done: float
    batch: int
    ok: bool


class Server:
    """Continuous-batching request loop over an executor.

    hbm_budget: bytes of device memory the server may hold (cached banks and
    in-flight job footprints together).  n_slots: concurrent launches.
    max_batch: jobs per batched launch; batch_bytes: a batch grows only
    while its footprint stays within this many bytes (the library runs the
    volumes of a batch one after another, so batching pays for small jobs,
    where launches are short, and only delays large ones).  starvation_s:
    once the oldest pending job has waited this long, younger jobs are not
    admitted ahead of it.

    Executors that keep per-slot scratch (a launch's workspace and scores,
    reused by the slot's next launch: no large allocation, and no stall of
    the scheduler while the driver maps it, once every slot has seen its
    largest job) report it, and the server counts it against the budget
    until it releases it: a slot's scratch is given back when the slot is
    idle and memory is needed, before any cached bank is dropped, and when
    the server closes.

    The budget is capped at 90 % of the device memory free when the server
    starts (after the executor has handed back its allocator's unused
    cache): a budget beyond it makes the allocator release and re-reserve
    memory mid-stream, which synchronises the device (measured: a 200-job
    stream started with a previous server's blocks still cached ran at p50
    1.1 s instead of 4 ms).  budget_requested keeps the value asked for.
    """

    def __init__(self, hbm_budget, n_slots=4, max_batch=8, executor=None, starvation_s=0.25, poll_s=2e-4,
                 batch_bytes=4 << 30):
        self.budget = self.budget_requested = int(hbm_budget)
        self.n_slots = int(n_slots)
        self.max_batch = int(max_batch)
        self.batch_bytes = int(batch_bytes)
        self.starvation_s = float(starvation_s)
        self.poll_s = float(poll_s)
        self.ex = executor if executor is not None else GpuExecutor(n_slots=self.n_slots)
        if getattr(self.ex, "n_slots", self.n_slots) < self.n_slots:
            raise ValueError("executor has fewer slots than the server")
        avail = getattr(self.ex, "device_bytes_available", None)
        if avail is not None:
            free = avail()
            if free is not None:
                self.budget = min(self.budget, int(0.9 * free))
        self._cv = threading.Condition()
        self._incoming = collections.deque()
        self._pending = []
        self._inflight = []
        self._free_slots = list(range(self.n_slots))
        self._banks = collections.OrderedDict()
        self._used = 0
        self.peak_bytes = 0
        self.bank_hits = 0
        self.bank_misses = 0
        self.bank_evictions = 0
        self.bank_build_s = []
        self.records = []
        self.errors = collections.Counter()
        self.error_examples = {}
        self._ids = itertools.count()
        self._closing = False
        self._error = None
        self._builders = set()
        self._scratch = hasattr(self.ex, "scratch_bytes")
        self._scratch_acc = [0] * self.n_slots  # bytes of each slot's scratch, counted in _used
        self._controls = collections.deque()     # work for the scheduler thread once every slot is idle
        self._thread = threading.Thread(target=self._loop, name="os3d-serve", daemon=True)
        self._thread.start()

    # ------------------------------------------------------------ client --
    def submit(self, volume, n_orients, L, op="reconstruct", dtype="c64", phi="soft_threshold", power=1.5,
               timeout=None):
        """Queue one job; the Future resolves to the output volume (a device
        tensor of the input's shape) or to the job's exception."""
        fut = Future()
        try:
            key = bank_key(tuple(volume.shape), n_orients, L)
            if op not in ("reconstruct", "process"):
                raise ValueError(f"unknown op {op!r}")
            if op == "process" and dtype != "c64":
                raise ValueError("processing via scores keeps the score in registers: dtype must be c64")
        except Exception as e:  # invalid request: fail it alone
            fut.set_exception(e)
            return fut
        now = time.perf_counter()
        job = _Job(next(self._ids), key, volume, op, dtype, phi, float(power), fut, now,
                   None if timeout is None else now + float(timeout))
        job.ready = self.ex.input_ready(volume)
        if hasattr(self.ex, "consumer_stream"):
            job.consumer = self.ex.consumer_stream(volume)
        with self._cv:
            if self._closing:
                raise RuntimeError("server is closed")
            self._incoming.append(job)
            self._cv.notify()
        return fut

    def close(self, wait=True):
        """Stop taking work, finish what was submitted and (wait=True)
        release the cached banks: a closed server holds no device memory."""
        with self._cv:
            self._closing = True
            self._cv.notify()
        if wait:
            self._thread.join()
            for t in list(self._builders):
                t.join()
            for key, e in list(self._banks.items()):
                if e.bank is not None:
                    self.ex.free_bank(e.bank)
                    e.bank = None
                self._account(-e.nbytes)
            self._banks.clear()
            for slot in range(self.n_slots):
                self._release_scratch(slot)
        if self._error is not None:
            raise RuntimeError("scheduler failed") from self._error

    def reserve_scratch(self, keys=None, batch=1, op="reconstruct", dtype="c64", timeout=60.0):
        """Size every slot's scratch for the largest job of `keys` (batches
        of `batch` jobs) among the cached banks (all of them by default), as
        far as the budget allows, so that the first launches of a burst do
        not grow it on the scheduler thread.  Runs on the scheduler thread
        once every slot is idle (admission pauses meanwhile).  Returns the
        scratch bytes per slot asked for (0 for executors without scratch)."""
        if not self._scratch:
            return 0
        done, box = threading.Event(), {}

        def run():
            try:
                ks = list(self._banks) if keys is None else [(tuple(k[0]), int(k[1]), int(k[2])) for k in keys]
                need = 0
                for k in ks:
                    e = self._banks.get(k)
                    if e is not None and e.bank is not None:
                        need = max(need, self.ex.scratch_bytes(k, e.bank, batch, op, dtype))
                for slot in range(self.n_slots):
                    grow = need - self._scratch_acc[slot]
                    if grow > 0 and self.budget - self._used >= grow:
                        self.ex.grow_scratch(slot, need)
                        self._account(grow)
                        self._scratch_acc[slot] = need
                box["bytes"] = need
            except Exception as e:  # reported to the caller
                box["error"] = e
            done.set()

        with self._cv:
            if self._closing:
                raise RuntimeError("server is closed")
            self._controls.append(run)
            self._cv.notify()
        if not done.wait(timeout):
            raise TimeoutError("reserve_scratch: the slots did not become idle")
        if "error" in box:
            raise box["error"]
        return box["bytes"]

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def stats(self):
        """Latency percentiles, throughput, bank-cache and memory figures
        over the finished jobs."""
        ok = [r for r in self.records if r.ok]
        out = dict(jobs=len(self.records), ok=len(ok), failed=len(self.records) - len(ok),
                   bank_hits=self.bank_hits, bank_misses=self.bank_misses, bank_evictions=self.bank_evictions,
                   bank_hit_rate=self.bank_hits / max(1, self.bank_hits + self.bank_misses),
                   bank_builds=len(self.bank_build_s),
                   bank_build_ms_max=1e3 * max(self.bank_build_s, default=0.0),
                   peak_bytes=self.peak_bytes, errors=dict(self.errors),
                   error_examples=dict(self.error_examples))
        if ok:
            lat = np.array([r.t_done - r.t_submit for r in ok]) * 1e3
            wait = np.array([r.t_admit - r.t_submit for r in ok]) * 1e3
            t0 = min(r.t_submit for r in ok)
            t1 = max(r.t_done for r in ok)
            out.update(p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                       mean_wait_ms=float(wait.mean()), span_s=t1 - t0,
                       jobs_per_s=len(ok) / max(t1 - t0, 1e-9),
                       vo_per_s=sum(r.vo for r in ok) / max(t1 - t0, 1e-9),
                       max_batch=max(r.batch for r in ok),
                       mean_batch=float(np.mean([r.batch for r in ok])))
            per = collections.defaultdict(list)
            for r in ok:
                per[r.key].append((r.t_done - r.t_submit) * 1e3)
            out["per_key"] = {"x".join(map(str, k[0])) + f" No={k[1]} L={k[2]}":
                              dict(jobs=len(v), p50_ms=float(np.percentile(v, 50)), p99_ms=float(np.percentile(v, 99)))
                              for k, v in sorted(per.items())}
        return out

    # --------------------------------------------------------- scheduler --
    def _loop(self):
        try:
            while True:
                with self._cv:
                    while self._incoming:
                        self._pending.append(self._incoming.popleft())
                    if self._closing and not self._pending and not self._inflight:
                        return
                progress = self._reap()
                progress |= self._expire()
                if self._controls:  # admission waits until every slot is idle
                    if not self._inflight and len(self._free_slots) == self.n_slots:
                        while self._controls:
                            self._controls.popleft()()
                        progress = True
                else:
                    progress |= self._admit()
                if not progress:
                    with self._cv:
                        if not self._incoming:
                            self._cv.wait(self.poll_s)
        except BaseException as e:  # never leave futures hanging
            self._error = e
            for j in self._pending + [j for ln in self._inflight for j in ln.jobs] + list(self._incoming):
                if not j.future.done():
                    j.future.set_exception(RuntimeError(f"scheduler failed: {e!r}"))

    def _account(self, delta):
        self._used += delta
        self.peak_bytes = max(self.peak_bytes, self._used)

    def _finish(self, job, ok, now, result=None, exc=None):
        job.state = "done"
        job.t_done = now
        self.records.append(_Record(job.key, job.op, int(np.prod(job.key[0])) * job.key[1], job.t_submit,
                                    job.t_admit if job.t_admit is not None else now, now, job.batch, ok))
        job.volume = None
        if ok:
            if job.consumer is not None:
                self.ex.hand_over(result, job.consumer)
            job.future.set_result(result)
        else:
            name = type(exc).__name__
            self.errors[name] += 1
            self.error_examples.setdefault(name, str(exc)[:300])
            if not job.future.done():
                job.future.set_exception(exc)

    def _reap(self):
        done = [ln for ln in self._inflight if self.ex.done(ln.handle)]
        if not done:
            return False
        now = time.perf_counter()
        for ln in done:
            self._inflight.remove(ln)
            try:
                outs = self.ex.results(ln.handle)
                err = None
            except Exception as e:
                outs, err = None, e
            for i, j in enumerate(ln.jobs):
                self._finish(j, err is None, now, outs[i] if err is None else None, err)
            ln.handle = None
            ln.entry.refs -= 1
            ln.entry.last_used = now
            self._account(-ln.nbytes)
            self._free_slots.append(ln.slot)
        return True

    def _expire(self):
        now = time.perf_counter()
        keep, changed = [], False
        for j in self._pending:
            if j.future.cancelled():
                j.state = "done"
                changed = True
            elif j.deadline is not None and now > j.deadline:
                self._finish(j, False, now, exc=JobTimeout(f"job {j.id} still pending after its timeout"))
                changed = True
            else:
                keep.append(j)
        self._pending = keep
        return changed

    def _release_scratch(self, slot):
        if self._scratch_acc[slot]:
            self.ex.release_scratch(slot)
            self._account(-self._scratch_acc[slot])
            self._scratch_acc[slot] = 0

    def _evict_for(self, need, keep_key, keep_slot=None):
        """Make `need` bytes free.  First give back the scratch of idle
        slots (other than keep_slot).  While the running launches will
        release enough on their own, wait for them (False) rather than drop
        a cached bank; otherwise drop idle banks, least recently used first.
        False if that is impossible now."""
        if self.budget - self._used >= need:
            return True
        for slot in self._free_slots:
            if self.budget - self._used >= need:
                return True
            if slot != keep_slot:
                self._release_scratch(slot)
        if self.budget - self._used >= need:
            return True
        if self.budget - self._used + sum(ln.nbytes for ln in self._inflight) >= need:
            return False
        idle = sorted((e.last_used, k) for k, e in self._banks.items() if e.refs == 0 and k != keep_key)
        free_after = self.budget - self._used + sum(self._banks[k].nbytes for _, k in idle)
        if free_after < need:
            return False
        for _, k in idle:
            if self.budget - self._used >= need:
                break
            e = self._banks.pop(k)
            self._account(-e.nbytes)
            if e.bank is not None:  # None: a failed build, nothing to free
                self.ex.free_bank(e.bank)
            self.bank_evictions += 1
        return True

    def _fail_group(self, jobs, exc):
        now = time.perf_counter()
        for j in jobs:
            if j in self._pending:
                self._pending.remove(j)
            self._finish(j, False, now, exc=exc)

    def _admit(self):
        if not self._pending or not self._free_slots:
            return False
        progress = False
        now = time.perf_counter()
        oldest = self._pending[0]
        starving = now - oldest.t_submit > self.starvation_s
        groups = collections.defaultdict(list)
        for j in self._pending:
            if not j.future.cancelled():
                groups[j.group].append(j)
        tried = set()
        for job in list(self._pending):
            if not self._free_slots:
                break
            if job.state != "pending" or job.group in tried:
                continue  # taken into a batch, failed, or its group already tried this pass
            if starving and job is not oldest:
                break
            tried.add(job.group)
            progress |= self._try_admit(job, [j for j in groups[job.group] if j.state == "pending"])
        return progress

    def _try_admit(self, job, candidates):
        key = job.key
        entry = self._banks.get(key)
        if entry is not None and entry.building:
            return False  # its builder thread has not finished
        if entry is not None and entry.error is not None:
            self._banks.pop(key)
            self._account(-entry.nbytes)
            self._fail_group([j for j in self._pending if j.key == key], entry.error)
            return True
        bank_need = 0
        if entry is None:
            try:
                bank_need = self.ex.bank_bytes(key)
            except Exception as e:
                self._fail_group([j for j in self._pending if j.key == key], e)
                return True
            # the exact footprint needs the bank's workspace size: check a
            # lower bound for a single job first, and build the bank (on a
            # thread of its own) only if that fits
            est = self.ex.job_bytes_estimate(key, 1, job.op, job.dtype)
            if bank_need + est > self.budget:
                self._fail_group([job], AdmissionError(
                    f"job {job.id} needs {bank_need + est} bytes, budget is {self.budget}"))
                return True
            # the job may run in the largest idle slot scratch: that much
            # of its footprint is already counted
            keep_slot = None
            if self._scratch and self._free_slots:
                keep_slot = max(self._free_slots, key=lambda k: (self._scratch_acc[k], -k))
                est = max(0, est - self._scratch_acc[keep_slot])
            need1 = bank_need + est
            if not self._evict_for(need1, key, keep_slot):
                return self._maybe_reject(job, need1)
            entry = _BankEntry(None, bank_need, refs=1, building=True)
            self._banks[key] = entry
            self._account(bank_need)
            self.bank_misses += 1
            t = threading.Thread(target=self._build, args=(key, entry), name="os3d-bank", daemon=True)
            self._builders.add(t)
            t.start()
            return True
        self._banks.move_to_end(key)
        group = candidates[: self.max_batch]
        # the free slot whose scratch is largest: the least to grow
        slot = max(self._free_slots, key=lambda k: (self._scratch_acc[k], -k))

        def footprint(m):
            """(bytes to add now, bytes released when the launch ends)."""
            total = self.ex.job_bytes(key, entry.bank, m, job.op, job.dtype)
            if not self._scratch:
                return total, total
            scratch = self.ex.scratch_bytes(key, entry.bank, m, job.op, job.dtype)
            return total - scratch + max(0, scratch - self._scratch_acc[slot]), total - scratch

        # largest prefix of the group whose footprint fits (and stays within
        # batch_bytes when it has more than one job)
        n = len(group)
        while n > 1 and self.ex.job_bytes(key, entry.bank, n, job.op, job.dtype) > self.batch_bytes:
            n -= 1
        while n > 0:
            need, transient = footprint(n)
            if need <= self.budget - entry.nbytes and self._evict_for(need, key, slot):
                break
            n -= 1
        if n == 0:
            need = self.ex.job_bytes(key, entry.bank, 1, job.op, job.dtype)
            if need + entry.nbytes > self.budget:
                self._fail_group([job], AdmissionError(
                    f"job {job.id} needs {need + entry.nbytes} bytes with its bank, budget is {self.budget}"))
                return True
            return self._maybe_reject(job, need)
        batch = []
        for j in group[:n]:
            if j.future.set_running_or_notify_cancel():
                batch.append(j)
                j.state = "running"
            else:
                j.state = "done"
            self._pending.remove(j)
        if not batch:
            return True
        need, transient = footprint(len(batch))
        self._free_slots.remove(slot)
        now = time.perf_counter()
        for j in batch:
            j.t_admit = now
            j.batch = len(batch)
        try:
            handle = self.ex.launch(slot, entry.bank, batch)
        except Exception as e:
            if self._scratch:  # whatever the failed launch left in the slot's scratch goes back
                self.ex.release_scratch(slot)
                self._account(-self._scratch_acc[slot])
                self._scratch_acc[slot] = 0
            self._free_slots.append(slot)
            for j in batch:
                self._finish(j, False, time.perf_counter(), exc=e)
            return True
        entry.refs += 1
        self.bank_hits += int(entry.launches > 0)
        entry.launches += 1
        self._account(need)
        if self._scratch:  # the slot's scratch stays counted after the launch
            self._scratch_acc[slot] += need - transient
        self._inflight.append(_Launch(slot, batch, handle, transient, entry))
        return True

    def _build(self, key, entry):
        """Builder thread: synthesise one bank, then wake the scheduler."""
        t0 = time.perf_counter()
        try:
            bank, err = self.ex.build_bank(key), None
        except Exception as e:
            bank, err = None, e
        with self._cv:
            entry.bank, entry.error = bank, err
            entry.building = False
            entry.refs -= 1
            entry.last_used = time.perf_counter()
            self.bank_build_s.append(entry.last_used - t0)
            self._builders.discard(threading.current_thread())
            self._cv.notify()

    def _maybe_reject(self, job, need):
        """A job that does not fit now waits, unless nothing is running and
        no idle bank is left to drop: then it can never fit."""
        if not self._inflight and all(e.refs == 0 for e in self._banks.values()):
            idle = sum(e.nbytes for k, e in self._banks.items() if k != job.key) + sum(self._scratch_acc)
            if self.budget - self._used + idle < need:
                self._fail_group([job], AdmissionError(f"job {job.id} needs {need} bytes, budget is {self.budget}"))
                return True
        return False


# ------------------------------------------------------------- the GPU --

def _orients(n):
    from . import inputs
    if n not in ORIENT_LEVEL:
        raise ValueError(f"N_o must be one of {sorted(ORIENT_LEVEL)} (icosahedral sets), got {n}")
    return inputs.icosahedral_orientations(ORIENT_LEVEL[n])


def _params(n, L):
    from . import inputs, os3d
    return os3d.make_params(L=L, s_theta=inputs.s_theta_for(n))


@dataclass(eq=False)
class _GpuHandle:
    event: object
    outs: list
    keep: list = field(default_factory=list)


class GpuExecutor:
    """Runs launches of the C ABI on n_slots HIP streams (default priority)."""

    def __init__(self, n_slots=4, device="cuda"):
        import torch
        from . import os3d
        os3d.lib()  # the HIP library must be there
        self.torch = torch
        self.device = torch.device(device)
        self.n_slots = int(n_slots)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(self.n_slots)]
        self.build_stream = torch.cuda.Stream(device=self.device)
        # per slot: one byte buffer holding a launch's workspace and scores,
        # reused by the slot's next launch (its stream orders the two)
        self._slot_buf = [None] * self.n_slots

    def device_bytes_available(self):
        """Device memory free for the server: the allocator's unused cache is
        handed back first (it could otherwise not be reused for blocks of
        other sizes without a device-wide release mid-stream)."""
        self.torch.cuda.synchronize(self.device)
        self.torch.cuda.empty_cache()
        free, _ = self.torch.cuda.mem_get_info(self.device)
        return int(free)

    def input_ready(self, volume):
        torch = self.torch
        if not (isinstance(volume, torch.Tensor) and volume.is_cuda):
            return None
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(volume.device))
        return ev

    def bank_bytes(self, key):
        from . import os3d
        shape, n, L = key
        return os3d.bank_bytes(shape, _orients(n), _params(n, L))

    def build_bank(self, key):
        """Synthesise a bank on the executor's build stream (called from a
        builder thread); launches wait for its `ready` event."""
        from . import os3d
        shape, n, L = key
        s = self.build_stream
        with self.torch.cuda.device(self.device), self.torch.cuda.stream(s):
            bank = os3d.Bank(shape, _orients(n), _params(n, L), device=self.device, stream=s)
            bank.ready = self.torch.cuda.Event()
            bank.ready.record(s)
        return bank

    def consumer_stream(self, volume):
        """The submitting thread's current stream: where the caller will use
        the job's result."""
        torch = self.torch
        dev = volume.device if isinstance(volume, torch.Tensor) and volume.is_cuda else self.device
        return torch.cuda.current_stream(dev)

    def hand_over(self, result, stream):
        """Mark the result's memory as used by the consumer's stream, so that
        once the caller drops it the allocator waits for the work queued
        there before giving the block to another launch."""
        result.record_stream(stream)

    def free_bank(self, bank):
        bank.close()

    @staticmethod
    def _score_bytes(shape, n, B, op, dtype):
        V = int(np.prod(shape))
        io = 2 * B * V * 4 + (B * V * 4 if B > 1 else 0)  # f, f_out, the stacked batch
        if op == "process":
            return io
        su = 8 if dtype == "c64" else 4
        return io + B * n * V * su + B * n * 4

    def job_bytes_estimate(self, key, B, op, dtype):
        """A lower bound of the footprint before the bank exists: the
        library's workspace is at least F, X and two intermediate volumes.
        The exact footprint (job_bytes) is taken once the bank is built."""
        shape, n, L = key
        V = int(np.prod(shape))
        return self._score_bytes(shape, n, B, op, dtype) + 4 * V * 8

    def job_bytes(self, key, bank, B, op, dtype):
        shape, n, L = key
        return self._score_bytes(shape, n, B, op, dtype) + bank.ws_bytes

    @staticmethod
    def _scratch_layout(bank, B, n, shape, op, dtype):
        """Byte offsets in a slot's scratch: workspace, scores, scales."""
        def up(x):
            return (x + 255) // 256 * 256
        V = int(np.prod(shape))
        ws = up(bank.ws_bytes)
        if op == "process":
            return ws, 0, 0, ws
        u = up(B * n * V * (8 if dtype == "c64" else 4))
        return ws, ws + u, up(B * n * 4), ws + u + up(B * n * 4)

    def scratch_bytes(self, key, bank, B, op, dtype):
        shape, n, L = key
        return self._scratch_layout(bank, B, n, shape, op, dtype)[3]

    def release_scratch(self, slot):
        self._slot_buf[slot] = None

    def grow_scratch(self, slot, nbytes):
        self._scratch(slot, nbytes)

    def _scratch(self, slot, nbytes):
        buf = self._slot_buf[slot]
        if buf is None or buf.numel() < nbytes:
            self._slot_buf[slot] = None  # the slot's stream has finished with it (the slot was free)
            buf = self._slot_buf[slot] = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
        return buf

    def launch(self, slot, bank, jobs):
        torch = self.torch
        s = self.streams[slot]
        with torch.cuda.stream(s):
            s.wait_event(bank.ready)
            for j in jobs:
                if j.ready is not None:
                    s.wait_event(j.ready)
            try:
                return self._enqueue(slot, s, bank, jobs)
            except torch.OutOfMemoryError:
                # blocks cached for other shapes may fragment the pool: return
                # them to the device and try once more
                torch.cuda.empty_cache()
                return self._enqueue(slot, s, bank, jobs)

    def _enqueue(self, slot, s, bank, jobs):
        """Take the launch's buffers (workspace and scores from the slot's
        scratch) and enqueue its work on stream s (the current stream)."""
        from . import os3d
        torch = self.torch
        j0 = jobs[0]
        vols = [j.volume if j.volume.is_cuda else j.volume.to(self.device, non_blocking=True) for j in jobs]
        f = vols[0].contiguous() if len(vols) == 1 else torch.stack(vols)
        if f.dtype != torch.float32:
            raise ValueError("volumes must be float32")
        B = len(jobs)
        shape, n = tuple(f.shape[-3:]), bank.n_orients
        o_u, o_sc, _, total = self._scratch_layout(bank, B, n, shape, j0.op, j0.dtype)
        buf = self._scratch(slot, total)
        ws = buf[: bank.ws_bytes]
        keep = [f]
        if j0.op == "reconstruct":
            V = int(np.prod(shape))
            if j0.dtype == "c64":
                U = buf[o_u: o_u + B * n * V * 8].view(torch.complex64).view((B, n) + shape)
                sc = None
            else:
                U = buf[o_u: o_u + B * n * V * 4].view(torch.int32).view((B, n) + shape)
                sc = buf[o_sc: o_sc + B * n * 4].view(torch.float32).view(B, n)
            fb = f if f.dim() == 4 else f.unsqueeze(0)
            U, sc = os3d.forward(fb, bank, dtype=j0.dtype, ws=ws, out=U, scales=sc, stream=s)
            out = os3d.reconstruct(U, bank, scales=sc, dtype=j0.dtype, ws=ws, stream=s)
            if f.dim() == 3:
                out = out[0]
        else:
            out = os3d.process(f, bank, j0.phi, j0.power, ws=ws, stream=s)
        ev = torch.cuda.Event()
        ev.record(s)
        outs = [out] if len(jobs) == 1 and out.dim() == 3 else [out[i] for i in range(len(jobs))]
        return _GpuHandle(ev, outs, keep)

    def done(self, handle):
        return handle.event.query()

    def results(self, handle):
        outs = handle.outs
        handle.keep.clear()  # the input copy goes back to the allocator (the scratch stays with its slot)
        return outs
