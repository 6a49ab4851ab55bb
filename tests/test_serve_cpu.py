"""Host logic of the serving loop (continuous batching, admission by HBM
footprint, bank cache, failure handling) driven through a fake executor on
the CPU: every launch "runs" for a fixed time and doubles its volumes."""
import threading
import time

import numpy as np
import pytest

from paper_1505_07690_amd.serve import AdmissionError, JobTimeout, Server


class FakeBank:
    def __init__(self, key):
        self.key = key
        V = int(np.prod(key[0]))
        self.ws_bytes = 4 * V * 8
        self.closed = False

    def close(self):
        self.closed = True


class FakeHandle:
    def __init__(self, jobs, t_end):
        self.outs = [2.0 * j.volume for j in jobs]
        self.t_end = t_end
        self.n = len(jobs)


class FakeExecutor:
    def __init__(self, n_slots, run_s=0.02, fail_keys=(), build_s=None):
        self.n_slots = n_slots
        self.run_s = run_s
        self.fail_keys = set(fail_keys)
        self.build_s = dict(build_s or {})
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.launches = []
        self.built = []
        self.freed = []

    def input_ready(self, volume):
        return None

    def bank_bytes(self, key):
        shape, n, L = key
        if n not in (12, 42, 162):
            raise ValueError("unsupported orientation count")
        return int(np.prod(shape)) * n * 2

    def build_bank(self, key):
        time.sleep(self.build_s.get(key, 0.0))
        if key in self.fail_keys:
            raise RuntimeError("bank build failed")
        self.built.append(key)
        return FakeBank(key)

    def free_bank(self, bank):
        self.freed.append(bank.key)
        bank.close()

    def job_bytes_estimate(self, key, B, op, dtype):
        return self.job_bytes(key, FakeBank(key), B, op, dtype)

    def job_bytes(self, key, bank, B, op, dtype):
        shape, n, L = key
        V = int(np.prod(shape))
        return B * n * V * 8 + bank.ws_bytes

    def launch(self, slot, bank, jobs):
        for j in jobs:
            if not np.all(np.isfinite(j.volume)):
                raise ValueError("invalid volume")
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
        self.launches.append([j.id for j in jobs])
        return FakeHandle(jobs, time.perf_counter() + self.run_s)

    def done(self, h):
        if time.perf_counter() >= h.t_end:
            if h.outs is not None and not getattr(h, "_counted", False):
                h._counted = True
                with self.lock:
                    self.active -= 1
            return True
        return False

    def results(self, h):
        return h.outs


def vol(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape).astype(np.float32)


def fp(shape, n):
    """Footprint of one job plus its bank under the fake executor."""
    V = int(np.prod(shape))
    return n * V * 8 + 4 * V * 8 + V * n * 2


def test_results_and_continuous_batching():
    ex = FakeExecutor(1, run_s=0.05)
    with Server(1 << 30, n_slots=1, max_batch=4, executor=ex) as s:
        vs = [vol((8, 8, 8), i) for i in range(7)]
        futs = [s.submit(vs[0], 42, 16)]
        time.sleep(0.02)
        futs += [s.submit(v, 42, 16) for v in vs[1:]]
        for f, v in zip(futs, vs):
            assert np.array_equal(f.result(timeout=5), 2 * v)
        st = s.stats()
    assert st["ok"] == 7 and st["max_batch"] > 1
    # the first job ran alone; the ones that arrived meanwhile shared launches
    assert ex.launches[0] == [0]
    assert sum(len(b) for b in ex.launches) == 7 and max(len(b) for b in ex.launches) <= 4
    assert st["bank_misses"] == 1 and st["bank_hits"] == len(ex.launches) - 1


def test_mixed_keys_run_concurrently_on_slots():
    ex = FakeExecutor(3, run_s=0.05)
    with Server(1 << 30, n_slots=3, executor=ex) as s:
        futs = [s.submit(vol(sh, i), n, L) for i, (sh, n, L) in
                enumerate([((8, 8, 8), 42, 16), ((6, 8, 10), 12, 8), ((8, 8, 8), 162, 24)])]
        for f in futs:
            f.result(timeout=5)
    assert ex.max_active == 3


def test_admission_rejects_what_cannot_fit_and_keeps_serving():
    ex = FakeExecutor(2)
    budget = fp((8, 8, 8), 42) + 100
    with Server(budget, n_slots=2, executor=ex) as s:
        big = s.submit(vol((16, 16, 16), 0), 42, 16)
        small = s.submit(vol((8, 8, 8), 1), 42, 16)
        with pytest.raises(AdmissionError):
            big.result(timeout=5)
        assert np.array_equal(small.result(timeout=5), 2 * vol((8, 8, 8), 1))


def test_exact_footprint_checked_after_the_bank_is_built():
    """Before a bank exists the server only knows a lower bound of a job's
    footprint (the workspace size comes with the bank).  A job that passes
    the bound but not the exact check is rejected once the bank is built;
    the bank stays cached and other jobs keep running."""
    class LowerBound(FakeExecutor):
        def job_bytes_estimate(self, key, B, op, dtype):
            shape, n, L = key
            return B * n * int(np.prod(shape)) * 8  # the scores only

    ex = LowerBound(2)
    shape = (8, 8, 8)
    V = 8 ** 3
    budget = V * 42 * 2 + 42 * V * 8 + 2 * V * 8  # bank + scores + less than the 4 V * 8 workspace
    with Server(budget, n_slots=2, executor=ex) as s:
        job = s.submit(vol(shape, 5), 42, 16)
        with pytest.raises(AdmissionError):
            job.result(timeout=5)
        small = s.submit(vol((4, 4, 4), 6), 12, 8)
        assert np.array_equal(small.result(timeout=5), 2 * vol((4, 4, 4), 6))
        st = s.stats()
    assert ex.built[0] == (shape, 42, 16) and st["errors"].get("AdmissionError", 0) >= 1


def test_memory_budget_serialises_jobs():
    """Room for one bank and one job: jobs wait for memory, never run two at
    a time, and all finish."""
    ex = FakeExecutor(4, run_s=0.01)
    budget = fp((8, 8, 8), 42) + 100
    with Server(budget, n_slots=4, max_batch=1, executor=ex) as s:
        futs = [s.submit(vol((8, 8, 8), i), 42, 16) for i in range(5)]
        for f in futs:
            f.result(timeout=5)
        st = s.stats()
    assert ex.max_active == 1
    assert st["peak_bytes"] <= budget


def test_invalid_job_fails_alone():
    ex = FakeExecutor(2)
    with Server(1 << 30, n_slots=2, max_batch=1, executor=ex) as s:
        bad = vol((8, 8, 8), 0)
        bad[0, 0, 0] = np.nan
        fb = s.submit(bad, 42, 16)
        fg = s.submit(vol((8, 8, 8), 1), 42, 16)
        fo = s.submit(vol((8, 8, 8), 2), 7, 16)      # no such orientation set
        fz = s.submit(vol((8, 8), 3), 42, 16)        # not a volume
        fq = s.submit(vol((8, 8, 8), 4), 42, 16, op="nonsense")
        with pytest.raises(ValueError):
            fb.result(timeout=5)
        with pytest.raises(ValueError):
            fo.result(timeout=5)
        with pytest.raises(ValueError):
            fz.result(timeout=5)
        with pytest.raises(ValueError):
            fq.result(timeout=5)
        fg.result(timeout=5)


def test_bank_build_failure_fails_only_that_key():
    ex = FakeExecutor(2, fail_keys=[((8, 8, 8), 162, 24)])
    with Server(1 << 30, n_slots=2, executor=ex) as s:
        f1 = s.submit(vol((8, 8, 8), 0), 162, 24)
        f2 = s.submit(vol((8, 8, 8), 1), 42, 16)
        with pytest.raises(RuntimeError, match="bank build failed"):
            f1.result(timeout=5)
        f2.result(timeout=5)


def test_cancel_before_admission_and_timeout_while_pending():
    ex = FakeExecutor(1, run_s=0.2)
    with Server(1 << 30, n_slots=1, max_batch=1, executor=ex) as s:
        first = s.submit(vol((8, 8, 8), 0), 42, 16)
        time.sleep(0.02)
        c = s.submit(vol((8, 8, 8), 1), 42, 16)
        t = s.submit(vol((8, 8, 8), 2), 12, 8, timeout=0.05)
        assert c.cancel()
        with pytest.raises(JobTimeout):
            t.result(timeout=5)
        first.result(timeout=5)
    assert all(1 not in b for b in ex.launches)


def test_lru_bank_eviction_and_hit_rate():
    """Room for one job and two cached banks: the least recently used idle
    bank is dropped when a third key arrives."""
    ex = FakeExecutor(1, run_s=0.001)
    V = 512
    job, bank = 42 * V * 8 + 4 * V * 8, V * 42 * 2
    with Server(job + 2 * bank + 100, n_slots=1, executor=ex) as s:
        for i, L in enumerate([8, 16, 8, 24, 8, 16]):
            s.submit(vol((8, 8, 8), i), 42, L).result(timeout=5)
        st = s.stats()
        evicted = list(ex.freed)
    assert evicted == [((8, 8, 8), 42, 16), ((8, 8, 8), 42, 24)]
    # closing the server released the two banks still cached
    assert sorted(ex.freed[2:]) == [((8, 8, 8), 42, 8), ((8, 8, 8), 42, 16)]
    assert (st["bank_hits"], st["bank_misses"], st["bank_evictions"]) == (2, 4, 2)
    assert st["peak_bytes"] <= job + 2 * bank + 100


def test_oldest_job_is_not_starved():
    """A large job that needs the whole budget is admitted before small jobs
    that arrive after it has waited past the starvation limit."""
    ex = FakeExecutor(2, run_s=0.03)
    big_fp = fp((12, 12, 12), 42)
    with Server(big_fp + 100, n_slots=2, max_batch=1, executor=ex, starvation_s=0.05) as s:
        s.submit(vol((8, 8, 8), 0), 12, 8)
        time.sleep(0.005)
        big = s.submit(vol((12, 12, 12), 1), 42, 16)
        late = []
        for i in range(12):
            time.sleep(0.01)
            late.append(s.submit(vol((8, 8, 8), 2 + i), 12, 8))
        big.result(timeout=5)
        for f in late:
            f.result(timeout=5)
    ids = [b[0] for b in ex.launches]
    # job 1 (the big one) runs before the small jobs submitted 0.05 s after it
    assert ids.index(1) < ids.index(1 + 8)


def test_close_drains_and_rejects_new_work():
    ex = FakeExecutor(2, run_s=0.01)
    s = Server(1 << 30, n_slots=2, executor=ex)
    futs = [s.submit(vol((8, 8, 8), i), 42, 16) for i in range(4)]
    s.close()
    assert all(f.done() and not f.exception() for f in futs)
    with pytest.raises(RuntimeError):
        s.submit(vol((8, 8, 8), 9), 42, 16)


def test_batch_bytes_caps_batches_of_large_jobs():
    """Small jobs share launches; jobs whose batch would exceed batch_bytes
    run one per launch."""
    ex = FakeExecutor(1, run_s=0.03)
    V = 512
    one = 42 * V * 8 + 4 * V * 8
    with Server(1 << 30, n_slots=1, max_batch=8, executor=ex, batch_bytes=3 * one) as s:
        first = s.submit(vol((8, 8, 8), 0), 42, 16)
        time.sleep(0.01)
        futs = [s.submit(vol((8, 8, 8), 1 + i), 42, 16) for i in range(6)]
        for f in [first] + futs:
            f.result(timeout=5)
    # job_bytes(n) = n * 42 V 8 + ws: at most 3 jobs fit in 3 * one
    assert max(len(b) for b in ex.launches) == 3


def test_waits_for_running_jobs_instead_of_evicting():
    """When the running launch will free enough memory, a new key waits for
    it rather than dropping a cached bank."""
    ex = FakeExecutor(2, run_s=0.05)
    V = 512
    job, bank = 42 * V * 8 + 4 * V * 8, V * 42 * 2
    with Server(2 * job + 2 * bank + 100, n_slots=2, max_batch=1, executor=ex) as s:
        s.submit(vol((8, 8, 8), 0), 42, 8).result(timeout=5)      # bank A cached, idle
        a = s.submit(vol((8, 8, 8), 1), 42, 16)                   # bank B + a running job
        time.sleep(0.01)
        b = s.submit(vol((8, 8, 8), 2), 42, 24)                   # bank C: fits only after `a`
        a.result(timeout=5)
        b.result(timeout=5)
        st = s.stats()
        assert st["bank_evictions"] == 0 and ex.freed == []
    assert st["ok"] == 3 and st["errors"] == {}


def test_a_slow_bank_build_does_not_stall_other_keys():
    """A bank is built on a thread of its own: while one key's bank takes
    0.5 s, jobs of a key whose bank is cached are still reaped and
    admitted."""
    slow = ((16, 16, 16), 162, 24)
    ex = FakeExecutor(2, run_s=0.01, build_s={slow: 0.5})
    with Server(1 << 30, n_slots=2, max_batch=1, executor=ex) as s:
        s.submit(vol((8, 8, 8), 0), 42, 16).result(timeout=5)  # caches the fast key's bank
        t0 = time.perf_counter()
        fs = s.submit(vol((16, 16, 16), 1), 162, 24)
        time.sleep(0.02)
        fast = [s.submit(vol((8, 8, 8), 2 + i), 42, 16) for i in range(5)]
        for f in fast:
            f.result(timeout=5)
        t_fast = time.perf_counter() - t0
        assert not fs.done()
        fs.result(timeout=5)
        st = s.stats()
    assert t_fast < 0.3, t_fast
    assert st["ok"] == 7 and st["bank_builds"] == 2 and st["bank_build_ms_max"] >= 500


def test_results_are_handed_to_the_submitting_stream():
    """An executor that knows streams gets each result handed over to the
    stream its job was submitted from, before the Future resolves."""
    class StreamExecutor(FakeExecutor):
        def __init__(self, *a, **k):
            super().__init__(*a, **k)
            self.handed = []

        def consumer_stream(self, volume):
            return ("stream of", threading.get_ident())

        def hand_over(self, result, stream):
            self.handed.append((id(result), stream))

    ex = StreamExecutor(2, run_s=0.005)
    with Server(1 << 30, n_slots=2, executor=ex) as s:
        futs = [s.submit(vol((8, 8, 8), i), 42, 16) for i in range(3)]
        outs = [f.result(timeout=5) for f in futs]
    assert sorted(h[0] for h in ex.handed) == sorted(id(o) for o in outs)
    assert all(h[1] == ("stream of", threading.get_ident()) for h in ex.handed)


def test_a_failed_build_left_in_the_cache_is_evictable():
    """A bank build that fails after its only job has timed out leaves an
    entry without a bank in the cache; when a later job needs the room, the
    entry is dropped and nothing is freed for it."""
    bad = ((16, 16, 16), 42, 16)
    ex = FakeExecutor(1, run_s=0.005, fail_keys={bad}, build_s={bad: 0.3})
    big = (32, 32, 32)
    budget = fp(big, 42) + 1024  # room for one bank and one job of the big shape only
    with Server(budget, n_slots=1, executor=ex) as s:
        f_bad = s.submit(vol((16, 16, 16), 1), 42, 16, timeout=0.05)
        with pytest.raises(JobTimeout):
            f_bad.result(timeout=5)
        time.sleep(0.4)  # the build has failed by now, with no job of its key left
        assert np.array_equal(s.submit(vol(big, 2), 42, 16).result(timeout=5), 2 * vol(big, 2))
        st = s.stats()
    assert st["bank_evictions"] >= 1
    assert None not in ex.freed and bad not in ex.freed


def test_budget_is_capped_at_the_free_device_memory():
    """A budget beyond what the device has free would make the allocator
    release and re-reserve memory mid-stream: the server takes 90 % of the
    free bytes the executor reports, and keeps the requested value."""

    class Small(FakeExecutor):
        def device_bytes_available(self):
            return 10 << 30

    with Server(64 << 30, n_slots=1, executor=Small(1)) as s:
        assert s.budget == int(0.9 * (10 << 30))
        assert s.budget_requested == 64 << 30
    with Server(4 << 30, n_slots=1, executor=Small(1)) as s:
        assert s.budget == 4 << 30
    with Server(64 << 30, n_slots=1, executor=FakeExecutor(1)) as s:  # no report: no cap
        assert s.budget == 64 << 30


def test_close_releases_the_cached_banks():
    """A closed server holds no device memory: every cached bank is freed
    once the submitted work has finished (a later server in the same
    process then starts from the memory the first one used)."""
    ex = FakeExecutor(2)
    s = Server(1 << 30, n_slots=2, executor=ex)
    futs = [s.submit(vol((8, 8, 8), i), 12, 8) for i in range(3)] + [s.submit(vol((8, 8, 12), 9), 42, 8)]
    s.close()
    assert all(f.done() and f.exception() is None for f in futs)
    assert sorted(ex.freed) == sorted(ex.built)
    assert len(ex.built) == 2
    assert s._used == 0 and not s._banks


class ScratchExecutor(FakeExecutor):
    """A fake executor whose slots keep scratch (half of a launch's
    footprint) from one launch to the next, as the GPU executor does."""

    def __init__(self, n_slots, **kw):
        super().__init__(n_slots, **kw)
        self.slot_bytes = [0] * n_slots
        self.released = []

    def scratch_bytes(self, key, bank, B, op, dtype):
        return self.job_bytes(key, bank, B, op, dtype) // 2

    def release_scratch(self, slot):
        self.released.append(slot)
        self.slot_bytes[slot] = 0

    def grow_scratch(self, slot, nbytes):
        self.slot_bytes[slot] = max(self.slot_bytes[slot], nbytes)

    def launch(self, slot, bank, jobs):
        need = self.scratch_bytes(jobs[0].key, bank, len(jobs), jobs[0].op, jobs[0].dtype)
        self.slot_bytes[slot] = max(self.slot_bytes[slot], need)
        return super().launch(slot, bank, jobs)


def test_slot_scratch_is_reused_and_counted():
    """A slot's scratch stays counted against the budget between launches,
    a second job of the same size reuses it (no growth), the accounting
    matches what the executor holds, and closing the server gives it back."""
    ex = ScratchExecutor(1, run_s=0.001)
    key = ((8, 8, 8), 42, 8)
    bank = ex.bank_bytes(key)
    job = ex.job_bytes(key, FakeBank(key), 1, "reconstruct", "c64")
    s = Server(1 << 30, n_slots=1, executor=ex)
    for i in range(3):
        s.submit(vol((8, 8, 8), i), 42, 8).result(timeout=5)
    time.sleep(0.01)
    assert s._scratch_acc == [job // 2] == ex.slot_bytes
    assert s._used == bank + job // 2
    assert s.peak_bytes == bank + job
    s.close()
    assert s._used == 0 and ex.released == [0]


def test_idle_scratch_is_released_before_a_bank_is_dropped():
    """Two slots hold the scratch of two finished jobs; a larger job of
    another key needs room: the idle slot's scratch goes back first and the
    cached bank of the first key stays."""
    ex = ScratchExecutor(2, run_s=0.05)
    ka, kb = ((8, 8, 8), 42, 8), ((8, 8, 16), 42, 8)
    bank_a, bank_b = ex.bank_bytes(ka), ex.bank_bytes(kb)
    job_a = ex.job_bytes(ka, FakeBank(ka), 1, "reconstruct", "c64")
    job_b = ex.job_bytes(kb, FakeBank(kb), 1, "reconstruct", "c64")
    # room for both banks, one slot's scratch of `a` grown to `b`'s and b's
    # transient half, but not for the second slot's scratch of `a` on top
    budget = bank_a + bank_b + job_b + job_a // 2 - 1
    with Server(budget, n_slots=2, max_batch=1, executor=ex) as s:
        f1, f2 = s.submit(vol((8, 8, 8), 0), 42, 8), s.submit(vol((8, 8, 8), 1), 42, 8)
        f1.result(timeout=5)
        f2.result(timeout=5)
        time.sleep(0.02)
        assert sorted(s._scratch_acc) == [job_a // 2, job_a // 2]
        s.submit(vol((8, 8, 16), 2), 42, 8).result(timeout=5)
        st = s.stats()
        assert ex.freed == [] and st["bank_evictions"] == 0
        assert len(ex.released) == 1
        assert st["peak_bytes"] <= budget


def test_reserve_scratch_sizes_every_slot_before_a_burst():
    """reserve_scratch sizes every slot for the largest cached key, counted
    against the budget, so that a burst's first launches need no growth."""
    ex = ScratchExecutor(3, run_s=0.002)
    ka, kb = ((8, 8, 8), 42, 8), ((8, 8, 16), 162, 8)
    with Server(1 << 30, n_slots=3, max_batch=1, executor=ex) as s:
        s.submit(vol((8, 8, 8), 0), 42, 8).result(timeout=5)
        s.submit(vol((8, 8, 16), 1), 162, 8).result(timeout=5)
        want = ex.job_bytes(kb, FakeBank(kb), 1, "reconstruct", "c64") // 2
        assert s.reserve_scratch() == want
        assert ex.slot_bytes == [want] * 3 and s._scratch_acc == [want] * 3
        assert s._used == ex.bank_bytes(ka) + ex.bank_bytes(kb) + 3 * want
        grown = list(ex.slot_bytes)
        futs = [s.submit(vol((8, 8, 16), 2 + i), 162, 8) for i in range(6)]
        for f in futs:
            f.result(timeout=5)
        assert ex.slot_bytes == grown and s._scratch_acc == [want] * 3
    assert s._used == 0


def test_reserve_scratch_edges():
    """reserve_scratch with an executor that keeps no scratch returns 0;
    keys that are not cached reserve nothing; a budget with room for only
    some slots grows only those (the rest stay as they were, the budget is
    never exceeded); a closed server refuses."""
    with Server(1 << 30, n_slots=2, executor=FakeExecutor(2)) as s:
        assert s.reserve_scratch() == 0
    ex = ScratchExecutor(3, run_s=0.001)
    key = ((8, 8, 8), 42, 8)
    bank = ex.bank_bytes(key)
    half = ex.job_bytes(key, FakeBank(key), 1, "reconstruct", "c64") // 2
    # the bank, one slot's scratch from a first job and room for one more
    s = Server(bank + 2 * half + half // 2, n_slots=3, max_batch=1, executor=ex)
    s.submit(vol((8, 8, 8), 0), 42, 8).result(timeout=5)
    assert s.reserve_scratch(keys=[((8, 8, 16), 42, 8)]) == 0  # not cached
    assert s.reserve_scratch() == half
    assert sorted(s._scratch_acc) == [0, half, half] and sorted(ex.slot_bytes) == [0, half, half]
    assert s._used == bank + 2 * half <= s.budget
    s.close()
    assert s._used == 0
    with pytest.raises(RuntimeError):
        s.reserve_scratch()
