"""CPU tests of the serving scheduler (queueing, admission by memory, slot
reuse, cancellation, errors, time stamps) through a fake executor."""
import ctypes as C
import os
import subprocess
import threading
import time

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2501_09308_amd", "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD, "libsched_fake.so")

OK, PENDING, EINVAL, ENOMEM, EDEVICE, EBUSY, ENOENT, ECANCELED, ENONFINITE = \
    0, 1, -1, -2, -3, -4, -5, -6, -7


@pytest.fixture(scope="module")
def lib():
    os.makedirs(BUILD, exist_ok=True)
    subprocess.check_call(
        ["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-pthread",
         "-I", CSRC, os.path.join(CSRC, "scheduler.cpp"),
         os.path.join(HERE, "native", "sched_fake.cpp"), "-o", LIB + ".tmp"])
    os.replace(LIB + ".tmp", LIB)
    l = C.CDLL(LIB)
    l.fake_create.restype = C.c_void_p
    l.fake_create.argtypes = [C.c_size_t, C.c_int, C.c_int, C.c_int, C.c_int]
    l.fake_submit.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_uint64,
                              C.c_void_p, C.c_void_p, C.POINTER(C.c_uint64)]
    l.fake_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_double)]
    l.fake_cancel.argtypes = [C.c_void_p, C.c_uint64]
    l.fake_stats.argtypes = [C.c_void_p] + [C.POINTER(C.c_int)] * 3
    l.fake_destroy.argtypes = [C.c_void_p]
    l.fake_changes.argtypes = [C.c_void_p] + [C.POINTER(C.c_int)] * 2
    l.fake_create_budget.restype = C.c_void_p
    l.fake_create_budget.argtypes = [C.c_size_t, C.c_int, C.c_int, C.c_int,
                                     C.c_int, C.c_size_t]
    l.fake_max_resident.restype = C.c_size_t
    l.fake_max_resident.argtypes = [C.c_void_p]
    return l


class Fake:
    def __init__(self, lib, arena=1 << 20, slots=4, queue=1000, steps=5, sleep_us=200,
                 resident=None):
        self.lib = lib
        if resident is None:
            self.h = lib.fake_create(arena, slots, queue, steps, sleep_us)
        else:
            self.h = lib.fake_create_budget(arena, slots, queue, steps, sleep_us,
                                            resident)
        self.bufs = {}

    def submit(self, K=8, N=100, steps=20, seed=1):
        loc = np.full(4 * K, np.nan)
        tr = np.full(steps, np.nan)
        t = C.c_uint64()
        rc = self.lib.fake_submit(self.h, K, N, steps, seed, loc.ctypes.data,
                                  tr.ctypes.data, C.byref(t))
        if rc == OK:
            self.bufs[t.value] = (loc, tr)
        return rc, t.value

    def poll(self, t):
        info = (C.c_double * 6)()
        rc = self.lib.fake_poll(self.h, t, info)
        return rc, list(info)

    def wait(self, tickets, timeout=20.0):
        res, t0 = {}, time.time()
        while len(res) < len(tickets):
            for t in tickets:
                if t in res:
                    continue
                rc, info = self.poll(t)
                if rc != PENDING:
                    res[t] = (rc, info)
            assert time.time() - t0 < timeout, "scheduler did not finish"
            time.sleep(0.001)
        return res

    def stats(self):
        a, r, u = C.c_int(), C.c_int(), C.c_int()
        self.lib.fake_stats(self.h, C.byref(a), C.byref(r), C.byref(u))
        return a.value, r.value, u.value

    def close(self):
        self.lib.fake_destroy(self.h)


def test_all_complete_with_routed_outputs_and_batching(lib):
    f = Fake(lib, slots=4)
    tickets = [f.submit(K=4 + i % 3, steps=10 + i)[1] for i in range(12)]
    res = f.wait(tickets)
    for t in tickets:
        rc, info = res[t]
        assert rc == OK
        loc, tr = f.bufs[t]
        assert np.array_equal(loc, t * 1000.0 + np.arange(len(loc)))
        assert np.array_equal(tr, np.arange(len(tr)))
        assert info[1] == len(tr) and info[5] == -t
        assert 0 <= info[2] <= info[3] <= info[4]
    max_active, runs, used = f.stats()
    assert max_active == 4          # continuous batching up to the slot limit
    assert used <= 4                 # slots are reused
    f.close()


def test_slot_reuse_is_announced_as_a_membership_change(lib):
    # one slot: every job runs in slot 0, so the slot-id set never changes;
    # the scheduler must still flag each new resident (regression: a stale
    # per-slot work prefix made batched kernels index past a smaller job)
    f = Fake(lib, slots=1, steps=4, sleep_us=100)
    tickets = [f.submit(K=3 + i, N=50 + 10 * i, steps=8)[1] for i in range(6)]
    f.wait(tickets)
    missed, changed = C.c_int(), C.c_int()
    lib.fake_changes(f.h, C.byref(missed), C.byref(changed))
    assert missed.value == 0
    assert changed.value >= 6
    f.close()


def test_membership_changes_announced_under_churn(lib):
    f = Fake(lib, slots=5, steps=3, sleep_us=100)
    tickets = [f.submit(K=2 + i % 7, steps=3 + (i * 7) % 11)[1] for i in range(40)]
    f.wait(tickets)
    missed, changed = C.c_int(), C.c_int()
    lib.fake_changes(f.h, C.byref(missed), C.byref(changed))
    assert missed.value == 0
    f.close()


def test_admission_in_arrival_order(lib):
    f = Fake(lib, slots=2, steps=5, sleep_us=500)
    tickets = [f.submit(steps=10)[1] for _ in range(8)]
    res = f.wait(tickets)
    admits = [res[t][1][3] for t in tickets]
    assert admits == sorted(admits)
    f.close()


def test_memory_admission_and_never_fits(lib):
    # each K=8, N=100 job needs 9792 bytes (10 KiB after rounding);
    # an arena of 25 KiB holds two at a time even with 8 slots
    f = Fake(lib, arena=25 << 10, slots=8, sleep_us=300)
    tickets = [f.submit(K=8, N=100, steps=15)[1] for _ in range(6)]
    res = f.wait(tickets)
    assert all(r[0] == OK for r in res.values())
    assert f.stats()[0] == 2
    rc, _ = f.submit(K=100, N=100)   # 104000 bytes > arena
    assert rc == ENOMEM
    f.close()


def test_queue_full_is_busy(lib):
    f = Fake(lib, slots=1, queue=3, sleep_us=20000)
    rcs = [f.submit(steps=1000)[0] for _ in range(6)]
    assert EBUSY in rcs
    f.close()


def test_cancel_pending_and_running(lib):
    f = Fake(lib, slots=1, steps=1, sleep_us=2000)
    rc, running = f.submit(steps=100000)
    rc, queued = f.submit(steps=5)
    time.sleep(0.02)
    assert lib.fake_cancel(f.h, queued) == OK
    assert lib.fake_cancel(f.h, running) == OK
    res = f.wait([running, queued])
    assert res[queued][0] == ECANCELED and res[running][0] == ECANCELED
    assert np.all(np.isnan(f.bufs[queued][0]))     # outputs untouched
    assert np.all(np.isnan(f.bufs[running][0]))
    assert lib.fake_cancel(f.h, 999999) == ENOENT
    f.close()


def test_errors_do_not_poison_others(lib):
    f = Fake(lib, slots=4)
    good = [f.submit(seed=1)[1] for _ in range(3)]
    bad_start = f.submit(seed=13)[1]
    bad_nan = f.submit(seed=666)[1]
    res = f.wait(good + [bad_start, bad_nan])
    assert all(res[t][0] == OK for t in good)
    assert res[bad_start][0] == EDEVICE
    assert res[bad_nan][0] == ENONFINITE
    f.close()


def test_terminal_state_reported_once(lib):
    f = Fake(lib)
    t = f.submit(steps=3)[1]
    assert f.wait([t])[t][0] == OK
    assert f.poll(t)[0] == ENOENT
    f.close()


def test_concurrent_submitters(lib):
    f = Fake(lib, slots=8, sleep_us=100)
    out, lock = [], threading.Lock()

    def worker():
        for _ in range(25):
            rc, t = f.submit(steps=7)
            assert rc == OK
            with lock:
                out.append(t)

    th = [threading.Thread(target=worker) for _ in range(4)]
    [x.start() for x in th]
    [x.join() for x in th]
    assert len(set(out)) == 100
    res = f.wait(out, timeout=60)
    assert all(r[0] == OK for r in res.values())
    f.close()


def test_destroy_with_work_in_flight(lib):
    f = Fake(lib, slots=2, sleep_us=1000)
    for _ in range(10):
        f.submit(steps=100000)
    time.sleep(0.01)
    f.close()       # cancels and joins without hanging


def test_scheduler_stress_under_sanitizers():
    """Concurrent submit/cancel/poll and destruction with work in flight,
    built with AddressSanitizer and UBSan (host code only)."""
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "sched_stress")
    subprocess.check_call(
        ["g++", "-O1", "-g", "-std=c++17", "-pthread",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-I", CSRC,
         os.path.join(CSRC, "scheduler.cpp"),
         os.path.join(HERE, "native", "sched_stress.cpp"), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok=" in r.stdout


def test_resident_budget_caps_the_working_set(lib):
    # each job K=8, N=100 occupies 8*1024 + 1600 = 9792 bytes (256-byte
    # rounding aside); a budget of 2.5 jobs keeps at most 2 resident even
    # with 8 free slots, and every job still completes
    fp = 8 * 1024 + 100 * 16
    f = Fake(lib, slots=8, steps=4, sleep_us=100, resident=int(2.5 * fp))
    ts = [f.submit(steps=12, seed=i)[1] for i in range(10)]
    res = f.wait(ts)
    assert all(r[0] == OK for r in res.values())
    assert lib.fake_max_resident(f.h) <= int(2.5 * fp)
    assert f.stats()[0] == 2
    f.close()


def test_resident_budget_admits_one_oversized_job(lib):
    fp = 8 * 1024 + 100 * 16
    f = Fake(lib, slots=4, steps=4, sleep_us=100, resident=fp // 2)
    ts = [f.submit(steps=8, seed=i)[1] for i in range(3)]
    res = f.wait(ts)
    assert all(r[0] == OK for r in res.values())
    assert f.stats()[0] == 1
    f.close()

