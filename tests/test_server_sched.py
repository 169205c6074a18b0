"""The server's scheduling core on the host (no GPU): admission by memory
footprint, least-recently-used residency, continuous batching, the plain
mode, failed builds, and a seeded random run checked against invariants."""
import ctypes as C
import os
import random
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
U64 = C.c_ulonglong


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = tmp_path_factory.mktemp("shim") / "libshim.so"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-shared", "-fPIC", "-o", str(out),
                    os.path.join(HERE, "sched_shim.cpp")], check=True)
    L = C.CDLL(str(out))
    L.shim_create.restype = C.c_void_p
    L.shim_create.argtypes = [C.c_longlong, C.c_int, C.c_int, C.c_int, C.c_int]
    for n in ("shim_used", "shim_resident", "shim_evictions"):
        getattr(L, n).restype = C.c_longlong
        getattr(L, n).argtypes = [C.c_void_p]
    for n in ("shim_inflight", "shim_pending", "shim_waiting", "shim_idle"):
        getattr(L, n).argtypes = [C.c_void_p]
    L.shim_has_part.argtypes = [C.c_void_p, U64]
    L.shim_pins.argtypes = [C.c_void_p, U64]
    L.shim_destroy.argtypes = [C.c_void_p]
    L.shim_submit.argtypes = [C.c_void_p, U64, U64, C.c_longlong, C.c_longlong, C.c_longlong]
    L.shim_admit.argtypes = [C.c_void_p] + [C.POINTER(U64)] * 5 + [C.c_int, C.POINTER(C.c_int)]
    L.shim_build_done.argtypes = [C.c_void_p, U64, C.c_int, C.POINTER(U64), C.c_int]
    L.shim_batch_failed.argtypes = [C.c_void_p, C.POINTER(U64), C.c_int, C.POINTER(U64), C.c_int]
    L.shim_cancel.argtypes = [C.c_void_p, U64, C.POINTER(U64), C.c_int, C.POINTER(C.c_int)]
    L.shim_broken.argtypes = [C.c_void_p, U64]
    L.shim_next_batch.argtypes = [C.c_void_p, C.POINTER(U64), C.c_int]
    L.shim_batch_done.argtypes = [C.c_void_p, C.POINTER(U64), C.c_int, C.POINTER(U64), C.c_int]
    return L


class Sched:
    CAP = 4096

    def __init__(self, L, budget, max_batch=64, max_inflight=2, plain=False, keep=True):
        self.L = L
        self.p = L.shim_create(budget, max_batch, max_inflight, int(plain), int(keep))

    def submit(self, t, key, part, build, stage):
        self.L.shim_submit(self.p, t, key, part, build, stage)

    def admit(self):
        arrs = [(U64 * self.CAP)() for _ in range(5)]
        cnt = (C.c_int * 5)()
        self.L.shim_admit(self.p, *arrs, self.CAP, cnt)
        names = ("evict", "build", "admitted", "hits", "rejected")
        return {n: list(a[:c]) for n, a, c in zip(names, arrs, cnt)}

    def build_done(self, key, ok=True):
        r = (U64 * self.CAP)()
        n = self.L.shim_build_done(self.p, key, int(ok), r, self.CAP)
        return list(r[:n])

    def batch_failed(self, tickets):
        t = (U64 * len(tickets))(*tickets)
        r = (U64 * self.CAP)()
        n = self.L.shim_batch_failed(self.p, t, len(tickets), r, self.CAP)
        return list(r[:n])

    def cancel(self, ticket):
        r = (U64 * self.CAP)()
        n = C.c_int()
        ok = self.L.shim_cancel(self.p, ticket, r, self.CAP, C.byref(n))
        return bool(ok), list(r[:n.value])

    def next_batch(self):
        a = (U64 * self.CAP)()
        n = self.L.shim_next_batch(self.p, a, self.CAP)
        return list(a[:n])

    def batch_done(self, tickets):
        t = (U64 * len(tickets))(*tickets)
        r = (U64 * self.CAP)()
        n = self.L.shim_batch_done(self.p, t, len(tickets), r, self.CAP)
        return list(r[:n])

    def __getattr__(self, name):
        f = getattr(self.L, "shim_" + name)
        return lambda *a: f(self.p, *a)

    def close(self):
        self.L.shim_destroy(self.p)


def test_admission_stops_at_budget_and_resumes(shim):
    s = Sched(shim, 1000)
    for t in range(1, 4):
        s.submit(t, 100 + t, 200, 50, 100)        # needs 350 each while building
    a = s.admit()
    assert a["admitted"] == [1, 2] and a["build"] == [101, 102] and not a["rejected"]
    assert s.used() == 700 and s.pending() == 1
    s.build_done(101)
    s.build_done(102)                              # scratch released: 600 in use
    assert s.used() == 600
    a = s.admit()
    assert a["admitted"] == [3] and s.used() == 950
    s.close()


def test_resident_hit_skips_build(shim):
    s = Sched(shim, 10_000)
    s.submit(1, 7, 500, 100, 50)
    assert s.admit()["build"] == [7]
    s.build_done(7)
    b = s.next_batch()
    assert b == [1]
    assert s.batch_done(b) == []                   # kept resident
    assert s.has_part(7) and s.pins(7) == 0 and s.used() == 500
    s.submit(2, 7, 500, 100, 50)
    a = s.admit()
    assert a["build"] == [] and a["hits"] == [2] and s.used() == 550
    s.close()


def test_lru_evicts_oldest_unpinned_first(shim):
    s = Sched(shim, 1000)
    for t, key in ((1, 11), (2, 12), (3, 13)):
        s.submit(t, key, 300, 0, 10)
        s.admit()
        s.build_done(key)
        s.batch_done(s.next_batch())
    assert s.resident() == 900 and s.used() == 900
    # touch 11 again so 12 becomes the oldest
    s.submit(4, 11, 300, 0, 10)
    assert s.admit()["hits"] == [4]
    s.batch_done(s.next_batch())
    s.submit(5, 14, 300, 0, 10)                   # needs 310: one eviction
    a = s.admit()
    assert a["evict"] == [12] and a["build"] == [14]
    assert not s.has_part(12) and s.evictions() == 1
    s.close()


def test_pinned_parts_are_never_evicted(shim):
    s = Sched(shim, 1000)
    s.submit(1, 21, 600, 0, 10)
    s.admit()
    s.build_done(21)                               # pinned by ticket 1 until its batch ends
    s.submit(2, 22, 600, 0, 10)
    a = s.admit()
    assert a["evict"] == [] and a["admitted"] == [] and s.has_part(21)
    b = s.next_batch()
    s.batch_done(b)                                # 21 unpinned now
    a = s.admit()
    assert a["evict"] == [21] and a["admitted"] == [2]
    s.close()


def test_request_larger_than_budget_is_rejected_only_when_alone(shim):
    s = Sched(shim, 1000)
    s.submit(1, 31, 400, 0, 10)
    s.admit()
    s.submit(2, 32, 2000, 0, 10)                   # can never fit
    s.submit(3, 33, 100, 0, 10)
    a = s.admit()
    assert a["rejected"] == [] and a["admitted"] == []   # waits behind ticket 1's memory
    s.build_done(31)
    s.batch_done(s.next_batch())
    a = s.admit()
    assert a["rejected"] == [2] and a["admitted"] == [3]
    s.close()


def test_continuous_batching_windows(shim):
    s = Sched(shim, 1 << 40, max_batch=4, max_inflight=2)
    for t in range(1, 11):
        s.submit(t, 500 + t, 10, 1, 1)
    assert s.admit()["admitted"] == [1, 2, 3, 4]   # one batch worth waits admitted
    b1 = s.next_batch()
    assert b1 == [1, 2, 3, 4]
    assert s.admit()["admitted"] == [5, 6, 7, 8]   # admitted while b1 runs
    b2 = s.next_batch()
    assert b2 == [5, 6, 7, 8] and s.inflight() == 2
    assert s.admit()["admitted"] == [9, 10]
    assert s.next_batch() == []                    # two batches on the device already
    s.batch_done(b1)
    assert s.next_batch() == [9, 10]
    s.batch_done(b2)
    s.close()


def test_plain_mode_is_one_at_a_time_and_keeps_nothing(shim):
    s = Sched(shim, 1 << 40, max_batch=64, max_inflight=4, plain=True)
    for t in range(1, 4):
        s.submit(t, 41, 100, 10, 5)                # same part every time
    a = s.admit()
    assert a["admitted"] == [1] and a["build"] == [41]
    assert s.admit()["admitted"] == []             # still building
    s.build_done(41)
    assert s.admit()["admitted"] == []             # waiting for launch
    b = s.next_batch()
    assert b == [1]
    assert s.batch_done(b) == [41]                 # released, not kept
    a = s.admit()
    assert a["admitted"] == [2] and a["build"] == [41] and a["hits"] == []
    s.close()


def test_failed_build_releases_part(shim):
    s = Sched(shim, 1 << 30)
    s.submit(1, 51, 100, 10, 5)
    s.submit(2, 51, 100, 10, 5)
    s.admit()
    s.build_done(51, ok=False)
    b = s.next_batch()
    assert b == [1, 2]
    assert s.batch_done(b) == [51] and not s.has_part(51) and s.used() == 0
    s.close()


def test_random_run_invariants(shim):
    """Seeded random arrivals, completions and build ends; after every step
    the bytes in use never exceed the budget, admission follows arrival
    order, every request ends exactly once, and at the end nothing is held
    but the resident parts."""
    rng = random.Random(1234)
    budget = 5000
    s = Sched(shim, budget, max_batch=5, max_inflight=2)
    parts = {k: rng.randint(100, 1500) for k in range(20)}
    next_ticket, submitted, admitted_order = 1, [], []
    building, inflight, ended, rejected = set(), [], set(), set()
    for step in range(3000):
        r = rng.random()
        if r < 0.35 and next_ticket <= 600:
            k = min(int(rng.paretovariate(1.1)) - 1, 19)
            s.submit(next_ticket, k, parts[k], parts[k] // 4, rng.randint(10, 400))
            submitted.append(next_ticket)
            next_ticket += 1
        elif r < 0.55:
            a = s.admit()
            admitted_order += a["admitted"] + a["rejected"]
            building.update(a["build"])
            rejected.update(a["rejected"])
        elif r < 0.7 and building:
            k = rng.choice(sorted(building))
            building.discard(k)
            s.build_done(k, ok=rng.random() > 0.02)
        elif r < 0.85:
            b = s.next_batch()
            if b:
                inflight.append(b)
        elif inflight:
            b = inflight.pop(rng.randrange(len(inflight)))
            s.batch_done(b)
            for t in b:
                assert t not in ended
                ended.add(t)
        assert 0 <= s.used() <= budget, step
        assert s.inflight() == len(inflight)
    # drain
    for _ in range(10000):
        if s.idle():
            break
        a = s.admit()
        admitted_order += a["admitted"] + a["rejected"]
        building.update(a["build"])
        rejected.update(a["rejected"])
        for k in sorted(building):
            s.build_done(k)
        building.clear()
        b = s.next_batch()
        if b:
            inflight.append(b)
        if inflight:
            b = inflight.pop(0)
            s.batch_done(b)
            ended.update(b)
        assert 0 <= s.used() <= budget
    assert s.idle()
    assert admitted_order == submitted                 # arrival order
    assert ended | rejected == set(submitted) and not (ended & rejected)
    assert s.used() == s.resident()                    # only resident hierarchies remain
    s.close()


# ---------------------------------------------------------------- faults and cancellation
def test_cancel_pending_admitted_and_launched(shim):
    s = Sched(shim, 10_000)
    for t in (1, 2, 3):
        s.submit(t, 40 + t, 300, 100, 50)
    s.submit(4, 41, 300, 100, 50)                  # a second request on part 41
    a = s.admit()
    assert a["admitted"] == [1, 2, 3, 4]
    s.submit(5, 45, 300, 100, 50)                  # still pending (not admitted yet)
    ok, rel = s.cancel(5)
    assert ok and rel == [] and s.pending() == 0
    for k in (41, 42, 43):
        s.build_done(k)
    used = s.used()
    ok, rel = s.cancel(2)                          # admitted, not launched: working set and pin back
    assert ok and rel == [] and s.used() == used - 50 and s.pins(42) == 0
    b = s.next_batch()
    assert b == [1, 3, 4]
    ok, _ = s.cancel(3)                            # launched: not cancellable
    assert not ok and s.pins(43) == 1
    assert s.cancel(99) == (False, [])             # unknown ticket
    s.batch_done(b)
    assert s.idle() and s.used() == 3 * 300        # three parts resident
    s.close()


def test_cancel_while_building_releases_at_build_done(shim):
    s = Sched(shim, 10_000, keep=False)
    s.submit(1, 51, 400, 200, 30)
    assert s.admit()["build"] == [51]
    ok, rel = s.cancel(1)
    assert ok and rel == []                        # the build still runs: nothing freed yet
    assert s.has_part(51) and not s.idle()
    assert s.build_done(51) == [51]                # released when the build ends
    assert not s.has_part(51) and s.used() == 0 and s.idle()
    s.close()


def test_device_error_on_batch_k(shim):
    """Batches 0..5 over three parts; the device error word of batch 3 is
    set: its requests fail, its parts are dropped once unpinned and rebuilt
    on their next use; everything else is unaffected and the accounting
    returns to the resident parts alone."""
    s = Sched(shim, 100_000, max_batch=2)
    t = 0
    rebuilt = []
    for k in range(6):
        keys = [60 + (k % 3), 60 + ((k + 1) % 3)]
        for key in keys:
            t += 1
            s.submit(t, key, 1000, 300, 40)
        a = s.admit()
        for key in a["build"]:
            rebuilt.append((k, key))
            assert s.build_done(key) == []
        b = s.next_batch()
        assert len(b) == 2
        if k == 3:
            rel = s.batch_failed(b)
            assert sorted(rel) == sorted(keys)     # both parts it read are dropped
            assert not any(s.has_part(x) for x in keys)
        else:
            assert s.batch_done(b) == []
        assert s.used() == s.resident()
    # batch 3 read parts 60 and 61: batch 4 (61, 62) rebuilds 61 and batch 5
    # (62, 60) rebuilds 60; nothing else was built after the first round
    assert [(k, key) for k, key in rebuilt if k >= 1] == [(1, 62), (4, 61), (5, 60)]
    assert s.idle() and s.resident() == 3 * 1000
    s.close()


def test_random_run_with_faults_keeps_invariants(shim):
    """A seeded run with cancellations, failed builds and failed batches:
    bytes in use never exceed the budget, equal the resident parts plus the
    admitted working sets, and return to the resident parts at the end."""
    rng = random.Random(11)
    budget = 5000
    s = Sched(shim, budget, max_batch=4, max_inflight=2)
    parts = {k: rng.randint(200, 1500) for k in range(70, 82)}
    stage = {}
    building = set()
    inflight = []
    t = 0
    for step in range(600):
        r = rng.random()
        if r < 0.35:
            t += 1
            k = rng.choice(list(parts))
            st = rng.randint(10, 200)
            stage[t] = st
            s.submit(t, k, parts[k], rng.randint(0, 300), st)
        elif r < 0.45 and stage:
            s.cancel(rng.choice(list(stage)))
        a = s.admit()
        building.update(a["build"])
        if building and rng.random() < 0.5:
            k = rng.choice(sorted(building))
            building.discard(k)
            s.build_done(k, rng.random() > 0.1)
        b = s.next_batch()
        if b:
            inflight.append(b)
        if inflight and rng.random() < 0.5:
            b = inflight.pop(0)
            (s.batch_failed if rng.random() < 0.1 else s.batch_done)(b)
        assert 0 <= s.used() <= budget
        assert s.used() >= s.resident()
    for k in sorted(building):
        s.build_done(k)
    while True:
        while inflight:
            s.batch_done(inflight.pop(0))
        s.admit()
        b = s.next_batch()
        if not b:
            break
        inflight.append(b)
    assert s.used() == s.resident() and s.inflight() == 0
    s.close()
