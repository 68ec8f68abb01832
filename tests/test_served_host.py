"""Scheduler of the served form on the CPU: admission by memory budget, continuous batching over
slots, time-outs, rejections and failed launches, with a fake executor on a fake clock (no device)."""
import math
import threading
import time

import numpy as np
import pytest

from paper_2111_05651_amd import inputs
from paper_2111_05651_amd.serve import (ADMITTED, DONE, FAILED, QUEUED, REJECTED, RUNNING, TIMEOUT, OffsetArena,
                                        Server, ServerError, align)


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Launches take sum(nelem) / rate seconds of the clock; launches that touch a mesh in `stuck`
    never finish until it is removed from the set; meshes in `broken` make launch() raise."""

    def __init__(self, sizes, clock, rate=1e8, slots=2, resident=4096, capacity=(256, 1 << 20)):
        self.sizes = list(sizes)
        self.nmesh = len(self.sizes)
        self.clock = clock
        self.rate = rate
        self.slots = slots
        self.resident_bytes = resident
        self.launch_capacity = capacity
        self.stuck, self.broken = set(), set()
        self.busy = set()
        self.launches = []

    def mesh_elems(self, i):
        return self.sizes[i]

    def mesh_tiles(self, i):
        return max(1, math.ceil(self.sizes[i] / 100))

    def request_bytes(self, i, with_velocity):
        return align(100 * self.sizes[i]) + (align(10 * self.sizes[i]) if with_velocity else 0)

    def attach_arena(self, nbytes):
        self.arena_bytes = nbytes

    def check_velocity(self, i, vel):
        if len(vel) != self.sizes[i]:
            raise ValueError("wrong velocity length")

    def mark_ready(self, vel):
        return None

    def launch(self, slot, reqs):
        assert slot not in self.busy, "slot reused while busy"
        meshes = [r.mesh_id for r in reqs]
        if self.broken & set(meshes):
            raise RuntimeError("injected launch failure")
        self.busy.add(slot)
        h = dict(slot=slot, t=self.clock(), dur=sum(r.nelem for r in reqs) / self.rate, meshes=meshes,
                 ids=[r.id for r in reqs])
        for r in reqs:
            r.values, r.rhs = ("values", r.id), ("rhs", r.id)
        self.launches.append(h)
        return h

    def done(self, h):
        return not (self.stuck & set(h["meshes"])) and self.clock() >= h["t"] + h["dur"]

    def retire(self, h):
        self.busy.discard(h["slot"])


def run_open_loop(srv, ex, clock, stream, dt=1e-5, horizon=60.0, check=None, keep=False):
    """Submit `stream` (served_requests dicts) at their arrival times on the fake clock and step the
    scheduler until everything has an outcome."""
    reqs, k = [], 0
    while clock.t < horizon:
        while k < len(stream) and stream[k]["t"] <= clock.t:
            s = stream[k]
            reqs.append(srv.submit(s["mesh"], s["rho"], s["mu"], s["dt"], vel_seed=s["vel_seed"], keep=keep,
                                   arrival=s["t"]))
            k += 1
        srv.step()
        if check:
            check()
        if k == len(stream) and srv.idle():
            break
        clock.t += dt
    return reqs


def test_admission_never_exceeds_budget():
    clock = Clock()
    sizes = [int(x) for x in np.random.default_rng(0).integers(1_000, 50_000, size=30)]
    ex = FakeExecutor(sizes, clock, rate=2e8, slots=3)
    room = 3 * max(ex.request_bytes(i, True) for i in range(ex.nmesh))
    srv = Server(ex, budget_bytes=ex.resident_bytes + room, clock=clock, timeout=None)
    stream = inputs.served_requests(300, ex.nmesh, rate=20_000, seed=1)

    def check():
        assert 0 <= srv.reserved_bytes <= room
        assert len(ex.busy) <= ex.slots

    reqs = run_open_loop(srv, ex, clock, stream, check=check)
    assert all(r.status == DONE for r in reqs)
    st = srv.stats()
    assert st["done"] == 300 and st["peak_reserved_bytes"] <= room
    assert srv.reserved_bytes == 0
    # the budget made requests wait for memory
    assert any(r.t_admit > r.t_arrival for r in reqs)
    # arrival order of admission
    admits = [r.t_admit for r in sorted(reqs, key=lambda r: r.id)]
    assert all(a <= b for a, b in zip(admits, admits[1:]))
    # every request's outputs were handed over and then dropped (keep=False)
    assert all(r.values is None for r in reqs)


def test_continuous_batching_overlaps_and_groups():
    clock = Clock()
    ex = FakeExecutor([1_000_000, 2_000, 2_000, 2_000, 2_000, 2_000], clock, rate=1e8, slots=2)
    srv = Server(ex, budget_bytes=1 << 40, clock=clock, timeout=None)
    big = srv.submit(0, 1.0, 1e-3, 1e-2, vel_seed=1)
    srv.step()                       # the big request runs on the first slot (10 ms)
    assert big.status == RUNNING
    clock.t = 1e-3
    a = srv.submit(1, 1.0, 1e-3, 1e-2, vel_seed=2)
    srv.step()                       # arrives while it runs: goes to the second slot at once
    assert a.status == RUNNING and a.launch_id != big.launch_id
    clock.t = 1.01e-3                # both slots busy: the next arrivals wait, then go together
    more = [srv.submit(i, 1.0, 1e-3, 1e-2, vel_seed=10 + i) for i in (2, 3, 4, 5)]
    srv.step()
    assert all(r.status == ADMITTED for r in more)
    clock.t = 1.02e-3 + 2_000 / 1e8  # the small launch finishes; the four share the freed slot
    srv.step()
    assert all(r.status == RUNNING for r in more)
    assert len({r.launch_id for r in more}) == 1
    assert big.status == RUNNING     # ... while the big one still runs
    clock.t = 0.02
    srv.step()
    assert all(r.status == DONE for r in [big, a] + more)
    st = srv.stats()
    assert st["launches"] == 3 and st["overlapped_launches"] == 2 and st["max_launch_requests"] == 4
    assert st["max_inflight"] == 2
    assert math.isclose(big.latency, 0.02) and math.isclose(a.latency, 0.02e-3 + 2_000 / 1e8)


def test_launch_caps_split_groups():
    clock = Clock()
    ex = FakeExecutor([10_000] * 8, clock, rate=1e8, slots=4, capacity=(3, 1 << 20))
    srv = Server(ex, budget_bytes=1 << 40, clock=clock, timeout=None, max_launch_elems=25_000)
    reqs = [srv.submit(i, 1.0, 1e-3, 1e-2, vel_seed=i) for i in range(8)]
    srv.step()
    # 25k elements per launch: groups of 2 (the mesh cap of 3 is not reached)
    assert [len(h["ids"]) for h in ex.launches] == [2, 2, 2, 2]
    clock.t = 1.0
    srv.step()
    assert all(r.status == DONE for r in reqs)


def test_oversized_request_rejected_others_served():
    clock = Clock()
    ex = FakeExecutor([1_000, 10_000_000, 1_000], clock, slots=1)
    room = 5 * ex.request_bytes(0, True)
    srv = Server(ex, budget_bytes=ex.resident_bytes + room, clock=clock, timeout=None)
    r0 = srv.submit(0, 1.0, 1e-3, 1e-2, vel_seed=1)
    big = srv.submit(1, 1.0, 1e-3, 1e-2, vel_seed=2)
    r2 = srv.submit(2, 1.0, 1e-3, 1e-2, vel_seed=3)
    srv.step()
    assert big.status == REJECTED and big.finished and "bytes" in big.error
    clock.t = 1.0
    srv.step()
    assert r0.status == DONE and r2.status == DONE
    assert srv.stats()["rejected"] == 1 and srv.reserved_bytes == 0


def test_timeout_reported_and_memory_held_until_done():
    clock = Clock()
    ex = FakeExecutor([1_000, 1_000], clock, slots=2)
    srv = Server(ex, budget_bytes=1 << 30, clock=clock, timeout=0.5)
    ex.stuck.add(0)
    stuck = srv.submit(0, 1.0, 1e-3, 1e-2, vel_seed=1)
    srv.step()
    clock.t = 0.1
    other = srv.submit(1, 1.0, 1e-3, 1e-2, vel_seed=2)
    srv.step()
    clock.t = 0.2
    srv.step()
    assert other.status == DONE and stuck.status == RUNNING
    clock.t = 0.6
    srv.step()
    assert stuck.status == TIMEOUT and stuck.finished and "not complete" in stuck.error
    assert srv.timeouts == [stuck] and srv.stats()["timeout"] == 1
    # the device may still write to its outputs: memory and slot stay held
    assert srv.reserved_bytes == stuck.nbytes and ex.busy == {0}
    ex.stuck.clear()
    srv.step()
    assert srv.reserved_bytes == 0 and not ex.busy
    assert stuck.status == TIMEOUT and stuck.values is None and stuck.latency is None
    assert srv.idle()


def test_failed_launch_releases_everything():
    clock = Clock()
    ex = FakeExecutor([1_000, 1_000], clock, slots=1)
    srv = Server(ex, budget_bytes=1 << 30, clock=clock, timeout=None)
    ex.broken.add(0)
    bad = srv.submit(0, 1.0, 1e-3, 1e-2, vel_seed=1)
    srv.step()
    assert bad.status == FAILED and "injected" in bad.error and srv.reserved_bytes == 0
    good = srv.submit(1, 1.0, 1e-3, 1e-2, vel_seed=2)
    srv.step()
    clock.t = 1.0
    srv.step()
    assert good.status == DONE and srv.stats()["failed"] == 1


def test_kept_results_hold_budget_until_release():
    clock = Clock()
    ex = FakeExecutor([1_000, 1_000], clock, slots=1)
    room = ex.request_bytes(0, True)
    srv = Server(ex, budget_bytes=ex.resident_bytes + room, clock=clock, timeout=None)
    a = srv.submit(0, 1.0, 1e-3, 1e-2, vel_seed=1, keep=True)
    with pytest.raises(ValueError):
        a.release()  # still queued
    b = srv.submit(1, 1.0, 1e-3, 1e-2, vel_seed=2)
    srv.step()
    clock.t = 1.0
    srv.step()
    assert a.status == DONE and a.values == ("values", a.id)
    srv.step()
    assert b.status == QUEUED  # a's kept outputs still use the whole room
    a.release()
    assert a.values is None
    srv.step()
    clock.t = 2.0
    srv.step()
    assert b.status == DONE and srv.reserved_bytes == 0


def test_latency_percentiles():
    clock = Clock()
    sizes = [1_000 * (i + 1) for i in range(100)]
    ex = FakeExecutor(sizes, clock, rate=1e6, slots=1)
    srv = Server(ex, budget_bytes=1 << 40, clock=clock, timeout=None)
    lat = []
    for i in range(100):  # one at a time: latency = its own launch duration (to the polling step)
        r = srv.submit(i, 1.0, 1e-3, 1e-2, vel_seed=i)
        srv.step()
        clock.t += sizes[i] / 1e6
        srv.step()
        assert r.status == DONE
        lat.append(r.latency)
        clock.t += 1.0
    st = srv.stats()
    assert np.allclose(lat, np.asarray(sizes) / 1e6)
    assert math.isclose(st["p50"], np.percentile(lat, 50)) and math.isclose(st["p99"], np.percentile(lat, 99))


def test_submit_validation_and_resident_budget():
    clock = Clock()
    ex = FakeExecutor([100], clock)
    with pytest.raises(ServerError):
        Server(ex, budget_bytes=ex.resident_bytes - 1, clock=clock)
    srv = Server(ex, budget_bytes=1 << 20, clock=clock)
    with pytest.raises(ValueError):
        srv.submit(1, 1.0, 1e-3, 1e-2, vel_seed=1)
    with pytest.raises(ValueError):
        srv.submit(0, 0.0, 1e-3, 1e-2, vel_seed=1)
    with pytest.raises(ValueError):
        srv.submit(0, 1.0, 1e-3, 1e-2)
    with pytest.raises(ValueError):
        srv.submit(0, 1.0, 1e-3, 1e-2, vel=[0.0] * 100, vel_seed=1)
    with pytest.raises(ValueError):
        srv.submit(0, 1.0, 1e-3, 1e-2, vel=[0.0] * 99)
    r = srv.submit(0, 1.0, 1e-3, 1e-2, vel=[0.0] * 100)
    assert r.nbytes == align(100 * 100)  # a caller's velocity is not counted


def test_threaded_loop_with_concurrent_clients():
    ex = FakeExecutor([2_000] * 10, time.perf_counter, rate=1e8, slots=2)
    srv = Server(ex, budget_bytes=ex.resident_bytes + 4 * ex.request_bytes(0, True), timeout=5.0)
    got = [[], []]

    def client(k):
        for i in range(50):
            got[k].append(srv.submit((i + k) % 10, 1.0, 1e-3, 1e-2, vel_seed=i))
            time.sleep(1e-4)

    with srv:
        th = [threading.Thread(target=client, args=(k,)) for k in (0, 1)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for r in got[0] + got[1]:
            assert r.wait(10.0)
    assert all(r.status == DONE for r in got[0] + got[1])
    assert srv.stats()["done"] == 100 and srv.reserved_bytes == 0


def test_offset_arena_against_a_bitmap():
    """Random alloc/free against a byte map: no overlap, in bounds, aligned, and everything
    coalesces back into one range."""
    rng = np.random.default_rng(3)
    size = 256 * 4096
    a = OffsetArena(size)
    owner = np.zeros(size // 256, dtype=np.int64)
    live = {}
    for step in range(4000):
        if live and (rng.random() < 0.45 or len(live) > 60):
            k = list(live)[rng.integers(len(live))]
            off, n = live.pop(k)
            assert (owner[off // 256:(off + align(n)) // 256] == k).all()
            owner[off // 256:(off + align(n)) // 256] = 0
            a.free(off, n)
        else:
            n = int(rng.integers(1, 256 * 200))
            off = a.alloc(n)
            free_units = (owner == 0)
            if off is None:
                # first fit failed: no free run of that length exists
                need = align(n) // 256
                run = best = 0
                for f in free_units:
                    run = run + 1 if f else 0
                    best = max(best, run)
                assert best < need
                continue
            assert off % 256 == 0 and off + align(n) <= size
            assert (owner[off // 256:(off + align(n)) // 256] == 0).all()
            owner[off // 256:(off + align(n)) // 256] = step + 1
            live[step + 1] = (off, n)
        assert a.used == int((owner != 0).sum()) * 256
    for k, (off, n) in list(live.items()):
        a.free(off, n)
    assert a.used == 0 and a.largest_free() == size and len(a._free) == 1
    with pytest.raises(AssertionError):
        off = a.alloc(1000)
        a.free(off, 1000)
        a.free(off, 1000)


def test_fragmented_arena_blocks_admission_in_order():
    """A request that fits the free total but no free range waits (arrival order), then goes once
    the ranges coalesce."""
    clock = Clock()
    ex = FakeExecutor([2_560, 2_560, 2_560, 5_120], clock, slots=4)
    unit = ex.request_bytes(0, True)
    srv = Server(ex, budget_bytes=ex.resident_bytes + 3 * unit + 255, clock=clock, timeout=None)
    a, b, c = (srv.submit(i, 1.0, 1e-3, 1e-2, vel_seed=i, keep=True) for i in range(3))
    srv.step()
    clock.t = 1.0
    srv.step()
    a.release()
    c.release()  # free: [a] and [c], two separate ranges of one unit each
    big = srv.submit(3, 1.0, 1e-3, 1e-2, vel_seed=9)
    assert big.nbytes == 2 * unit
    srv.step()
    assert big.status == QUEUED and srv.reserved_bytes == unit
    b.release()  # now all three units coalesce
    srv.step()
    assert big.status == RUNNING
