"""Served form of the assembly: resident meshes, memory-budget admission and continuous batching.

A Server keeps a set of meshes resident on the device (tile plans, block pattern and coordinates
uploaded once) and accepts assembly requests from any thread: a mesh id, the advection velocity (a
device tensor, or a seed from which the server draws U[-1,1)^3 per node on the device), rho, mu and
dt. One scheduler loop moves each request through

  queued -> admitted -> running -> done            (or rejected / timeout / failed)

  admission   in arrival order, while the bytes a request needs on the device (its block values, its
              RHS and a generated velocity) can be placed in the arena: one device buffer of the
              budget left beside the resident meshes, sub-allocated first-fit, so the loop never
              calls the device allocator and the budget holds by construction. A request larger than
              the whole arena is rejected at once.
  launch      whenever one of the `slots` (a stream with a reusable batch) is free, every admitted
              request not yet running, up to a per-launch cap, goes into one batched
              launch on that stream. Requests that arrive while earlier launches run are admitted as
              memory frees up and go into the next free slot, so launches of different slots overlap
              on the device (the tail of one launch runs beside the head of the next).
  completion  an event recorded after each launch is polled; when it has fired, the launch's
              requests are stamped (latency = arrival to results ready), their budget is returned
              (or kept until release() when the caller keeps the results) and waiters wake.
  timeout     a launch whose event has not fired within its deadline marks its requests timed out
              and reports them; the slot and the memory stay held until the device is done with
              them, since the kernel may still write there.

The device work is that of the batched form: one launch of the library's tiled kernel
over the tiles of every mesh in the launch. The scheduler itself is device-agnostic (an executor
does the launches), so its admission, batching and timeout logic also runs on the CPU.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time

import numpy as np

from . import nsa

QUEUED, ADMITTED, RUNNING, DONE, REJECTED, TIMEOUT, FAILED = (
    "queued", "admitted", "running", "done", "rejected", "timeout", "failed")


ALIGN = 256


def default_tile_blocks(scatter: int, precision: int, mode: str = "batched") -> int | None:
    """Tile size of the resident meshes' plan: None, the library's default plan, for every mode and
    precision (both forms of the run-walking tile kernel hold two 256-thread workgroups per CU, so a
    smaller tile would only leave lanes without runs)."""
    return None


def align(n: int) -> int:
    return (int(n) + ALIGN - 1) // ALIGN * ALIGN


class OffsetArena:
    """First-fit sub-allocator of [0, size) in ALIGN-byte units; freed ranges coalesce. Sizes are
    rounded up to ALIGN."""

    def __init__(self, size: int):
        self.size = int(size) // ALIGN * ALIGN
        self._free = [(0, self.size)] if self.size > 0 else []  # sorted (offset, length)
        self.used = 0

    def alloc(self, n: int) -> int | None:
        n = align(n)
        for k, (off, ln) in enumerate(self._free):
            if ln >= n:
                if ln == n:
                    del self._free[k]
                else:
                    self._free[k] = (off + n, ln - n)
                self.used += n
                return off
        return None

    def free(self, off: int, n: int):
        n = align(n)
        lo, hi = 0, len(self._free)
        while lo < hi:
            mid = (lo + hi) // 2
            if self._free[mid][0] < off:
                lo = mid + 1
            else:
                hi = mid
        k = lo
        if k > 0:
            p_off, p_ln = self._free[k - 1]
            assert p_off + p_ln <= off, "double free"
        if k < len(self._free):
            assert off + n <= self._free[k][0], "double free"
        self._free.insert(k, (off, n))
        self.used -= n
        # coalesce with the neighbours
        if k + 1 < len(self._free) and off + n == self._free[k + 1][0]:
            self._free[k] = (off, n + self._free[k + 1][1])
            del self._free[k + 1]
        if k > 0 and self._free[k - 1][0] + self._free[k - 1][1] == off:
            self._free[k - 1] = (self._free[k - 1][0], self._free[k - 1][1] + self._free[k][1])
            del self._free[k]

    def largest_free(self) -> int:
        return max((ln for _, ln in self._free), default=0)


@dataclasses.dataclass(eq=False)
class Request:
    """One assembly request and its life-cycle stamps (seconds on the server's clock)."""
    id: int
    mesh_id: int
    rho: float
    mu: float
    dt: float
    vel: object = None            # device tensor [npoin][3] float64, or None to draw from vel_seed
    vel_ready: object = None      # event recorded on the submitting thread's stream after vel was written
    vel_seed: int | None = None
    keep: bool = False            # keep the outputs (and their budget) until release()
    timeout: float | None = None  # seconds from launch to completion before it is reported
    nelem: int = 0
    nbytes: int = 0
    ntiles: int = 0
    offset: int | None = None     # of its memory in the server's arena, while admitted
    t_arrival: float = 0.0
    t_admit: float | None = None
    t_launch: float | None = None
    t_done: float | None = None
    status: str = QUEUED
    error: str | None = None
    launch_id: int | None = None
    values: object = None
    rhs: object = None
    velocity: object = None       # the velocity the assembly used (kept with the outputs)
    _server: object = dataclasses.field(default=None, repr=False)
    _event: threading.Event = dataclasses.field(default_factory=threading.Event, repr=False)
    _held: bool = False           # budget still reserved for this request

    @property
    def latency(self) -> float | None:
        return None if self.t_done is None else self.t_done - self.t_arrival

    @property
    def finished(self) -> bool:
        return self._event.is_set()

    def wait(self, timeout: float | None = None) -> bool:
        """Block until the request has an outcome (done, rejected, timeout or failed)."""
        return self._event.wait(timeout)

    def release(self):
        """Give the kept outputs (and their budget) back to the server."""
        if self._server is not None:
            self._server._release(self)


@dataclasses.dataclass(eq=False)
class _Launch:
    id: int
    slot: int
    reqs: list
    handle: object
    t_launch: float
    deadline: float | None
    timed_out: bool = False


class ServerError(RuntimeError):
    pass


class Server:
    """Scheduler over an executor (see GpuExecutor for the device one).

    budget_bytes      device bytes for resident meshes plus every admitted request
    max_launch_elems  cap on the elements of one launch (the first request always goes)
    timeout           default seconds from launch to completion before a request is reported
    poll              seconds the loop sleeps when nothing changed while launches are in flight
    """

    def __init__(self, executor, budget_bytes: int = 64 << 30, max_launch_elems: int = 4_000_000,
                 timeout: float | None = 30.0, poll: float = 20e-6, clock=time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.resident = int(executor.resident_bytes)
        if self.resident > self.budget:
            raise ServerError(f"resident meshes need {self.resident} bytes, budget is {self.budget}")
        self.arena = OffsetArena(self.budget - self.resident)
        executor.attach_arena(self.arena.size)
        self.max_launch_elems = int(max_launch_elems)
        self.timeout = timeout
        self.poll = poll
        self.clock = clock
        self._lock = threading.Lock()
        self._cv = threading.Condition(self._lock)
        self._queue: collections.deque[Request] = collections.deque()
        self._admitted: collections.deque[Request] = collections.deque()
        self._free_slots = list(range(executor.slots))[::-1]
        self._inflight: list[_Launch] = []
        self._reserved = 0
        self._next_id = 0
        self._next_launch = 0
        self._thread = None
        self._stop = False
        self.reset_stats()

    # ---- client side ---------------------------------------------------------------------------

    def submit(self, mesh_id: int, rho: float, mu: float, dt: float, *, vel=None, vel_seed: int | None = None,
               keep: bool = False, timeout: float | None = None, arrival: float | None = None) -> Request:
        """Queue a request; returns at once. `arrival` overrides the arrival stamp (an open-loop
        load generator passes the scheduled time). A caller-owned `vel` may still be in the making
        on the calling thread's current stream: the launch that reads it waits for everything that
        stream had queued at this call."""
        if not 0 <= mesh_id < self.ex.nmesh:
            raise ValueError(f"mesh id {mesh_id} out of range [0, {self.ex.nmesh})")
        if not (rho > 0 and mu >= 0 and dt > 0 and np.isfinite([rho, mu, dt]).all()):
            raise ValueError("need rho > 0, mu >= 0, dt > 0 (finite)")
        if (vel is None) == (vel_seed is None):
            raise ValueError("give exactly one of vel and vel_seed")
        if vel is not None:
            self.ex.check_velocity(mesh_id, vel)
        r = Request(0, int(mesh_id), float(rho), float(mu), float(dt), vel=vel, vel_seed=vel_seed, keep=keep,
                    timeout=self.timeout if timeout is None else timeout)
        if vel is not None:
            # the caller may still be writing vel on its own stream: the launch waits for this point
            r.vel_ready = self.ex.mark_ready(vel)
        r.nelem = self.ex.mesh_elems(mesh_id)
        r.ntiles = self.ex.mesh_tiles(mesh_id)
        r.nbytes = self.ex.request_bytes(mesh_id, vel is None)
        r._server = self
        with self._cv:
            r.id = self._next_id
            self._next_id += 1
            r.t_arrival = self.clock() if arrival is None else arrival
            self._queue.append(r)
            self._cv.notify()
        return r

    def start(self):
        """Run the scheduler loop in a background thread."""
        if self._thread is not None:
            return self
        self._stop = False
        self._thread = threading.Thread(target=self._loop, name="nsa-serve", daemon=True)
        self._thread.start()
        return self

    def stop(self, drain: bool = True, timeout: float | None = None):
        """Stop the loop; with drain, first let every queued and running request finish."""
        if drain:
            t0 = time.monotonic()
            while not self.idle():
                if self._thread is None:
                    self.step()
                else:
                    time.sleep(1e-3)
                if timeout is not None and time.monotonic() - t0 > timeout:
                    break
        if self._thread is not None:
            with self._cv:
                self._stop = True
                self._cv.notify()
            self._thread.join()
            self._thread = None

    def __enter__(self):
        return self.start()

    def __exit__(self, *exc):
        self.stop(drain=exc[0] is None)

    def idle(self) -> bool:
        with self._lock:
            return not self._queue and not self._admitted and not self._inflight

    @property
    def reserved_bytes(self) -> int:
        return self._reserved

    # ---- scheduler -----------------------------------------------------------------------------

    def _loop(self):
        while True:
            with self._cv:
                if self._stop:
                    return
                if not self._queue and not self._admitted and not self._inflight:
                    self._cv.wait(0.05)
                    continue
            if not self.step():
                time.sleep(self.poll)

    def step(self) -> bool:
        """One pass of the scheduler: completions, timeouts, admission, launches. Returns whether
        anything changed."""
        changed = self._complete()
        changed |= self._admit()
        changed |= self._launch()
        return changed

    def _complete(self) -> bool:
        changed = False
        for L in list(self._inflight):
            if self.ex.done(L.handle):
                now = self.clock()
                with self._lock:
                    self._inflight.remove(L)
                    self._free_slots.append(L.slot)
                for r in L.reqs:
                    if r.status == RUNNING:
                        r.status = DONE
                        r.t_done = now
                        self._stats["done"] += 1
                        self._latencies.append(now - r.t_arrival)
                        self._done_elems += r.nelem
                        self._t_last_done = now
                        if self._t_first_arrival is None or r.t_arrival < self._t_first_arrival:
                            self._t_first_arrival = r.t_arrival
                    else:
                        r.values = r.rhs = r.velocity = None  # timed out: results are not handed over
                    if not (r.keep and r.status == DONE):
                        r.values = r.rhs = r.velocity = None
                        self._release(r)
                    r._event.set()
                self.ex.retire(L.handle)
                changed = True
            elif L.deadline is not None and not L.timed_out and self.clock() > L.deadline:
                L.timed_out = True
                for r in L.reqs:
                    if r.status == RUNNING:
                        r.status = TIMEOUT
                        r.error = (f"launch {L.id} (slot {L.slot}) not complete {self.clock() - L.t_launch:.3f} s "
                                   f"after it started")
                        self._stats["timeout"] += 1
                        self.timeouts.append(r)
                        r._event.set()
                changed = True
        return changed

    def _admit(self) -> bool:
        changed = False
        room = self.arena.size
        with self._lock:
            while self._queue:
                r = self._queue[0]
                if r.nbytes > room:
                    self._queue.popleft()
                    r.status = REJECTED
                    r.error = (f"request needs {r.nbytes} bytes; the budget leaves {room} beside the resident "
                               f"meshes")
                    self._stats["rejected"] += 1
                    r._event.set()
                    changed = True
                    continue
                off = self.arena.alloc(r.nbytes)
                if off is None:
                    break  # arrival order: later requests wait behind this one
                self._queue.popleft()
                r.offset = off
                self._reserved += r.nbytes
                r._held = True
                self._peak_reserved = max(self._peak_reserved, self._reserved)
                r.status = ADMITTED
                r.t_admit = self.clock()
                self._admitted.append(r)
                changed = True
        return changed

    def _launch(self) -> bool:
        changed = False
        max_meshes, max_tiles = self.ex.launch_capacity
        while True:
            with self._lock:
                if not self._free_slots or not self._admitted:
                    return changed
                slot = self._free_slots.pop()
                group, elems, tiles = [], 0, 0
                while self._admitted and len(group) < max_meshes:
                    r = self._admitted[0]
                    if group and (elems + r.nelem > self.max_launch_elems or tiles + r.ntiles > max_tiles):
                        break
                    group.append(self._admitted.popleft())
                    elems += r.nelem
                    tiles += r.ntiles
                overlapped = bool(self._inflight)
            lid = self._next_launch
            self._next_launch += 1
            now = self.clock()
            for r in group:
                r.status = RUNNING
                r.t_launch = now
                r.launch_id = lid
            try:
                handle = self.ex.launch(slot, group)
            except Exception as e:  # the launch never reached the device: fail its requests
                with self._lock:
                    self._free_slots.append(slot)
                for r in group:
                    r.status = FAILED
                    r.error = f"launch failed: {e}"
                    r.values = r.rhs = r.velocity = None
                    self._stats["failed"] += 1
                    self._release(r)
                    r._event.set()
                changed = True
                continue
            deadline = None
            tmo = [r.timeout for r in group if r.timeout is not None]
            if tmo:
                deadline = now + min(tmo)
            with self._lock:
                self._inflight.append(_Launch(lid, slot, group, handle, now, deadline))
                self._max_inflight = max(self._max_inflight, len(self._inflight))
            self._stats["launches"] += 1
            self._stats["overlapped_launches"] += overlapped
            self._launch_sizes.append(len(group))
            changed = True

    def _release(self, r: Request):
        if r.status in (QUEUED, ADMITTED, RUNNING):
            raise ValueError(f"request {r.id} is {r.status}: only a finished request can be released")
        with self._lock:
            if r._held:
                r._held = False
                self._reserved -= r.nbytes
                self.arena.free(r.offset, r.nbytes)
                r.offset = None
            r.values = r.rhs = r.velocity = None

    # ---- statistics ----------------------------------------------------------------------------

    def reset_stats(self):
        self._stats = collections.Counter(done=0, rejected=0, timeout=0, failed=0, launches=0,
                                          overlapped_launches=0)
        self._latencies = []
        self._launch_sizes = []
        self._done_elems = 0
        self._t_last_done = None
        self._t_first_arrival = None
        self._peak_reserved = self._reserved
        self._max_inflight = len(self._inflight)
        self.timeouts = []

    def stats(self, t_start: float | None = None) -> dict:
        """Counts, latency percentiles (seconds) of completed requests, elements/s from t_start
        (default: the first completed request's arrival) to the last completion, peak reserved
        bytes, and how often a launch started while another was still running."""
        lat = np.asarray(self._latencies, dtype=np.float64)
        out = dict(self._stats)
        out.update(peak_reserved_bytes=int(self._peak_reserved), budget_bytes=self.budget,
                   resident_bytes=self.resident, max_inflight=int(self._max_inflight),
                   mean_launch_requests=float(np.mean(self._launch_sizes)) if self._launch_sizes else 0.0,
                   max_launch_requests=int(max(self._launch_sizes)) if self._launch_sizes else 0,
                   elements=int(self._done_elems))
        if lat.size:
            out.update(p50=float(np.percentile(lat, 50)), p99=float(np.percentile(lat, 99)),
                       mean=float(lat.mean()), max=float(lat.max()))
            t0 = self._t_first_arrival if t_start is None else t_start
            if self._t_last_done is not None and self._t_last_done > t0:
                out["elements_per_s"] = self._done_elems / (self._t_last_done - t0)
        return out


class GpuExecutor:
    """Device side of a Server: resident meshes, one stream and one reusable batch per slot.

    meshes      sequence of (lnods [nelem][4] int32, coord [npoin][3] float64) pairs or objects with
                .lnods and .coord
    mode        "batched": every launch is one nsa_assemble_batched over its requests;
                "plain": one request per launch through nsa_assemble (the unbatched comparison)
    resident    instead of meshes: nsa.Mesh objects already uploaded with a tile plan for `scatter`
                (shared with another executor)
    trace       record each launch's device interval (device_overlap())
    """

    def __init__(self, meshes, scatter: int = nsa.ATOMIC, precision: int = nsa.MIXED, slots: int = 3,
                 mode: str = "batched", device="cuda", tile_blocks: int | None = None, block_threads: int = 0,
                 grid_wgs: int = 0, max_launch_meshes: int = 256, max_launch_tiles: int = 1 << 20, trace: bool = False,
                 resident=None, log=None):
        import torch
        if mode not in ("batched", "plain"):
            raise ValueError("mode must be 'batched' or 'plain'")
        if mode == "plain":
            slots, max_launch_meshes = 1, 1
        self.mode = mode
        self.scatter, self.precision = int(scatter), int(precision)
        self.block_threads, self.grid_wgs = int(block_threads), int(grid_wgs)
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        self.slots = int(slots)
        # the plan size for this mode and precision unless given (None leaves it to the library)
        tb = tile_blocks if tile_blocks is not None else default_tile_blocks(self.scatter, self.precision, mode)
        self.meshes = list(resident) if resident is not None else []
        self.shared = resident is not None
        t0 = time.perf_counter()
        for i, m in enumerate(meshes if resident is None else []):
            lnods, coord = (m.lnods, m.coord) if hasattr(m, "lnods") else m
            kw = dict(tile_blocks=tb, tile_blocks_colour=0) if self.scatter == nsa.ATOMIC else \
                dict(tile_blocks=0, tile_blocks_colour=tb)
            h = nsa.Mesh(lnods, coord, keep_direct=False, **kw)
            if not h.info.ntiles[self.scatter] and h.nelem:
                raise ServerError(f"mesh {i} has no tile plan for scatter mode {self.scatter}")
            h.upload(self.device)
            h.release_host()
            self.meshes.append(h)
            if log and (i + 1) % 50 == 0:
                log(f"resident meshes: {i + 1} ({time.perf_counter() - t0:.1f} s)")
        self.nmesh = len(self.meshes)
        max_tiles = max([int(h.info.ntiles[self.scatter]) for h in self.meshes] + [1])
        self.launch_capacity = (int(max_launch_meshes), max(int(max_launch_tiles), max_tiles))
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(self.slots)]
        self.batches = []
        if mode == "batched":
            for s in self.streams:
                self.batches.append(nsa.Batch.reserve(*self.launch_capacity, scatter=self.scatter,
                                                      device=self.device, stream=s))
            for s in self.streams:
                s.synchronize()
        for i, h in enumerate(self.meshes):
            if h.ws is None or (h.nelem and not h.info.ntiles[self.scatter]):
                raise ServerError(f"mesh {i} is not uploaded with a tile plan for scatter mode {self.scatter}")
        self.resident_bytes = sum(int(h.ws.numel()) for h in self.meshes) + \
            sum(int(b.ws.numel()) for b in self.batches)
        self._arena = None
        # trace: device-clock interval of every launch's kernel, in ms from a reference event
        self.trace = trace
        self.intervals = []
        self._ref = None
        if trace:
            self._ref = torch.cuda.Event(enable_timing=True)
            self._ref.record(self.streams[0])

    # sizes
    def mesh_elems(self, i):
        return int(self.meshes[i].nelem)

    def mesh_tiles(self, i):
        return int(self.meshes[i].info.ntiles[self.scatter])

    def request_bytes(self, i, with_velocity: bool) -> int:
        """Arena bytes of one request: values [nnzb][4][4], rhs [npoin][4] and, when the server
        draws it, the velocity [npoin][3] (FP64, each ALIGN-aligned)."""
        m = self.meshes[i]
        return align(128 * int(m.nnzb)) + align(32 * int(m.npoin)) + (align(24 * int(m.npoin)) if with_velocity else 0)

    def attach_arena(self, nbytes: int):
        """The device buffer requests are placed in (kept across servers if large enough)."""
        import torch
        if self._arena is None or self._arena.numel() < nbytes:
            self._arena = None
            self._arena = torch.empty(max(int(nbytes), ALIGN), dtype=torch.uint8, device=self.device)

    def _view(self, off, count, shape):
        import torch
        return self._arena[off:off + 8 * count].view(torch.float64).view(shape)

    def check_velocity(self, i, vel):
        import torch
        m = self.meshes[i]
        if not (isinstance(vel, torch.Tensor) and vel.dtype == torch.float64 and vel.device == self.device
                and tuple(vel.shape) == (m.npoin, 3) and vel.is_contiguous()):
            raise ValueError(f"velocity of mesh {i} must be a contiguous float64 [{m.npoin}][3] tensor on "
                             f"{self.device}")

    def mark_ready(self, vel):
        """An event on the calling thread's current stream of vel's device, after whatever it has
        queued so far (the writes of vel among them)."""
        import torch
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(vel.device))
        return ev

    def velocity(self, i, seed, out=None):
        """The velocity a request with this seed uses: U[-1,1)^3 per node, drawn on the device by the
        library's seeded generator (nsa_fill_uniform) on the current stream."""
        import torch
        m = self.meshes[i]
        if out is None:
            out = torch.empty((m.npoin, 3), dtype=torch.float64, device=self.device)
        return nsa.fill_uniform(out, seed, -1.0, 1.0, torch.cuda.current_stream(self.device))

    # launches
    def launch(self, slot, reqs):
        import torch
        s = self.streams[slot]
        with torch.cuda.stream(s):
            vels, outs = [], []
            for r in reqs:
                m = self.meshes[r.mesh_id]
                nnzb, npoin = int(m.nnzb), int(m.npoin)
                o_rhs = r.offset + align(128 * nnzb)
                o_vel = o_rhs + align(32 * npoin)
                if o_vel + (align(24 * npoin) if r.vel is None else 0) > r.offset + r.nbytes:
                    raise ServerError("request placement does not match its size")
                vals = self._view(r.offset, 16 * nnzb, (nnzb, 4, 4))
                rhs = self._view(o_rhs, 4 * npoin, (npoin, 4))
                if r.vel is not None:
                    # order the read of the caller's velocity after the work that produced it, and keep
                    # its memory from being reused before this stream is done with it
                    s.wait_event(r.vel_ready)
                    r.vel.record_stream(s)
                    v = r.vel
                else:
                    v = self.velocity(r.mesh_id, r.vel_seed, self._view(o_vel, 3 * npoin, (npoin, 3)))
                vels.append(v)
                outs.append((vals, rhs))
                r.values, r.rhs, r.velocity = vals, rhs, v
            t_start = None
            if self.mode == "batched":
                b = self.batches[slot]
                b.reset([self.meshes[r.mesh_id] for r in reqs])
                b.set_inputs(vels, [r.rho for r in reqs], [r.mu for r in reqs], [r.dt for r in reqs], outs,
                             stream=s)
                if self.trace:
                    t_start = torch.cuda.Event(enable_timing=True)
                    t_start.record(s)
                b.assemble(self.precision, grid_wgs=self.grid_wgs, block_threads=self.block_threads, stream=s)
            else:
                r = reqs[0]
                if self.trace:
                    t_start = torch.cuda.Event(enable_timing=True)
                    t_start.record(s)
                nsa.assemble(self.meshes[r.mesh_id], vels[0], r.rho, r.mu, r.dt, precision=self.precision,
                             scatter=self.scatter, values=outs[0][0], rhs=outs[0][1], stream=s)
            ev = torch.cuda.Event(enable_timing=self.trace)
            ev.record(s)
        return (ev, vels, outs, t_start, slot, sum(r.nelem for r in reqs))

    def done(self, handle) -> bool:
        return handle[0].query()

    def retire(self, handle):
        if self.trace and handle[3] is not None:
            self.intervals.append((self._ref.elapsed_time(handle[3]), self._ref.elapsed_time(handle[0]),
                                   handle[4], handle[5]))

    def device_overlap(self) -> dict:
        """From the traced launches: how many ran on the device while a launch of another slot was
        running, the busy time (union of intervals) and the summed launch durations, in ms."""
        iv = sorted(self.intervals)
        if not iv:
            return dict(launches=0)
        overlapping = 0
        for k, (a, b, slot, _) in enumerate(iv):
            if any(x < b and a < y and sl != slot for j, (x, y, sl, _) in enumerate(iv) if j != k
                   and x < b + 1e3):
                overlapping += 1
        busy, cur_a, cur_b = 0.0, iv[0][0], iv[0][1]
        for a, b, _, _ in iv[1:]:
            if a > cur_b:
                busy += cur_b - cur_a
                cur_a, cur_b = a, b
            else:
                cur_b = max(cur_b, b)
        busy += cur_b - cur_a
        return dict(launches=len(iv), overlapping=overlapping, busy_ms=busy,
                    sum_ms=float(sum(b - a for a, b, _, _ in iv)), span_ms=iv[-1][1] - iv[0][0])

    def synchronize(self):
        for s in self.streams:
            s.synchronize()
