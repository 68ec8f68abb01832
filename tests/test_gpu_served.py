"""GPU tests of the served form: a stream of requests over resident meshes gives, for every request,
the same result in the mix (continuous batching, several slots, a tight memory budget) as alone
(bitwise in the colour mode, within the FP64 tolerance in the atomic mode), served results match the
oracle, and the budget is never exceeded."""
import queue
import sys
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2111_05651_amd import inputs, nsa
from paper_2111_05651_amd.serve import DONE, GpuExecutor, Server
from tests.parity import TOL_FP64, TOL_MIXED, assert_parity, class_errors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def meshes():
    return inputs.config_served(nmesh=12, seed=51, tmin=1e3, tmax=2e5)


def outputs(r):
    return r.values.cpu().numpy(), r.rhs.cpu().numpy(), r.velocity.cpu().numpy()


@pytest.mark.parametrize("scatter", [nsa.ATOMIC, nsa.COLOUR])
def test_served_mix_equals_alone(meshes, scatter):
    say(f"[served] scatter={scatter} sizes={[m.nelem for m in meshes]}")
    ex = GpuExecutor(meshes, scatter=scatter, precision=nsa.MIXED, slots=3, trace=True)
    largest = max(ex.request_bytes(i, True) for i in range(ex.nmesh))
    srv = Server(ex, budget_bytes=ex.resident_bytes + 4 * largest, timeout=30.0, max_launch_elems=300_000)
    stream = inputs.served_requests(48, ex.nmesh, rate=20_000, seed=52)
    with srv:
        # alone: one request at a time on an idle server
        alone = []
        for s in stream:
            r = srv.submit(s["mesh"], s["rho"], s["mu"], s["dt"], vel_seed=s["vel_seed"], keep=True)
            assert r.wait(30.0) and r.status == DONE, r.error
            alone.append(outputs(r))
            r.release()
        assert srv.stats()["max_launch_requests"] == 1
        srv.reset_stats()
        # the mix: open-loop arrivals (about 2.4 ms for all 48); a consumer copies each result out
        # and releases it (kept results hold their budget until then)
        fed = queue.Queue()
        got = []

        def consumer():
            for _ in stream:
                r = fed.get()
                ok = r.wait(30.0) and r.status == DONE
                got.append((r, outputs(r) if ok else None))
                if ok:
                    r.release()

        th = threading.Thread(target=consumer)
        th.start()
        t0 = time.perf_counter()
        for s in stream:
            while time.perf_counter() - t0 < s["t"]:
                pass
            fed.put(srv.submit(s["mesh"], s["rho"], s["mu"], s["dt"], vel_seed=s["vel_seed"], keep=True))
        th.join(120.0)
        assert len(got) == len(stream)
        st = srv.stats()
        say(f"[served] mix: {st}")
        say(f"[served] device overlap: {ex.device_overlap()}")
        assert st["done"] == len(stream)
        assert st["peak_reserved_bytes"] <= srv.budget - srv.resident
        for k, ((r, res), (av, ar, au)) in enumerate(zip(got, alone)):
            assert res is not None, f"request {k}: {r.status} {r.error}"
            v, rh, u = res
            assert np.array_equal(u, au), "the request's velocity is drawn from its seed"
            if scatter == nsa.COLOUR:
                assert np.array_equal(v, av) and np.array_equal(rh, ar), f"request {k}: mix != alone (bitwise)"
            else:
                err = class_errors(v, av, rh, ar)
                assert max(err.values()) <= TOL_FP64, f"request {k}: mix vs alone {err}"
    assert srv.reserved_bytes == 0


def test_served_results_match_oracle(meshes):
    ex = GpuExecutor(meshes, scatter=nsa.ATOMIC, precision=nsa.MIXED, slots=2)
    srv = Server(ex, budget_bytes=ex.resident_bytes + (1 << 30), timeout=30.0)
    small = sorted(range(ex.nmesh), key=lambda i: meshes[i].nelem)[:4]
    with srv:
        reqs = [srv.submit(i, 1.3, 2e-3, 4e-3, vel_seed=1000 + i, keep=True) for i in small]
        for r in reqs:
            assert r.wait(30.0) and r.status == DONE, r.error
        for i, r in zip(small, reqs):
            v, rh, u = outputs(r)
            ref_v, ref_r = oracle.assemble(meshes[i], rho=1.3, mu=2e-3, dt=4e-3, velocity=u)
            assert_parity(v, ref_v, rh, ref_r, TOL_MIXED, f"served mesh {i}")
            r.release()


def test_plain_fp64_one_at_a_time(meshes):
    """The unbatched comparison path: plain FP64 launches, one request each, one stream."""
    ex = GpuExecutor(meshes[:4], scatter=nsa.ATOMIC, precision=nsa.FP64, mode="plain")
    srv = Server(ex, budget_bytes=ex.resident_bytes + (1 << 30), timeout=30.0)
    with srv:
        reqs = [srv.submit(i, 0.7, 1e-3, 5e-3, vel_seed=7 + i, keep=True) for i in range(4)]
        for r in reqs:
            assert r.wait(30.0) and r.status == DONE, r.error
    st = srv.stats()
    assert st["launches"] == 4 and st["max_launch_requests"] == 1
    for i, r in enumerate(reqs):
        v, rh, u = outputs(r)
        ref_v, ref_r = oracle.assemble(meshes[i], rho=0.7, mu=1e-3, dt=5e-3, velocity=u)
        assert_parity(v, ref_v, rh, ref_r, TOL_FP64, f"plain served mesh {i}")
        r.release()


def test_served_caller_velocity_and_concurrent_clients(meshes):
    """Two client threads submit caller-owned velocities at once; every result equals the plain
    kernel's on the same inputs (colour mode: bitwise)."""
    ex = GpuExecutor(meshes[:6], scatter=nsa.COLOUR, precision=nsa.MIXED, slots=3)
    srv = Server(ex, budget_bytes=ex.resident_bytes + (1 << 30), timeout=30.0)
    rng = np.random.default_rng(53)
    vels = [torch.from_numpy(rng.uniform(-1, 1, size=(m.npoin, 3))).cuda() for m in meshes[:6]]
    got = [[], []]

    def client(k):
        for j in range(12):
            i = (j + 3 * k) % 6
            got[k].append((i, srv.submit(i, 1.0, 1e-3, 1e-2, vel=vels[i], keep=True)))

    with srv:
        th = [threading.Thread(target=client, args=(k,)) for k in (0, 1)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for i, r in got[0] + got[1]:
            assert r.wait(30.0) and r.status == DONE, r.error
    plain = {}
    for i in range(6):
        h = nsa.Mesh.from_inputs(meshes[i], tile_blocks=0).upload()
        plain[i] = nsa.assemble(h, vels[i], 1.0, 1e-3, 1e-2, precision=nsa.MIXED, scatter=nsa.COLOUR,
                                kernel=nsa.KERNEL_TILED)
    torch.cuda.synchronize()
    for i, r in got[0] + got[1]:
        assert torch.equal(r.values, plain[i][0]) and torch.equal(r.rhs, plain[i][1])
        r.release()


def test_served_velocity_written_on_another_stream(meshes):
    """A client writes each velocity on its own stream behind slow work and submits at once, without
    synchronising: the server's launch waits for that stream, so every result equals the plain
    kernel's on the finished velocity (colour mode: bitwise)."""
    ex = GpuExecutor(meshes[:3], scatter=nsa.COLOUR, precision=nsa.MIXED, slots=2)
    srv = Server(ex, budget_bytes=ex.resident_bytes + (1 << 30), timeout=30.0)
    rng = np.random.default_rng(57)
    srcs = [torch.from_numpy(rng.uniform(-1, 1, size=(m.npoin, 3))).cuda() for m in meshes[:3]]
    a = torch.randn(2048, 2048, device="cuda")
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    reqs = []
    with srv:
        for j in range(6):
            i = j % 3
            with torch.cuda.stream(side):
                vel = torch.full_like(srcs[i], float("nan"))
                for _ in range(8):      # slow work ahead of the write on the same stream
                    a = torch.tanh(a @ a) * 0.5
                vel.copy_(srcs[i])
                reqs.append((i, vel, srv.submit(i, 1.0, 1e-3, 1e-2, vel=vel, keep=True)))
        for i, _, r in reqs:
            assert r.wait(30.0) and r.status == DONE, r.error
    torch.cuda.synchronize()
    for i, vel, r in reqs:
        h = nsa.Mesh.from_inputs(meshes[i], tile_blocks=0).upload()
        pv, pr = nsa.assemble(h, srcs[i], 1.0, 1e-3, 1e-2, precision=nsa.MIXED, scatter=nsa.COLOUR,
                              kernel=nsa.KERNEL_TILED)
        torch.cuda.synchronize()
        assert torch.equal(r.values, pv) and torch.equal(r.rhs, pr)
        r.release()


def splitmix_uniform(n, seed, lo, hi):
    """lo + (hi - lo) * u_i, u_i = top 53 bits of splitmix64 at counter seed + (i + 1) * gamma,
    written from the generator's published definition (independent of the library's kernel)."""
    i = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed % (1 << 64)) + i * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return lo + (hi - lo) * u


@pytest.mark.parametrize("n,seed,lo,hi", [(0, 5, 0.0, 1.0), (1, 0, -1.0, 1.0), (777, 2 ** 64 - 1, 0.5, 2.0),
                                          (3 * 274625, 123456789, -1.0, 1.0)])
def test_fill_uniform_matches_definition(n, seed, lo, hi):
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    nsa.fill_uniform(out, seed, lo, hi)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(got, splitmix_uniform(n, seed, lo, hi)), "bitwise equal to the definition"
    if n > 100000:
        assert got.min() >= lo and got.max() < hi and abs(got.mean() - 0.5 * (lo + hi)) < 5e-3
        assert np.unique(got).size == n
