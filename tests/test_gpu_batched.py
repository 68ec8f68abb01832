"""GPU tests of the batched form: each mesh's result in the batch equals its solo result
(bitwise in the colour mode), matches the oracle, and a captured HIP graph replays correctly with
new inputs installed between replays."""
import sys

import numpy as np
import pytest

import oracle
from paper_2111_05651_amd import inputs, nsa
from tests.parity import TOL_FP64, TOL_MIXED, assert_parity

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def small_batch(nmesh=9, seed=41):
    ps = inputs.batch_params(nmesh, seed=seed, nmin=1, nmax=9)
    return [inputs.make_mesh(p["n"], jitter=True, permute=True, velocity="vortex", seed=p["seed"], rho=p["rho"],
                             mu=p["mu"], dt=p["dt"]) for p in ps]


@pytest.mark.parametrize("scatter", [nsa.ATOMIC, nsa.COLOUR])
@pytest.mark.parametrize("precision", [nsa.FP64, nsa.MIXED])
def test_batch_equals_solo_and_oracle(scatter, precision):
    ms = small_batch()
    say(f"[batched] sizes {[m.nelem for m in ms]} scatter={scatter} precision={precision}")
    meshes = [nsa.Mesh.from_inputs(m, tile_blocks=128, tile_blocks_colour=96).upload() for m in ms]
    b = nsa.Batch(meshes, scatter)
    vels = [torch.from_numpy(m.velocity).cuda() for m in ms]
    outs = b.alloc_outputs()
    b.set_inputs(vels, [m.rho for m in ms], [m.mu for m in ms], [m.dt for m in ms], outs)
    with pytest.raises(nsa.NsaError):
        b.assemble(precision, grid_wgs=-8)
    # one workgroup per tile, and persistent grids smaller than the tile count
    for grid in (0, 8, 24):
        b.assemble(precision, grid_wgs=grid)
        torch.cuda.synchronize()
        for m, mesh, vel, (v, r) in zip(ms, meshes, vels, outs):
            sv, sr = nsa.assemble(mesh, vel, m.rho, m.mu, m.dt, precision=precision, scatter=scatter,
                                  kernel=nsa.KERNEL_TILED)
            torch.cuda.synchronize()
            if scatter == nsa.COLOUR:
                assert torch.equal(v, sv) and torch.equal(r, sr), "colour mode: batched == solo, bitwise"
            ref_v, ref_r = oracle.assemble(m)
            assert_parity(v.cpu().numpy(), ref_v, r.cpu().numpy(), ref_r,
                          TOL_FP64 if precision == nsa.FP64 else TOL_MIXED, f"batched n={m.n}")


def test_batch_graph_replay():
    """Capture one batched launch; replay it three times with different velocities installed in
    between (eager work and synchronisation between replays), each replay checked against an eager
    launch."""
    ms = small_batch(6, seed=43)
    meshes = [nsa.Mesh.from_inputs(m, tile_blocks=128).upload() for m in ms]
    b = nsa.Batch(meshes, nsa.ATOMIC)
    rng = np.random.default_rng(7)
    vels = [torch.zeros((m.npoin, 3), dtype=torch.float64, device="cuda") for m in ms]
    outs = b.alloc_outputs()
    args = ([m.rho for m in ms], [m.mu for m in ms], [m.dt for m in ms])
    b.set_inputs(vels, *args, outs)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.assemble(nsa.FP64)          # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        b.assemble(nsa.FP64)
    torch.cuda.synchronize()
    for rep in range(3):
        for v, m in zip(vels, ms):
            v.copy_(torch.from_numpy(rng.uniform(-1, 1, size=(m.npoin, 3))))
        eager = [(torch.empty_like(o[0]), torch.empty_like(o[1])) for o in outs]
        b.set_inputs(vels, *args, eager)
        b.assemble(nsa.FP64)
        torch.cuda.synchronize()
        b.set_inputs(vels, *args, outs)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (v, r), (ev, er) in zip(outs, eager):
            assert torch.allclose(v, ev, rtol=0, atol=1e-12 * float(ev.abs().max())), f"replay {rep}"
            assert torch.allclose(r, er, rtol=0, atol=1e-12 * float(er.abs().max() + 1e-300)), f"replay {rep}"
