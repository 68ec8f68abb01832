"""GPU test of the allocation-free batched launch (nsa_assemble_batched_static) through the C ABI: its
results equal those of the batched form with a batch handle and workspace (nsa_batch_* +
nsa_assemble_batched) on two calls in a row, the second over fewer and smaller meshes, so that
tables the first call left in the library's fixed device array cannot leak into the second; the
size limits are refused before anything is launched; and no device memory is allocated."""
import sys

import numpy as np
import pytest

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


@pytest.fixture(scope="module", autouse=True)
def static_ready(need_gpu):
    """One call on a tiny mesh first: the entry point's first call on a device takes the address of
    the library's fixed array there, and the runtime maps that array (held until the process ends)
    when it loads the code holding it, so free device memory may move once, on that first call."""
    m = inputs.make_mesh(2, jitter=True, seed=70)
    h = nsa.Mesh.from_inputs(m, tile_blocks=128).upload()
    vel = torch.from_numpy(m.velocity).cuda()
    nsa.assemble_batched_static([h], [vel], [m.rho], [m.mu], [m.dt], [h.alloc_outputs()], precision=nsa.FP64)
    torch.cuda.synchronize()


def meshes_of(nmesh, seed, nmax):
    ps = inputs.batch_params(nmesh, seed=seed, nmin=1, nmax=nmax)
    return [inputs.make_mesh(p["n"], jitter=True, permute=True, velocity="vortex", seed=p["seed"], rho=p["rho"],
                             mu=p["mu"], dt=p["dt"]) for p in ps]


def with_handle(hs, ms, vels, scatter, precision):
    """The existing batched entry point on the same meshes and inputs."""
    b = nsa.Batch(hs, scatter)
    outs = b.alloc_outputs()
    b.set_inputs(vels, [m.rho for m in ms], [m.mu for m in ms], [m.dt for m in ms], outs)
    b.assemble(precision)
    torch.cuda.synchronize()
    return outs


def static_call(hs, ms, vels, scatter, precision, accumulate=False, fill=float("nan")):
    outs = [(torch.full((h.nnzb, 4, 4), fill, dtype=torch.float64, device="cuda"),
             torch.full((h.npoin, 4), fill, dtype=torch.float64, device="cuda")) for h in hs]
    torch.cuda.synchronize()
    before = torch.cuda.memory_stats().get("num_device_alloc", 0)
    free0 = torch.cuda.mem_get_info()[0]
    nsa.assemble_batched_static(hs, vels, [m.rho for m in ms], [m.mu for m in ms], [m.dt for m in ms], outs,
                                precision=precision, scatter=scatter, accumulate=accumulate)
    torch.cuda.synchronize()
    # neither torch's allocator nor the device's free memory moved during the call
    assert torch.cuda.memory_stats().get("num_device_alloc", 0) == before
    assert torch.cuda.mem_get_info()[0] == free0
    return outs


def compare(outs, ref, scatter, precision, what):
    for i, ((v, r), (rv, rr)) in enumerate(zip(outs, ref)):
        if scatter == nsa.COLOUR:
            # the deterministic plan sums in a fixed order: the same launch gives the same bits
            assert torch.equal(v, rv) and torch.equal(r, rr), f"{what} mesh {i}: colour mode bitwise"
        assert_parity(v.cpu().numpy(), rv.cpu().numpy(), r.cpu().numpy(), rr.cpu().numpy(),
                      TOL_FP64 if precision == nsa.FP64 else TOL_MIXED, f"{what} mesh {i}")


@pytest.mark.parametrize("scatter", [nsa.ATOMIC, nsa.COLOUR])
@pytest.mark.parametrize("precision", [nsa.FP64, nsa.MIXED])
def test_static_equals_batched_two_calls(scatter, precision):
    first = meshes_of(11, seed=71, nmax=12)      # two descriptor chunks
    second = meshes_of(3, seed=72, nmax=5)       # fewer, smaller meshes
    for call, ms in (("first", first), ("second", second)):
        say(f"[no-alloc] {call} call: sizes {[m.nelem for m in ms]} scatter={scatter} precision={precision}")
        hs = [nsa.Mesh.from_inputs(m, tile_blocks=128, tile_blocks_colour=96).upload() for m in ms]
        vels = [torch.from_numpy(m.velocity).cuda() for m in ms]
        ref = with_handle(hs, ms, vels, scatter, precision)
        outs = static_call(hs, ms, vels, scatter, precision)
        compare(outs, ref, scatter, precision, f"{call} call")


def test_static_repeats_and_accumulate():
    ms = meshes_of(4, seed=73, nmax=8)
    hs = [nsa.Mesh.from_inputs(m, tile_blocks=128).upload() for m in ms]
    # a mesh twice, with its own inputs each time
    order = [0, 2, 0, 3, 1]
    mo = [ms[i] for i in order]
    ho = [hs[i] for i in order]
    vels = [torch.from_numpy(m.velocity).cuda() * (1.0 + 0.1 * k) for k, m in enumerate(mo)]
    say(f"[no-alloc] repeats: order {order}")
    ref = with_handle(ho, mo, vels, nsa.ATOMIC, nsa.FP64)
    outs = static_call(ho, mo, vels, nsa.ATOMIC, nsa.FP64)
    compare(outs, ref, nsa.ATOMIC, nsa.FP64, "repeats")
    # accumulate onto a prefilled output
    say("[no-alloc] accumulate")
    outs = static_call(ho, mo, vels, nsa.ATOMIC, nsa.FP64, accumulate=True, fill=0.25)
    for i, ((v, r), (rv, rr)) in enumerate(zip(outs, ref)):
        assert_parity(v.cpu().numpy() - 0.25, rv.cpu().numpy(), r.cpu().numpy() - 0.25, rr.cpu().numpy(),
                      TOL_FP64, f"accumulate mesh {i}")


def test_static_limits_refused():
    m = inputs.make_mesh(3, jitter=True, seed=74)
    h = nsa.Mesh.from_inputs(m, tile_blocks=128).upload()
    vel = torch.from_numpy(m.velocity).cuda()
    out = h.alloc_outputs()
    n = 257
    say("[no-alloc] 257 meshes refused")
    with pytest.raises(nsa.NsaError, match="at most 256"):
        nsa.assemble_batched_static([h] * n, [vel] * n, [1.0] * n, [1e-3] * n, [1e-2] * n, [out] * n)
    # more than 2^20 tiles in total: 17 x 128^3-sized tile counts are not needed, a fine tiling does it
    big = inputs.make_mesh(40, jitter=True, seed=75)
    hb = nsa.Mesh.from_inputs(big, tile_blocks=64).upload()
    tiles = hb.info.ntiles[nsa.ATOMIC]
    k = (1 << 20) // tiles + 1
    assert k <= 256, tiles
    vb = torch.from_numpy(big.velocity).cuda()
    ob = hb.alloc_outputs()
    say(f"[no-alloc] {k} x {tiles} tiles refused")
    with pytest.raises(nsa.NsaError, match="tiles, at most"):
        nsa.assemble_batched_static([hb] * k, [vb] * k, [1.0] * k, [1e-3] * k, [1e-2] * k, [ob] * k)
    # the fixed array still serves a good call afterwards
    ref = with_handle([h], [m], [vel], nsa.ATOMIC, nsa.FP64)
    outs = static_call([h], [m], [vel], nsa.ATOMIC, nsa.FP64)
    compare(outs, ref, nsa.ATOMIC, nsa.FP64, "after refusals")
    assert np.isfinite(outs[0][0].cpu().numpy()).all()
