"""GPU parity: the HIP path through the C-ABI against the CPU oracle on the same seeded inputs.

Bar (block-class metric of parity.py): 1e-12 for FP64, 1e-5 for the mixed form; the pattern and
element-to-block map bit-exact; the colouring path bit-identical run to run."""
import sys

import numpy as np
import pytest

import oracle
from paper_2111_05651_amd import inputs, nsa
from tests.parity import TOL_FP64, TOL_MIXED, assert_parity, class_errors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MODES = [(nsa.FP64, nsa.ATOMIC), (nsa.FP64, nsa.COLOUR), (nsa.MIXED, nsa.ATOMIC), (nsa.MIXED, nsa.COLOUR)]


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gpu_assemble(mesh, m, precision, scatter, kernel=nsa.KERNEL_AUTO, vel=None, **kw):
    v = torch.from_numpy(m.velocity if vel is None else vel).cuda()
    values, rhs = nsa.assemble(mesh, v, kw.pop("rho", m.rho), kw.pop("mu", m.mu), kw.pop("dt", m.dt),
                               precision=precision, scatter=scatter, kernel=kernel, **kw)
    torch.cuda.synchronize()
    return values.cpu().numpy(), rhs.cpu().numpy()


def tol_of(precision):
    return TOL_FP64 if precision == nsa.FP64 else TOL_MIXED


SMALL = {"cube8": inputs.config_small,
         "cube7_perm": lambda: inputs.make_mesh(7, jitter=True, permute=True, velocity="vortex", seed=17),
         "cube5_rcm": lambda: inputs.make_mesh(5, jitter=True, permute=True, rcm=True, sort_elements=True, seed=18),
         "cube3": lambda: inputs.make_mesh(3, jitter=True, velocity="uniform", seed=19, rho=1.7, mu=3e-2, dt=2e-3)}
KERNELS = [("direct", nsa.KERNEL_DIRECT, None), ("tiled64", nsa.KERNEL_TILED, 64),
           ("tiled_default", nsa.KERNEL_TILED, None), ("tiled1024", nsa.KERNEL_TILED, 1024),
           ("gather64", nsa.KERNEL_GATHER, 64), ("gather320", nsa.KERNEL_GATHER, 320),
           ("gather4096_512thr", nsa.KERNEL_GATHER, 4096)]


def mesh_for(m, kern):
    """Mesh with the plan a KERNELS entry asks for."""
    if kern[1] == nsa.KERNEL_GATHER:
        return nsa.Mesh.from_inputs(m, tile_blocks_gather=kern[2]).upload()
    return nsa.Mesh.from_inputs(m, tile_blocks=kern[2], tile_blocks_colour=kern[2]).upload()


def kernel_kw(kern):
    return dict(block_threads=512) if kern[0].endswith("512thr") else {}


@pytest.mark.parametrize("cfg", list(SMALL))
@pytest.mark.parametrize("kern", KERNELS, ids=lambda k: k[0])
@pytest.mark.parametrize("mode", MODES, ids=lambda m: f"{'fp64' if m[0] == 0 else 'mixed'}-{'atomic' if m[1] == 0 else 'colour'}")
def test_small_meshes(cfg, kern, mode):
    m = SMALL[cfg]()
    say(f"[parity] {cfg} nelem={m.nelem} kernel={kern[0]} mode={mode}")
    ref_v, ref_r = oracle.assemble(m)
    mesh = mesh_for(m, kern)
    v, r = gpu_assemble(mesh, m, *mode, kernel=kern[1], **kernel_kw(kern))
    assert_parity(v, ref_v, r, ref_r, tol_of(mode[0]), f"{cfg} {kern[0]} {mode}")


def test_degenerate_parameters():
    """mu = 0 with zero velocity (pure mass/Laplacian), huge and tiny dt, zero velocity RHS."""
    m = inputs.make_mesh(4, jitter=True, permute=True, seed=23)
    mesh = nsa.Mesh.from_inputs(m, tile_blocks_gather=320).upload()
    for rho, mu, dt, vel in ((1.0, 0.0, 1e-2, np.zeros_like(m.velocity)), (2.0, 1e-3, 1e6, m.velocity),
                             (0.5, 1e-1, 1e-9, m.velocity), (1.0, 1e-3, 1e-2, np.zeros_like(m.velocity))):
        ref_v, ref_r = oracle.assemble(m, rho=rho, mu=mu, dt=dt, velocity=vel)
        for mode in MODES + [(p, s_, k) for p, s_ in MODES for k in (nsa.KERNEL_DIRECT, nsa.KERNEL_GATHER)]:
            v, r = gpu_assemble(mesh, m, *mode, vel=vel, rho=rho, mu=mu, dt=dt)
            err = class_errors(v, ref_v, r, ref_r)
            for k, e in err.items():
                if k.startswith("rhs") and np.abs(ref_r).max() == 0:
                    assert np.abs(r).max() == 0
                    continue
                assert e <= tol_of(mode[0]), (rho, mu, dt, mode, err)



def test_tiny_velocity_fp64():
    """Velocities of order 1e-152: every element's squared velocity sum lies below 1e-300, where the
    kernels take the velocity norm in tau as 0 (beside rho/dt it is far below FP64 resolution there)
    while the oracle takes the exact norm. Catches a NaN or infinity from the reciprocal square root
    of such a value. FP64 only: FP32 cannot represent these velocities."""
    m = inputs.make_mesh(4, jitter=True, permute=True, velocity="vortex", seed=25)
    vel = np.ascontiguousarray(m.velocity * 1e-152)
    su = vel[m.lnods].sum(axis=1)
    assert (su * su).sum(axis=1).max() < 1e-300 and np.abs(vel).max() > 1e-153
    say(f"[tiny velocity] nelem={m.nelem}")
    ref_v, ref_r = oracle.assemble(m, velocity=vel)
    mesh = nsa.Mesh.from_inputs(m, tile_blocks_gather=320, tile_rows_residual=64).upload()
    for scat in (nsa.ATOMIC, nsa.COLOUR):
        for kern in (nsa.KERNEL_TILED, nsa.KERNEL_DIRECT, nsa.KERNEL_GATHER):
            v, r = gpu_assemble(mesh, m, nsa.FP64, scat, kernel=kern, vel=vel)
            assert np.isfinite(v).all() and np.isfinite(r).all()
            assert_parity(v, ref_v, r, ref_r, TOL_FP64, f"tiny velocity {scat} {kern}")
    ref = oracle.residual(m, velocity=vel)
    outs = nsa.assemble_residual(mesh, torch.from_numpy(vel).cuda(), m.rho, m.mu, m.dt, precision=nsa.FP64)
    torch.cuda.synchronize()
    for name, g, r in zip(("rhsid", "dt_rho", "mass_rho"), outs, ref):
        g = g.cpu().numpy()
        assert np.isfinite(g).all(), name
        assert np.abs(g - r).max() <= TOL_FP64 * np.abs(r).max(), name

def test_accumulate():
    m = inputs.make_mesh(4, jitter=True, permute=True, seed=24)
    ref_v, ref_r = oracle.assemble(m)
    mesh = nsa.Mesh.from_inputs(m, tile_blocks_gather=320).upload()
    vel = torch.from_numpy(m.velocity).cuda()
    values, rhs = mesh.alloc_outputs()
    values.fill_(1.0)
    rhs.fill_(-2.0)
    for kernel in (nsa.KERNEL_TILED, nsa.KERNEL_DIRECT, nsa.KERNEL_GATHER):
        for scatter in (nsa.ATOMIC, nsa.COLOUR):
            values.fill_(1.0)
            rhs.fill_(-2.0)
            for _ in range(2):
                nsa.assemble(mesh, vel, m.rho, m.mu, m.dt, scatter=scatter, accumulate=True, values=values, rhs=rhs,
                             kernel=kernel)
            torch.cuda.synchronize()
            assert_parity(values.cpu().numpy() - 1.0, 2 * ref_v, rhs.cpu().numpy() + 2.0, 2 * ref_r, 1e-12,
                          f"accumulate kernel={kernel} scatter={scatter}")


def test_colour_path_bit_reproducible():
    m = inputs.make_mesh(12, jitter=True, permute=True, velocity="vortex", seed=25)
    mesh = nsa.Mesh.from_inputs(m, tile_blocks_gather=320).upload()
    for kernel in (nsa.KERNEL_TILED, nsa.KERNEL_DIRECT, nsa.KERNEL_GATHER):
        for prec in (nsa.FP64, nsa.MIXED):
            v0, r0 = gpu_assemble(mesh, m, prec, nsa.COLOUR, kernel=kernel)
            for _ in range(9):
                v, r = gpu_assemble(mesh, m, prec, nsa.COLOUR, kernel=kernel)
                assert np.array_equal(v, v0) and np.array_equal(r, r0)


def test_colour_path_reproducible_under_load():
    """Bit-identical results while another stream keeps the GPU busy (different wave interleavings),
    and across different launch streams."""
    m = inputs.make_mesh(20, jitter=True, permute=True, velocity="vortex", seed=27)
    mesh = nsa.Mesh.from_inputs(m, tile_blocks_gather=320).upload()
    vel = torch.from_numpy(m.velocity).cuda()
    v0, r0 = nsa.assemble(mesh, vel, m.rho, m.mu, m.dt, scatter=nsa.COLOUR)
    torch.cuda.synchronize()
    v0, r0 = v0.cpu().numpy(), r0.cpu().numpy()
    side = torch.cuda.Stream()
    a = torch.randn(2048, 2048, device="cuda")
    for it in range(12):
        with torch.cuda.stream(side):
            for _ in range(4):
                a = (a @ a).tanh_()
        s = torch.cuda.Stream() if it % 2 else torch.cuda.current_stream()
        with torch.cuda.stream(s):
            v, r = nsa.assemble(mesh, vel, m.rho, m.mu, m.dt, scatter=nsa.COLOUR, stream=s)
        torch.cuda.synchronize()
        assert np.array_equal(v.cpu().numpy(), v0) and np.array_equal(r.cpu().numpy(), r0), f"run {it}"


def test_binding_rejects_bad_tensors():
    """The C entry points take bare pointers; the binding refuses tensors that would make a kernel
    read or write outside them, before any launch."""
    m = inputs.make_mesh(2, jitter=True, seed=3)
    mesh = nsa.Mesh.from_inputs(m).upload()
    vel = torch.from_numpy(m.velocity).cuda()
    values, rhs = mesh.alloc_outputs()
    bad_vel = [vel.float(), vel[:-1], vel.t().contiguous(), vel.t(), vel.cpu()]
    for v in bad_vel:
        with pytest.raises(ValueError):
            nsa.assemble(mesh, v, m.rho, m.mu, m.dt, values=values, rhs=rhs)
    with pytest.raises(ValueError):
        nsa.assemble(mesh, vel, m.rho, m.mu, m.dt, values=values[:-1], rhs=rhs)
    with pytest.raises(ValueError):
        nsa.assemble(mesh, vel, m.rho, m.mu, m.dt, values=values, rhs=rhs.t())
    with pytest.raises(ValueError):
        nsa.assemble_residual(mesh, vel, m.rho, m.mu, m.dt, rhsid=torch.empty((m.npoin, 3), device="cuda"))
    # the well-formed call still works after the refusals
    v, r = nsa.assemble(mesh, vel, m.rho, m.mu, m.dt, values=values, rhs=rhs)
    torch.cuda.synchronize()
    ref_v, ref_r = oracle.assemble(m)
    assert_parity(v.cpu().numpy(), ref_v, r.cpu().numpy(), ref_r, TOL_FP64, "after refusals")


def test_empty_and_tiny():
    mesh = nsa.Mesh(np.zeros((0, 4), np.int32), np.zeros((3, 3))).upload()
    vel = torch.zeros((3, 3), dtype=torch.float64, device="cuda")
    values, rhs = mesh.alloc_outputs()
    rhs.fill_(7.0)
    nsa.assemble(mesh, vel, 1.0, 1e-3, 1e-2, values=values, rhs=rhs)
    torch.cuda.synchronize()
    assert values.numel() == 0 and torch.all(rhs == 0)
    m = inputs.make_mesh(1, jitter=True, seed=26)           # 6 tets
    ref_v, ref_r = oracle.assemble(m)
    mesh = nsa.Mesh.from_inputs(m, tile_blocks_gather=320).upload()
    for kernel in (nsa.KERNEL_TILED, nsa.KERNEL_DIRECT, nsa.KERNEL_GATHER):
        for mode in MODES:
            v, r = gpu_assemble(mesh, m, *mode, kernel=kernel)
            assert_parity(v, ref_v, r, ref_r, tol_of(mode[0]), f"one hex {mode} kernel={kernel}")


@pytest.mark.parametrize("scatter", [nsa.ATOMIC, nsa.COLOUR])
def test_cube64_full(scatter):
    """The 64^3 workload (1,572,864 tets, nodes randomly permuted), every entry against the oracle."""
    m = inputs.config_64()
    say(f"[parity] cube64 nelem={m.nelem} scatter={scatter}: oracle ...")
    pat = oracle.pattern(m.npoin, m.lnods)
    ref_v, ref_r = oracle.assemble(m, pat)
    mesh = nsa.Mesh.from_inputs(m, tile_blocks_gather=320).upload()
    bptr, bcol, emap = mesh.pattern()
    assert np.array_equal(bptr, pat[0]) and np.array_equal(bcol, pat[1]) and np.array_equal(emap, pat[2])
    for kernel in (nsa.KERNEL_TILED, nsa.KERNEL_DIRECT, nsa.KERNEL_GATHER):
        for prec in (nsa.FP64, nsa.MIXED):
            say(f"[parity] cube64 kernel={kernel} precision={prec} scatter={scatter}")
            v, r = gpu_assemble(mesh, m, prec, scatter, kernel=kernel)
            err = assert_parity(v, ref_v, r, ref_r, tol_of(prec), f"cube64 {prec} {scatter} kernel={kernel}")
            say(f"[parity] cube64 errors {err}")


def device_class_errors(v, ref_v, r, ref_r):
    """The parity metric of tests/parity.py (per class max |got - ref| / max |ref|) on device tensors."""
    v, ref_v, r, ref_r = v.view(-1, 4, 4), ref_v.view(-1, 4, 4), r.view(-1, 4), ref_r.view(-1, 4)
    out = {}
    for k, (a, b) in {"uu": (slice(0, 3), slice(0, 3)), "up": (slice(0, 3), slice(3, 4)),
                      "pu": (slice(3, 4), slice(0, 3)), "pp": (slice(3, 4), slice(3, 4))}.items():
        out[k] = float((v[:, a, b] - ref_v[:, a, b]).abs().max() / ref_v[:, a, b].abs().max())
    for k, sel in (("rhs_u", slice(0, 3)), ("rhs_p", slice(3, 4))):
        out[k] = float((r[:, sel] - ref_r[:, sel]).abs().max() / ref_r[:, sel].abs().max())
    return out


def test_cube128_whole_mesh():
    """The 128^3 workload (12,582,912 tets, 509M matrix values) element by element against the
    oracle, which assembles the whole mesh (set-based pattern, Gauss-rule element pipeline): the
    pattern and element-to-block map bit-exact; the benchmark's launch (tiled kernel, 512-block
    tiles, atomic scatter) and the deterministic tiled plan in both precisions, the direct kernel with
    its global colour classes and the gather kernel, every entry within the bar of its precision;
    the deterministic plan repeats bit for bit."""
    m = inputs.config_128()
    say(f"[parity] cube128 whole mesh nelem={m.nelem}: oracle pattern and assembly ...")
    pat = oracle.pattern(m.npoin, m.lnods)
    ref_v, ref_r = oracle.assemble(m, pat)
    mesh = nsa.Mesh.from_inputs(m, tile_blocks=512, tile_blocks_gather=320).upload()
    bptr, bcol, emap = mesh.pattern()
    assert np.array_equal(bptr, pat[0]) and np.array_equal(bcol, pat[1]) and np.array_equal(emap, pat[2])
    del pat, bcol, emap
    ref_v = torch.from_numpy(ref_v).cuda()
    ref_r = torch.from_numpy(ref_r).cuda()
    vel = torch.from_numpy(m.velocity).cuda()

    def run(precision, scatter, kernel):
        out = nsa.assemble(mesh, vel, m.rho, m.mu, m.dt, precision=precision, scatter=scatter, kernel=kernel)
        torch.cuda.synchronize()
        return out

    cases = [("tiled atomic", nsa.ATOMIC, nsa.KERNEL_TILED), ("tiled deterministic", nsa.COLOUR, nsa.KERNEL_TILED),
             ("gather", nsa.ATOMIC, nsa.KERNEL_GATHER), ("direct colour classes", nsa.COLOUR, nsa.KERNEL_DIRECT)]
    for prec in (nsa.FP64, nsa.MIXED):
        for name, scat, kern in cases:
            if kern == nsa.KERNEL_DIRECT and prec == nsa.MIXED:
                continue
            say(f"[parity] cube128 whole mesh {name} precision={prec}")
            v, r = run(prec, scat, kern)
            err = device_class_errors(v, ref_v, r, ref_r)
            say(f"[parity] cube128 whole mesh {name} precision={prec}: {err}")
            assert max(err.values()) <= tol_of(prec), (name, prec, err)
            if name == "tiled deterministic":
                v2, r2 = run(prec, scat, kern)
                assert torch.equal(v, v2) and torch.equal(r, r2), "deterministic plan: bitwise repeat"
                del v2, r2
            del v, r
            torch.cuda.empty_cache()


def test_gather_bitwise_independent_of_tiling_and_mode():
    """Each block is summed in element order whatever the tile size, the workgroup size or the
    scatter mode: all of them give the same bits."""
    m = inputs.make_mesh(10, jitter=True, permute=True, velocity="vortex", seed=29)
    for prec in (nsa.FP64, nsa.MIXED):
        base = None
        for tb, nt in ((64, 256), (512, 256), (4096, 512), (300, 512)):
            mesh = nsa.Mesh.from_inputs(m, tile_blocks_gather=tb).upload()
            for scatter in (nsa.ATOMIC, nsa.COLOUR):
                v, r = gpu_assemble(mesh, m, prec, scatter, kernel=nsa.KERNEL_GATHER, block_threads=nt)
                if base is None:
                    base = (v, r)
                assert np.array_equal(v, base[0]) and np.array_equal(r, base[1]), (prec, tb, nt, scatter)


@pytest.mark.parametrize("level", [2, 4])
def test_high_degree_hub(level):
    """A node in 128 / 2048 elements: every kernel the mesh supports (the row-tiled one only for
    rows up to 256 blocks; the direct one with 128 / 2048 global colours; the residual path)
    against the oracle."""
    m = inputs.hub_mesh(level, seed=level)
    say(f"[parity] hub level {level} nelem={m.nelem}")
    ref_v, ref_r = oracle.assemble(m)
    ref_res = oracle.residual(m)
    mesh = nsa.Mesh.from_inputs(m, tile_rows_residual=64, tile_blocks_gather=512).upload()
    kernels = [nsa.KERNEL_AUTO, nsa.KERNEL_DIRECT]
    if mesh.info.ntiles[0]:
        kernels.append(nsa.KERNEL_TILED)
    if mesh.info.gather_ntiles:
        kernels.append(nsa.KERNEL_GATHER)
    for kernel in kernels:
        for mode in MODES:
            v, r = gpu_assemble(mesh, m, *mode, kernel=kernel)
            assert_parity(v, ref_v, r, ref_r, tol_of(mode[0]), f"hub {level} {mode} kernel={kernel}")
    if not mesh.info.ntiles[0]:
        with pytest.raises(nsa.NsaError):
            gpu_assemble(mesh, m, nsa.FP64, nsa.ATOMIC, kernel=nsa.KERNEL_TILED)
    vel = torch.from_numpy(m.velocity).cuda()
    for prec in (nsa.FP64, nsa.MIXED):
        got = [x.cpu().numpy() for x in nsa.assemble_residual(mesh, vel, m.rho, m.mu, m.dt, precision=prec)]
        for g, ref in zip(got, ref_res):
            assert np.abs(g - ref).max() <= tol_of(prec) * np.abs(ref).max()
