"""GPU parity of the explicit-residual path (the outputs of Listing 2: rhsid, dt_rho_nsi,
mass_rho_nsi) against the CPU oracle on the same seeded inputs. Metric per output array:
max |got - ref| / max |ref|, 1e-12 in FP64 and 1e-5 in the mixed form."""
import sys

import numpy as np
import pytest

import oracle
from paper_2111_05651_amd import inputs, nsa
from tests.parity import TOL_FP64, TOL_MIXED

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def errors(got, ref):
    out = {}
    for name, g, r in zip(("rhsid", "dt_rho", "mass_rho"), got, ref):
        den = np.abs(r).max() if r.size else 0.0
        diff = np.abs(np.asarray(g) - r).max() if r.size else 0.0
        out[name] = float(diff / den) if den > 0 else float(diff)
    return out


def run(mesh, m, precision, velocity=None, **kw):
    vel = torch.from_numpy(m.velocity if velocity is None else velocity).cuda()
    outs = nsa.assemble_residual(mesh, vel, kw.get("rho", m.rho), kw.get("mu", m.mu), kw.get("dt", m.dt),
                                 precision=precision)
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


def tol(precision):
    return TOL_FP64 if precision == nsa.FP64 else TOL_MIXED


SMALL = {"cube8": inputs.config_small,
         "cube7_perm": lambda: inputs.make_mesh(7, jitter=True, permute=True, velocity="vortex", seed=41),
         "cube5_rcm": lambda: inputs.make_mesh(5, jitter=True, permute=True, rcm=True, sort_elements=True, seed=42),
         "cube1": lambda: inputs.make_mesh(1, jitter=True, seed=43, rho=1.7, mu=3e-2, dt=2e-3)}


@pytest.mark.parametrize("cfg", list(SMALL))
@pytest.mark.parametrize("rows", [1, 64, 256, 4096])
@pytest.mark.parametrize("precision", [nsa.FP64, nsa.MIXED], ids=["fp64", "mixed"])
def test_small_meshes(cfg, rows, precision):
    m = SMALL[cfg]()
    say(f"[residual] {cfg} nelem={m.nelem} rows={rows} precision={precision}")
    ref = oracle.residual(m)
    mesh = nsa.Mesh.from_inputs(m, tile_blocks=0, tile_blocks_colour=0, tile_rows_residual=rows).upload()
    err = errors(run(mesh, m, precision), ref)
    assert max(err.values()) <= tol(precision), (cfg, rows, err)


def test_uniform_flow_has_no_residual():
    m = inputs.make_mesh(9, jitter=True, permute=True, seed=44, rho=1.3, mu=2e-3, dt=4e-3)
    mesh = nsa.Mesh.from_inputs(m, tile_rows_residual=256).upload()
    U = np.tile(np.array([0.7, -0.4, 0.25]), (m.npoin, 1))
    _, rhs = oracle.assemble(m, velocity=U)
    rhsid, _, _ = run(mesh, m, nsa.FP64, velocity=U)
    assert np.abs(rhsid).max() <= 1e-12 * np.abs(rhs[:, :3]).max()


def test_accumulate_and_empty():
    m = inputs.make_mesh(4, jitter=True, permute=True, seed=45)
    ref = oracle.residual(m)
    mesh = nsa.Mesh.from_inputs(m, tile_rows_residual=64).upload()
    vel = torch.from_numpy(m.velocity).cuda()
    r = torch.full((m.npoin, 3), 1.0, dtype=torch.float64, device="cuda")
    t = torch.full((m.npoin,), -2.0, dtype=torch.float64, device="cuda")
    w = torch.full((m.npoin,), 3.0, dtype=torch.float64, device="cuda")
    for _ in range(2):
        nsa.assemble_residual(mesh, vel, m.rho, m.mu, m.dt, accumulate=True, rhsid=r, dt_rho=t, mass_rho=w)
    torch.cuda.synchronize()
    got = [r.cpu().numpy() - 1.0, t.cpu().numpy() + 2.0, w.cpu().numpy() - 3.0]
    err = errors(got, [2 * x for x in ref])
    assert max(err.values()) <= 1e-12, err
    empty = nsa.Mesh(np.zeros((0, 4), np.int32), np.zeros((3, 3)), tile_rows_residual=16).upload()
    outs = nsa.assemble_residual(empty, torch.zeros((3, 3), dtype=torch.float64, device="cuda"), 1.0, 1e-3, 1e-2)
    torch.cuda.synchronize()
    assert all(torch.all(o == 0) for o in outs)


@pytest.mark.parametrize("name", ["cube64", "cube128"])
def test_full_meshes(name):
    """Every output of the 64^3 (randomly numbered) and 128^3 (RCM) workloads against the oracle."""
    m = {"cube64": inputs.config_64, "cube128": inputs.config_128}[name]()
    say(f"[residual] {name} nelem={m.nelem}: oracle ...")
    ref = oracle.residual(m)
    mesh = nsa.Mesh.from_inputs(m, tile_blocks=0, tile_blocks_colour=0, tile_rows_residual=256,
                                keep_direct=False).upload()
    for precision in (nsa.FP64, nsa.MIXED):
        err = errors(run(mesh, m, precision), ref)
        say(f"[residual] {name} precision={precision} errors {err}")
        assert max(err.values()) <= tol(precision), err


@pytest.mark.parametrize("cfg", ["cube7_perm", "cube5_rcm", "cube1"])
@pytest.mark.parametrize("rows", [1, 64, 256])
@pytest.mark.parametrize("precision", [nsa.FP64, nsa.MIXED], ids=["fp64", "mixed"])
def test_precomputed_geometry(cfg, rows, precision):
    """nsa_mesh_set_residual_geometry: the residual kernel reading stored element geometry (in the
    record's vertex order) gives the oracle's outputs, and within 1e-12 the formed-geometry kernel's."""
    m = SMALL[cfg]()
    say(f"[residual] cached geometry {cfg} rows={rows} precision={precision}")
    ref = oracle.residual(m)
    cached = nsa.Mesh.from_inputs(m, tile_blocks=0, tile_blocks_colour=0, tile_rows_residual=rows,
                                  residual_geometry=True).upload()
    plain = nsa.Mesh.from_inputs(m, tile_blocks=0, tile_blocks_colour=0, tile_rows_residual=rows).upload()
    got = run(cached, m, precision)
    err = errors(got, ref)
    assert max(err.values()) <= tol(precision), (cfg, rows, err)
    same = errors(got, run(plain, m, precision))
    assert max(same.values()) <= (1e-12 if precision == nsa.FP64 else 1e-6), same


def test_precomputed_geometry_cube64():
    m = inputs.config_64()
    ref = oracle.residual(m)
    mesh = nsa.Mesh.from_inputs(m, tile_blocks=0, tile_blocks_colour=0, tile_rows_residual=256, keep_direct=False,
                                residual_geometry=True).upload()
    for precision in (nsa.FP64, nsa.MIXED):
        err = errors(run(mesh, m, precision), ref)
        say(f"[residual] cached geometry cube64 precision={precision} errors {err}")
        assert max(err.values()) <= tol(precision), err
