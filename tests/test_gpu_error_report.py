"""The err_out report of nsa_assemble (nsa_options.err_out): per block class and RHS class, the
largest |value - FP64 value| and the largest |FP64 value| over the sampled elements' element blocks.

Pinned against the oracle: the FP64 maxima must equal the largest entries of the oracle's element
matrices (oracle.element, Listing 1's routine order) over the same sample -- elements floor(i nelem /
ns), ns = min(nelem, 4096) -- which checks the sampling, the class map and the FP64 path. The FP64 form
reports zero differences; the mixed form reports relative errors inside the 1e-5 bar and above zero
(FP32 integration cannot be exact on jittered meshes), on ordinary and on badly shaped elements."""
import sys

import numpy as np
import pytest

import oracle
from paper_2111_05651_amd import inputs, nsa
from tests.parity import TOL_MIXED

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SAMPLE = 4096
CLASSES = nsa.ERR_CLASSES


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def oracle_maxima(m):
    """Largest |entry| per class of the oracle's element matrices and RHS over the sampled elements."""
    ne = m.nelem
    ns = min(ne, SAMPLE)
    mx = np.zeros(6)
    ci = np.array([c for c in range(4)] * 4)  # component of dof 4a + c
    for i in range(ns):
        e = i * ne // ns
        nodes = m.lnods[e].astype(np.int64)
        A, b = oracle.element(m.coord[nodes], m.velocity[nodes], m.rho, m.mu, m.dt)
        rv, cv = ci[:, None] < 3, ci[None, :] < 3
        for k, mask in enumerate((rv & cv, rv & ~cv, ~rv & cv, ~rv & ~cv)):
            mx[k] = max(mx[k], np.abs(A[mask]).max())
        mx[4] = max(mx[4], np.abs(b[ci < 3]).max())
        mx[5] = max(mx[5], np.abs(b[ci == 3]).max())
    return mx


CASES = {
    "cube5_jitter": lambda: inputs.make_mesh(5, jitter=True, permute=True, velocity="vortex", seed=21),
    "cube12_jitter": lambda: inputs.make_mesh(12, jitter=True, permute=True, velocity="vortex", seed=22),
    "soup_eps1e-3": lambda: inputs.bad_element_soup(eps=(1e-3,)),
    "layer_1e-5": lambda: inputs.boundary_layer_mesh(thickness=1e-5),
}


@pytest.mark.parametrize("name", list(CASES))
def test_error_report(name):
    m = CASES[name]()
    say(f"[err_out] {name}: {m.nelem} elements, sample {min(m.nelem, SAMPLE)}")
    mesh = nsa.Mesh.from_inputs(m).upload()
    vel = torch.from_numpy(m.velocity).cuda()
    ref = oracle_maxima(m)
    X = m.coord[m.lnods.astype(np.int64)]
    kappa = np.linalg.cond(X[:, 1:, :] - X[:, :1, :]).max()
    bar64 = max(1e-12, 100 * 2.0 ** -53 * kappa)
    for prec in (nsa.FP64, nsa.MIXED):
        err = torch.full((12,), -1.0, dtype=torch.float64, device="cuda")  # overwritten by the call
        nsa.assemble(mesh, vel, m.rho, m.mu, m.dt, precision=prec, err_out=err)
        torch.cuda.synchronize()
        e = err.cpu().numpy()
        rel_max = np.abs(e[6:] - ref) / ref
        say(f"[err_out] {name} precision={prec}: FP64 maxima vs oracle {rel_max.max():.2e}; "
            f"report {nsa.error_report(err)}")
        assert np.all(ref > 0)
        assert np.all(rel_max <= bar64), (rel_max, bar64)
        rel = e[:6] / e[6:]
        if prec == nsa.FP64:
            assert np.all(e[:6] == 0.0)
        else:
            assert np.all(rel <= TOL_MIXED), dict(zip(CLASSES, rel))
            assert np.all(rel[:4] > 0), dict(zip(CLASSES, rel))


def test_error_report_only_on_assemble():
    m = inputs.make_mesh(3, jitter=True, seed=23)
    mesh = nsa.Mesh.from_inputs(m, tile_rows_residual=64).upload()
    vel = torch.from_numpy(m.velocity).cuda()
    err = torch.zeros(12, dtype=torch.float64, device="cuda")
    o = nsa.make_options(nsa.MIXED)
    o.err_out = err.data_ptr()
    rhsid = torch.zeros((m.npoin, 3), dtype=torch.float64, device="cuda")
    dtr = torch.zeros(m.npoin, dtype=torch.float64, device="cuda")
    mr = torch.zeros(m.npoin, dtype=torch.float64, device="cuda")
    lib = nsa.load()
    st = lib.nsa_assemble_residual(mesh._h, vel.data_ptr(), m.rho, m.mu, m.dt, nsa.C.byref(o), rhsid.data_ptr(),
                                   dtr.data_ptr(), mr.data_ptr(), None)
    assert st == nsa.NSA_EINVAL
    o.err_out = err.data_ptr() + 4  # misaligned
    v, r = mesh.alloc_outputs("cuda")
    st = lib.nsa_assemble(mesh._h, vel.data_ptr(), m.rho, m.mu, m.dt, nsa.C.byref(o), v.data_ptr(), r.data_ptr(),
                          None)
    assert st == nsa.NSA_EINVAL
