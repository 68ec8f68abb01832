"""Host-side tests of libnsa (no GPU): exports, pattern bit-exactness against the oracle,
colouring validity, validation status codes and argument checking."""
import re
import os

import numpy as np
import pytest

import oracle
from paper_2111_05651_amd import inputs, nsa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return nsa.load()


def header_functions():
    src = open(os.path.join(ROOT, "include", "nsa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nsa_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert names, "no declarations found"
    assert sorted(nsa.EXPORTS) == names
    for n in names:
        assert hasattr(lib, n), f"libnsa.so does not export {n}"
    assert lib.nsa_version() >= 100


@pytest.mark.parametrize("cfg", ["small", "perm4", "rcm5"])
def test_pattern_bit_exact(lib, cfg):
    m = {"small": lambda: inputs.config_small(),
         "perm4": lambda: inputs.make_mesh(4, jitter=True, permute=True, seed=7),
         "rcm5": lambda: inputs.make_mesh(5, jitter=True, permute=True, rcm=True, sort_elements=True, seed=8)}[cfg]()
    ob, oc, oe = oracle.pattern(m.npoin, m.lnods)
    nb, nc, ne = nsa.pattern(m.npoin, m.lnods)
    assert np.array_equal(ob, nb) and np.array_equal(oc, nc) and np.array_equal(oe, ne)
    mesh = nsa.Mesh.from_inputs(m)
    mb, mc, me = mesh.pattern()
    assert np.array_equal(ob, mb) and np.array_equal(oc, mc) and np.array_equal(oe, me)
    assert mesh.nnzb == inputs.cube_counts(m.n)[3]


def test_pattern_64_bit_exact(lib):
    m = inputs.make_mesh(24, jitter=True, permute=True, seed=9)
    ob, oc, oe = oracle.pattern(m.npoin, m.lnods)
    nb, nc, ne = nsa.pattern(m.npoin, m.lnods)
    assert np.array_equal(ob, nb) and np.array_equal(oc, nc) and np.array_equal(oe, ne)


def test_colouring_is_valid(lib):
    m = inputs.make_mesh(6, jitter=True, permute=True, seed=10)
    mesh = nsa.Mesh.from_inputs(m)
    cptr, celems = mesh.colouring()
    assert cptr[0] == 0 and cptr[-1] == m.nelem
    assert np.array_equal(np.sort(celems), np.arange(m.nelem))
    for c in range(len(cptr) - 1):
        els = celems[cptr[c]:cptr[c + 1]]
        assert np.all(np.diff(els) > 0)
        nodes = m.lnods[els].ravel()
        assert np.unique(nodes).size == nodes.size, f"colour {c} has elements sharing a node"
    # an interior Kuhn node lies in 24 tets: at least 24 colours
    assert 24 <= mesh.info.ncolours <= 40


def test_status_codes(lib):
    m = inputs.make_mesh(2, jitter=True, seed=3)
    bad = m.lnods.copy()
    bad[5, 1] = -1
    with pytest.raises(nsa.NsaError) as ei:
        nsa.Mesh(bad, m.coord)
    assert ei.value.status == nsa.NSA_ERANGE and "element 5" in str(ei.value)
    flat = m.coord.copy()
    flat[m.lnods[7]] = flat[m.lnods[7][0]]
    with pytest.raises(nsa.NsaError) as ei:
        nsa.Mesh(m.lnods, flat)
    assert ei.value.status == nsa.NSA_EDEGENERATE
    nanc = m.coord.copy()
    nanc[m.lnods[3][2], 1] = np.nan
    with pytest.raises(nsa.NsaError) as ei:
        nsa.Mesh(m.lnods, nanc)
    assert ei.value.status == nsa.NSA_EDEGENERATE
    # assemble before upload: refused on the host, nothing launched
    mesh = nsa.Mesh.from_inputs(m)
    import ctypes as C
    o = nsa.make_options()
    st = lib.nsa_assemble(mesh._h, 16, 1.0, 1e-3, 1e-2, C.byref(o), 16, 16, None)
    assert st == nsa.NSA_ESTATE
    assert lib.nsa_mesh_get_info(None, None) == nsa.NSA_EINVAL
    assert lib.nsa_mesh_upload(mesh._h, None, 0, None) == nsa.NSA_EINVAL
    assert lib.nsa_mesh_release_host(mesh._h) == nsa.NSA_ESTATE


def test_empty_mesh(lib):
    mesh = nsa.Mesh(np.zeros((0, 4), np.int32), np.zeros((5, 3)))
    assert mesh.nelem == 0 and mesh.nnzb == 0 and mesh.info.ncolours == 0
    bptr, bcol, _ = mesh.pattern()
    assert np.array_equal(bptr, np.zeros(6)) and bcol.size == 0


def test_isolated_nodes_match_oracle(lib):
    m = inputs.make_mesh(2, jitter=True, seed=4)
    # three extra nodes that belong to no element, one of them in the middle of the numbering
    coord = np.vstack([m.coord, np.ones((3, 3))])
    ln = m.lnods.copy()
    ln[ln >= 10] += 1
    coord = np.vstack([coord[:10], [[5.0, 5, 5]], coord[10:m.npoin], [[6.0, 6, 6], [7.0, 7, 7]]])
    ob, oc, oe = oracle.pattern(coord.shape[0], ln)
    mesh = nsa.Mesh(ln, coord)
    mb, mc, me = mesh.pattern()
    assert np.array_equal(ob, mb) and np.array_equal(oc, mc) and np.array_equal(oe, me)
    assert mb[11] == mb[10]
