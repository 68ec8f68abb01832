"""Host side of the 2-D family (bilinear quadrilaterals): the library's block pattern and element map
bit-exact against the oracle's set-based build, validation codes, and every index the quadrilateral
kernel derives from the row-tile plan (local node ids, owned-vertex masks, block slots) checked on the
CPU against the pattern."""
import numpy as np
import pytest

import oracle
from paper_2111_05651_amd import inputs, nsa


@pytest.fixture(scope="module")
def lib():
    return nsa.load()


MESHES = {
    "grid5x4": lambda: inputs.make_quad_mesh(5, 4, seed=1),
    "perm9x7": lambda: inputs.make_quad_mesh(9, 7, jitter=True, permute=True, seed=2),
    "rcm12": lambda: inputs.make_quad_mesh(12, jitter=True, permute=True, rcm=True, seed=3),
    "cylinder2d": inputs.config_cylinder2d,
    "one": lambda: inputs.make_quad_mesh(1, jitter=True, seed=4),
}


@pytest.mark.parametrize("name", list(MESHES))
def test_q1_pattern_bit_exact(lib, name):
    m = MESHES[name]()
    mesh = nsa.Mesh.from_quads(m)
    assert mesh.family == nsa.QUAD4 and mesh.ndofn == 3
    b, c, e = mesh.pattern()
    ob, oc, oe = oracle.pattern(m.npoin, m.lnods)
    assert np.array_equal(b, ob) and np.array_equal(c, oc) and np.array_equal(e, oe)


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("blocks", [64, 128, 768])
def test_q1_tile_plan(lib, name, blocks):
    m = MESHES[name]()
    mesh = nsa.Mesh.from_quads(m, tile_blocks=blocks, tile_blocks_colour=blocks)
    bptr, bcol, emap = mesh.pattern()
    for scatter in (nsa.ATOMIC, nsa.COLOUR):
        t = mesh.q1_tiles(scatter)
        rows, nptr, eptr = t["tile_row"], t["tile_nptr"], t["tile_eptr"]
        assert rows[0] == 0 and rows[-1] == m.npoin and np.all(np.diff(rows) >= 1)
        lds = mesh.info.tile_lds_bytes[scatter]
        seen = np.zeros((m.nelem, 4), dtype=np.int64)
        for k in range(len(rows) - 1):
            r0, r1 = rows[k], rows[k + 1]
            nodes = t["tile_nodes"][nptr[k]:nptr[k + 1]]
            assert np.array_equal(nodes[:r1 - r0], np.arange(r0, r1))
            nblk = bptr[r1] - bptr[r0]
            nr, nn = r1 - r0, len(nodes)
            need = 8 * ((((9 * nblk + 3 * nr + 1) // 2) * 2) + 4 * nn)
            assert need <= lds <= 160 * 1024
            for p in range(eptr[k], eptr[k + 1]):
                e, rec = t["elems"][p], t["recs"][p]
                g = nodes[rec["loc"].astype(np.int64)]
                assert np.array_equal(g, m.lnods[e])          # local ids map to the element's vertices
                for a in range(4):
                    owned = r0 <= m.lnods[e, a] < r1
                    assert bool((rec["own"] >> a) & 1) == owned
                    if owned:
                        seen[e, a] += 1
                        for bb in range(4):
                            s = int(rec["slot"][4 * a + bb])
                            assert 0 <= s < nblk and s == emap[e, a, bb] - bptr[r0]
        assert np.all(seen == 1), "every (element, vertex) pair owned by exactly one tile"


def test_q1_status_codes(lib):
    m = inputs.make_quad_mesh(3, jitter=True, seed=5)
    bad = m.lnods.copy()
    bad[2, 0] = m.npoin
    with pytest.raises(nsa.NsaError) as ex:
        nsa.Mesh(bad, m.coord, family=nsa.QUAD4)
    assert ex.value.status == nsa.NSA_ERANGE
    bow = m.lnods.copy()
    bow[4] = bow[4][[0, 2, 1, 3]]
    with pytest.raises(nsa.NsaError) as ex:
        nsa.Mesh(bow, m.coord, family=nsa.QUAD4)
    assert ex.value.status == nsa.NSA_EDEGENERATE and "quadrilateral 4" in str(ex.value)
    with pytest.raises(ValueError):
        nsa.Mesh(m.lnods, np.zeros((m.npoin, 3)), family=nsa.QUAD4)
    mesh = nsa.Mesh.from_quads(m)
    for call in (lambda: mesh.tiles(), lambda: mesh.gather(), lambda: mesh.colouring(),
                 lambda: mesh.residual_tiles(), lambda: mesh.scalar_csr()):
        with pytest.raises(nsa.NsaError) as ex:
            call()
        assert ex.value.status == nsa.NSA_EUNSUPPORTED
    with pytest.raises(nsa.NsaError):
        mesh.set_tiling(64, nsa.RESIDUAL_PLAN)
    tet = nsa.Mesh.from_inputs(inputs.make_mesh(2, seed=1))
    with pytest.raises(nsa.NsaError) as ex:
        tet.q1_tiles()
    assert ex.value.status == nsa.NSA_EUNSUPPORTED
