"""The tile planner's record order against the LDS model it is built for (CPU only).

The tiled kernel adds every block value with an 8-byte LDS atomic; the LDS serves such an
instruction 16 lanes at a time, one pass per lane on the busiest bank pair, and value i of tile
block slot s lies on bank pair (s + i) mod 16 (17-double slot stride). Consecutive records go to
consecutive lanes, so for every group of 16 records, owned-row iteration k and column b the planner
tries to put the blocks on distinct bank pairs and in distinct rows. These tests pin that the plan
beats the plain element order by a clear margin, in passes per instruction and in lanes that share
an address (a deterministic-plan tile of ~11 rows cannot give 16 lanes distinct rows, hence its
looser bound)."""
import numpy as np
import pytest

from paper_2111_05651_amd import inputs, nsa


def group_stats(mesh, scatter, order=None):
    """Mean over (group of 16, k, b) instructions of the largest number of lanes on one bank pair,
    and the number of lanes that share an address with an earlier lane of the same instruction."""
    t = mesh.tiles(scatter)
    bptr, _, _ = mesh.pattern()
    tr, te = t["tile_row"], t["tile_eptr"]
    worst, same, n = 0, 0, 0
    for k in range(len(tr) - 1):
        r0, r1 = tr[k], tr[k + 1]
        nr = r1 - r0
        rowoff = bptr[r0:r1 + 1] - bptr[r0]
        recs = t["records"][te[k]:te[k + 1]]
        if order is not None:
            recs = recs[order(recs, nr)]
        loc = recs["loc"].astype(np.int64)
        rank = recs["rank"].astype(np.int64)
        nown = (loc < nr).sum(1)
        for h in range(0, len(recs), 16):
            g = slice(h, h + 16)
            for q in range(4):
                sel = nown[g] > q
                if not sel.any():
                    continue
                lr = loc[g][sel, q]
                for b in range(4):
                    slot = rowoff[lr] + rank[g][sel, q, b]
                    worst += np.bincount(slot % 16).max()
                    same += len(slot) - len(np.unique(slot))
                    n += 1
    return worst / n, same / n


def element_order(recs, nr):
    """The records of a tile in a plain order: owned-row count descending, then by local node ids
    (stands in for element order)."""
    loc = recs["loc"].astype(np.int64)
    nown = (loc < nr).sum(1)
    return np.lexsort((loc[:, 3], loc[:, 2], loc[:, 1], loc[:, 0], -nown))


@pytest.mark.parametrize("scatter", [nsa.ATOMIC, nsa.COLOUR])
@pytest.mark.parametrize("name", ["rcm", "random"])
def test_bank_aware_order(scatter, name):
    m = (inputs.make_mesh(16, jitter=True, permute=True, rcm=True, sort_elements=True, seed=61) if name == "rcm"
         else inputs.make_mesh(12, jitter=True, permute=True, seed=62))
    mesh = nsa.Mesh.from_inputs(m)
    got, got_same = group_stats(mesh, scatter)
    base, base_same = group_stats(mesh, scatter, element_order)
    # the planner's order: clearly fewer passes per instruction than the plain order, and almost no
    # two lanes of one instruction on one address
    assert got <= 0.85 * base, (got, base)
    share = 0.25 if scatter == nsa.ATOMIC else 0.5
    assert got_same <= share * max(base_same, 0.4), (got_same, base_same)
