"""Seeded synthetic inputs: jittered Kuhn-cube tetrahedral meshes and nodal velocity fields.

This module only *generates inputs*. It holds none of the assembly arithmetic, so both the
CPU oracle's tests and the GPU path draw their meshes from here.

The paper evaluates on Alya's benchmark meshes (Table 2: 1.2k to 32.7M elements, about 5.7-5.8
tetrahedra per node for the Sphere cases). Those meshes are not available, so unit cubes split
into hexahedra and each hexahedron into six Kuhn tetrahedra stand in for them: a 64^3 cube gives
1,572,864 tets on 274,625 nodes, a 128^3 cube 12,582,912 tets on 2,146,689 nodes.

Node ids: (i, j, k) -> i + (n+1) * (j + (n+1) * k) before any renumbering.
Element order: hexes with i fastest, then j, then k; six tets per hex in the axis-permutation
order (x,y,z), (x,z,y), (y,x,z), (y,z,x), (z,x,y), (z,y,x). Every tet is positively oriented.

Random draws use ``numpy.random.default_rng(seed)`` in this fixed order:
jitter (npoin x 3), then node permutation, then velocity noise.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Kuhn split of the unit hex along its (0,0,0)->(1,1,1) diagonal: one tet per permutation
# of the axes. Vertex path: origin, +e_p0, +e_p1, +e_p2.
_AXIS_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def _perm_sign(p):
    s = 1
    for i in range(3):
        for j in range(i + 1, 3):
            if p[i] > p[j]:
                s = -s
    return s


def _kuhn_corner_table():
    """(6, 4, 3) int array of hex-corner offsets for each tet, positively oriented."""
    tab = np.zeros((6, 4, 3), dtype=np.int64)
    for t, p in enumerate(_AXIS_PERMS):
        v = np.zeros(3, dtype=np.int64)
        verts = [v.copy()]
        for ax in p:
            v[ax] += 1
            verts.append(v.copy())
        if _perm_sign(p) < 0:  # odd permutation: swap two vertices to flip the orientation
            verts[2], verts[3] = verts[3], verts[2]
        tab[t] = np.array(verts)
    return tab


@dataclasses.dataclass
class Mesh:
    """A linear-tetrahedron mesh with a nodal velocity field (all host NumPy arrays)."""
    n: int                    # hexes per cube edge
    lnods: np.ndarray         # int32 [nelem][4], 0-based node ids
    coord: np.ndarray         # float64 [npoin][3]
    velocity: np.ndarray      # float64 [npoin][3]
    rho: float = 1.0
    mu: float = 1e-3
    dt: float = 1e-2
    name: str = ""

    @property
    def npoin(self) -> int:
        return int(self.coord.shape[0])

    @property
    def nelem(self) -> int:
        return int(self.lnods.shape[0])


def cube_counts(n: int):
    """(npoin, nelem, nedges, nnzb) of the Kuhn-split n^3 cube (closed forms)."""
    npoin = (n + 1) ** 3
    nelem = 6 * n ** 3
    edges = 3 * n * (n + 1) ** 2 + 3 * n ** 2 * (n + 1) + n ** 3
    return npoin, nelem, edges, npoin + 2 * edges


def kuhn_cube(n: int):
    """Unjittered Kuhn cube: (lnods int32 [6n^3][4], coord float64 [(n+1)^3][3])."""
    m = n + 1
    g = np.arange(m, dtype=np.float64) / n
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    coord = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = (i + m * (j + m * k)).ravel().astype(np.int64)           # hex origin node, i fastest
    tab = _kuhn_corner_table()                                       # (6,4,3)
    off = tab[..., 0] + m * (tab[..., 1] + m * tab[..., 2])          # (6,4)
    lnods = (base[:, None, None] + off[None, :, :]).reshape(-1, 4)
    return lnods.astype(np.int32), coord


def taylor_green(coord: np.ndarray) -> np.ndarray:
    """Smooth vortex (Taylor-Green) velocity at the given points, float64 [npoin][3]."""
    x, y, z = coord[:, 0], coord[:, 1], coord[:, 2]
    px, py, pz = math.pi * x, math.pi * y, math.pi * z
    u = np.sin(px) * np.cos(py) * np.cos(pz)
    v = -np.cos(px) * np.sin(py) * np.cos(pz)
    return np.stack([u, v, np.zeros_like(u)], axis=1)


def node_graph_rcm(lnods: np.ndarray, npoin: int) -> np.ndarray:
    """Reverse Cuthill-McKee order of the node graph (SciPy); returns new_id[old_id]."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee

    ln = lnods.astype(np.int64)
    rows, cols = [], []
    for a in range(4):
        for b in range(a + 1, 4):
            lo = np.minimum(ln[:, a], ln[:, b])
            hi = np.maximum(ln[:, a], ln[:, b])
            rows.append(lo)
            cols.append(hi)
    key = np.unique(np.concatenate(rows) * npoin + np.concatenate(cols))
    lo, hi = key // npoin, key % npoin
    r = np.concatenate([lo, hi])
    c = np.concatenate([hi, lo])
    g = sp.csr_matrix((np.ones(r.size, dtype=np.int8), (r, c)), shape=(npoin, npoin))
    order = reverse_cuthill_mckee(g, symmetric_mode=True)            # order[k] = old id at slot k
    new_id = np.empty(npoin, dtype=np.int64)
    new_id[order] = np.arange(npoin, dtype=np.int64)
    return new_id


def make_mesh(n: int, *, jitter: bool = False, permute: bool = False, rcm: bool = False,
              sort_elements: bool = False, velocity: str = "uniform", seed: int = 0,
              rho: float = 1.0, mu: float = 1e-3, dt: float = 1e-2, name: str = "") -> Mesh:
    """Build a seeded Kuhn-cube mesh.

    jitter        every node coordinate component moves by U[-0.2h, 0.2h], h = 1/n
                  (keeps every tet positively oriented: the smallest altitude is h/sqrt(2)).
    permute       random relabelling of the nodes.
    rcm           after the permutation, renumber by reverse Cuthill-McKee on the node graph.
    sort_elements stable sort of the elements by their smallest node id.
    velocity      "uniform": U[-1,1]^3 per node; "vortex": Taylor-Green at the (jittered)
                  coordinates plus 0.01 * U[-1,1]^3.
    """
    rng = np.random.default_rng(seed)
    lnods, coord = kuhn_cube(n)
    npoin = coord.shape[0]
    if jitter:
        h = 1.0 / n
        coord = coord + rng.uniform(-0.2 * h, 0.2 * h, size=(npoin, 3))
    if permute:
        perm = rng.permutation(npoin)                                # new id of old node
        new_coord = np.empty_like(coord)
        new_coord[perm] = coord
        coord = new_coord
        lnods = perm[lnods].astype(np.int32)
    if velocity == "uniform":
        vel = rng.uniform(-1.0, 1.0, size=(npoin, 3))
    elif velocity == "vortex":
        vel = taylor_green(coord) + 0.01 * rng.uniform(-1.0, 1.0, size=(npoin, 3))
    elif velocity == "zero":
        vel = np.zeros((npoin, 3))
    else:
        raise ValueError(f"unknown velocity field {velocity!r}")
    if rcm:
        new_id = node_graph_rcm(lnods, npoin)
        new_coord = np.empty_like(coord)
        new_coord[new_id] = coord
        new_vel = np.empty_like(vel)
        new_vel[new_id] = vel
        coord, vel = new_coord, new_vel
        lnods = new_id[lnods].astype(np.int32)
    if sort_elements:
        order = np.argsort(lnods.min(axis=1), kind="stable")
        lnods = np.ascontiguousarray(lnods[order])
    return Mesh(n=n, lnods=np.ascontiguousarray(lnods, dtype=np.int32),
                coord=np.ascontiguousarray(coord, dtype=np.float64),
                velocity=np.ascontiguousarray(vel, dtype=np.float64),
                rho=rho, mu=mu, dt=dt, name=name)


# ---------------------------------------------------------------------------------------------
# The workloads. Sizes and value distributions follow the five configurations of the build; the
# cube meshes stand in for Alya's Sphere/Elbow benchmarks (Table 2 of the paper).
# ---------------------------------------------------------------------------------------------

def config_small() -> Mesh:
    """8^3 cube (3,072 tets, 729 nodes), unjittered, identity numbering, U[-1,1]^3 velocity."""
    return make_mesh(8, velocity="uniform", seed=1, rho=1.0, mu=1e-3, dt=1e-2, name="cube8")


def config_64() -> Mesh:
    """64^3 cube (1,572,864 tets), jittered, random node permutation, elements in generation order."""
    return make_mesh(64, jitter=True, permute=True, velocity="vortex", seed=2,
                     rho=1.0, mu=1e-3, dt=5e-3, name="cube64_perm")


def config_128() -> Mesh:
    """128^3 cube (12,582,912 tets), jittered, permuted then RCM-renumbered, elements sorted."""
    return make_mesh(128, jitter=True, permute=True, rcm=True, sort_elements=True,
                     velocity="vortex", seed=3, rho=1.0, mu=1e-3, dt=5e-3, name="cube128_rcm")


def batch_params(nmesh: int = 64, seed: int = 4, nmin: int = 8, nmax: int = 48):
    """Per-mesh (n, rho, mu, dt, mesh_seed) for the batched workload."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=nmesh)
    rho = rng.uniform(0.5, 2.0, size=nmesh)
    mu = 10.0 ** rng.uniform(-4.0, -2.0, size=nmesh)
    dt = rng.uniform(1e-3, 1e-2, size=nmesh)
    seeds = rng.integers(0, 2 ** 31 - 1, size=nmesh)
    return [dict(n=int(ns[i]), rho=float(rho[i]), mu=float(mu[i]), dt=float(dt[i]),
                 seed=int(seeds[i])) for i in range(nmesh)]


def config_batch(nmesh: int = 64, seed: int = 4, nmin: int = 8, nmax: int = 48):
    """64 jittered, permuted cubes with n ~ U{8..48}; per-mesh rho, mu, dt as drawn."""
    out = []
    for i, p in enumerate(batch_params(nmesh, seed, nmin, nmax)):
        out.append(make_mesh(p["n"], jitter=True, permute=True, velocity="vortex",
                             seed=p["seed"], rho=p["rho"], mu=p["mu"], dt=p["dt"],
                             name=f"batch{i}_n{p['n']}"))
    return out


def served_sizes(nmesh: int = 200, seed: int = 5, tmin: float = 1e3, tmax: float = 5e6):
    """Cube edge n per resident mesh: tet count T log-uniform in [tmin, tmax], n = round((T/6)^(1/3))."""
    rng = np.random.default_rng(seed)
    t = np.exp(rng.uniform(math.log(tmin), math.log(tmax), size=nmesh))
    return [max(1, int(round((x / 6.0) ** (1.0 / 3.0)))) for x in t]


def request_velocity(npoin: int, seed: int) -> np.ndarray:
    """Per-request velocity field: U[-1,1]^3 per node from the request seed."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(npoin, 3))


def config_served(nmesh: int = 200, seed: int = 5, tmin: float = 1e3, tmax: float = 5e6):
    """Resident meshes of the served workload: jittered cubes with the edge counts of served_sizes."""
    out = []
    for i, n in enumerate(served_sizes(nmesh, seed, tmin, tmax)):
        out.append(make_mesh(n, jitter=True, velocity="zero", seed=seed * 100_003 + i, name=f"served{i}_n{n}"))
    return out


def served_requests(nreq: int, nmesh: int, rate: float, seed: int = 6):
    """Open-loop request stream: Poisson arrivals at `rate` per second (times from 0), a uniformly
    chosen resident mesh, rho ~ U[0.5, 2], mu log-uniform in [1e-4, 1e-2], dt ~ U[1e-3, 1e-2] and a
    velocity seed per request."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=nreq))
    mesh = rng.integers(0, nmesh, size=nreq)
    rho = rng.uniform(0.5, 2.0, size=nreq)
    mu = 10.0 ** rng.uniform(-4.0, -2.0, size=nreq)
    dt = rng.uniform(1e-3, 1e-2, size=nreq)
    vseed = rng.integers(0, 2 ** 62, size=nreq)
    return [dict(t=float(t[i]), mesh=int(mesh[i]), rho=float(rho[i]), mu=float(mu[i]), dt=float(dt[i]),
                 vel_seed=int(vseed[i])) for i in range(nreq)]


def shape_quality(lnods: np.ndarray, coord: np.ndarray) -> np.ndarray:
    """|det J| / L^3 per element, L the longest edge: 1/sqrt(2) for the regular tetrahedron's
    |det J| = L^3 / sqrt(2), tending to 0 for slivers, needles, caps and wedges."""
    X = coord[lnods.astype(np.int64)]
    J = X[:, 1:, :] - X[:, :1, :]
    det = np.abs(np.linalg.det(J))
    edges = [np.linalg.norm(X[:, a] - X[:, b], axis=1) for a in range(4) for b in range(a + 1, 4)]
    return det / np.max(edges, axis=0) ** 3


def bad_element_soup(eps=(1e-2, 1e-3, 1e-4, 1e-5, 1e-6), copies: int = 8, seed: int = 7, rho: float = 1.0,
                     mu: float = 1e-3, dt: float = 1e-2) -> Mesh:
    """Disjoint, badly shaped tetrahedra (each with its own four nodes), for every flatness eps:
      sliver  four near-coplanar vertices of a unit square, lifted alternately by +-eps/2;
      needle  a base triangle of side ~eps and an apex at distance 1;
      cap     a unit triangle and an apex eps above a point inside it;
      wedge   two long opposite edges that nearly cross (distance eps).
    Each shape is randomly rotated, scaled by U[0.5, 2] and translated, `copies` times per eps; the
    velocity is U[-1,1]^3 per node. |det J| / L^3 (L the longest edge) reaches ~eps (sliver, cap,
    wedge) and ~eps^2 (needle): 1e-2 down to 1e-12."""
    rng = np.random.default_rng(seed)
    tets = []
    for e in eps:
        shapes = [np.array([[0, 0, e / 2], [1, 0, -e / 2], [1, 1, e / 2], [0, 1, -e / 2]]),
                  np.array([[0, 0, 0], [e, 0, 0], [0.5 * e, 0.87 * e, 0], [0.3 * e, 0.3 * e, 1.0]]),
                  np.array([[0, 0, 0], [1, 0, 0], [0.5, 0.87, 0], [0.45, 0.3, e]]),
                  np.array([[0, 0, 0], [1, 0, 0], [0.5, -0.5, e], [0.5, 0.5, e]])]
        for _ in range(copies):
            for sh in shapes:
                q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
                tets.append((sh @ q.T) * rng.uniform(0.5, 2.0) + rng.uniform(-5.0, 5.0, size=3))
    coord = np.concatenate(tets).astype(np.float64)
    lnods = np.arange(coord.shape[0], dtype=np.int32).reshape(-1, 4)
    velocity = rng.uniform(-1.0, 1.0, size=coord.shape)
    return Mesh(n=0, lnods=lnods, coord=coord, velocity=velocity, rho=rho, mu=mu, dt=dt, name="bad_soup")


def boundary_layer_mesh(n: int = 6, thickness: float = 1e-3, seed: int = 8, rho: float = 1.0, mu: float = 1e-3,
                        dt: float = 1e-2) -> Mesh:
    """A jittered Kuhn cube squashed to [0,1]^2 x [0, thickness] (the flat cells of a boundary layer):
    every element is a connected sliver with |det J| / L^3 ~ thickness / 10; velocity U[-1,1]^3."""
    m = make_mesh(n, jitter=True, velocity="uniform", seed=seed, rho=rho, mu=mu, dt=dt)
    coord = m.coord * np.array([1.0, 1.0, thickness])
    return Mesh(n=n, lnods=m.lnods, coord=coord, velocity=m.velocity, rho=rho, mu=mu, dt=dt,
                name=f"layer{n}_{thickness:g}")


def hub_mesh(level: int = 4, seed: int = 0, rho: float = 1.0, mu: float = 1e-3, dt: float = 1e-2) -> Mesh:
    """A fan of tets around one hub node: the octahedron's faces split `level` times into four,
    pushed to the unit sphere, each surface triangle joined to the centre. The hub's block row has
    one block per surface vertex plus its own (4^level * 4 + 2 + 1 = 1027 at level 4), far beyond
    what a row tile holds; every other row has about eight. Velocity U[-1,1]^3 per node."""
    rng = np.random.default_rng(seed)
    verts = [np.array(v, dtype=np.float64) for v in
             ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))]
    faces = [(0, 2, 4), (2, 1, 4), (1, 3, 4), (3, 0, 4), (2, 0, 5), (1, 2, 5), (3, 1, 5), (0, 3, 5)]
    for _ in range(level):
        mid = {}

        def midpoint(i, j):
            key = (min(i, j), max(i, j))
            if key not in mid:
                p = verts[i] + verts[j]
                verts.append(p / np.linalg.norm(p))
                mid[key] = len(verts) - 1
            return mid[key]
        new = []
        for a, b, c in faces:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            new += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        faces = new
    surf = np.array(verts) * (1.0 + 0.05 * rng.uniform(-1.0, 1.0, size=(len(verts), 1)))
    coord = np.vstack([np.zeros((1, 3)), surf])
    lnods = np.array([(0, a + 1, b + 1, c + 1) for a, b, c in faces], dtype=np.int32)
    velocity = rng.uniform(-1.0, 1.0, size=coord.shape)
    return Mesh(n=level, lnods=lnods, coord=coord, velocity=velocity, rho=rho, mu=mu, dt=dt, name=f"hub{level}")


# ---------------------------------------------------------------------------------------------
# 2-D family: bilinear quadrilaterals. Table 2's two 2-D benchmarks have about one element per
# nodal point (Cylinder 2D: 1,200 elements on 1,280 points; Venturi 2D: 4,200 on 4,371) and the
# paper states four nodes per element, so they are quadrilateral meshes. Structured unit squares
# split into nx x ny quadrilaterals stand in for them.
# Node ids: (i, j) -> i + (nx+1) j before renumbering; element (i, j) has the vertices
# (i, j), (i+1, j), (i+1, j+1), (i, j+1) (counter-clockwise), elements with i fastest.
# Random draws in this order: jitter (npoin x 2), node permutation, velocity noise.
# ---------------------------------------------------------------------------------------------

@dataclasses.dataclass
class QuadMesh:
    """A 2-D quadrilateral mesh with a nodal velocity field and the flow parameters."""
    nx: int
    ny: int
    lnods: np.ndarray         # int32 [nelem][4], counter-clockwise
    coord: np.ndarray         # float64 [npoin][2]
    velocity: np.ndarray      # float64 [npoin][2]
    rho: float = 1.0
    mu: float = 1e-3
    dt: float = 1e-2
    name: str = ""

    @property
    def npoin(self) -> int:
        return int(self.coord.shape[0])

    @property
    def nelem(self) -> int:
        return int(self.lnods.shape[0])


def quad_grid(nx: int, ny: int):
    """Unit-square grid of nx x ny quadrilaterals: lnods int32 [nx*ny][4], coord float64 [npoin][2]."""
    i, j = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    coord = np.stack([i.ravel() / nx, j.ravel() / ny], axis=1).astype(np.float64)
    ei, ej = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ei, ej = ei.ravel(), ej.ravel()
    node = lambda a, b: a + (nx + 1) * b
    lnods = np.stack([node(ei, ej), node(ei + 1, ej), node(ei + 1, ej + 1), node(ei, ej + 1)], axis=1)
    return lnods.astype(np.int32), coord


def vortex_2d(coord: np.ndarray) -> np.ndarray:
    """Smooth 2-D vortex (sin pi x cos pi y, -cos pi x sin pi y) at the given points, [npoin][2]."""
    px, py = math.pi * coord[:, 0], math.pi * coord[:, 1]
    return np.stack([np.sin(px) * np.cos(py), -np.cos(px) * np.sin(py)], axis=1)


def make_quad_mesh(nx: int, ny: int | None = None, *, jitter: bool = False, permute: bool = False,
                   rcm: bool = False, velocity: str = "vortex", seed: int = 0, rho: float = 1.0,
                   mu: float = 1e-3, dt: float = 1e-2, name: str = "") -> QuadMesh:
    """Seeded quadrilateral mesh of the unit square.

    jitter   every node coordinate moves by U[-0.2h, 0.2h] per component (h the cell size in that
             direction): every quadrilateral stays convex and counter-clockwise.
    permute  random relabelling of the nodes; rcm: then reverse Cuthill-McKee renumbering.
    velocity "vortex": vortex_2d plus 0.01 U[-1,1]^2; "uniform": U[-1,1]^2; "zero".
    """
    ny = nx if ny is None else ny
    rng = np.random.default_rng(seed)
    lnods, coord = quad_grid(nx, ny)
    npoin = coord.shape[0]
    if jitter:
        coord = coord + rng.uniform(-0.2, 0.2, size=(npoin, 2)) * np.array([1.0 / nx, 1.0 / ny])
    if permute:
        perm = rng.permutation(npoin)
        new_coord = np.empty_like(coord)
        new_coord[perm] = coord
        coord = new_coord
        lnods = perm[lnods].astype(np.int32)
    if velocity == "vortex":
        vel = vortex_2d(coord) + 0.01 * rng.uniform(-1.0, 1.0, size=(npoin, 2))
    elif velocity == "uniform":
        vel = rng.uniform(-1.0, 1.0, size=(npoin, 2))
    elif velocity == "zero":
        vel = np.zeros((npoin, 2))
    else:
        raise ValueError(f"unknown velocity field {velocity!r}")
    if rcm:
        new_id = node_graph_rcm(lnods, npoin)
        new_coord = np.empty_like(coord)
        new_coord[new_id] = coord
        new_vel = np.empty_like(vel)
        new_vel[new_id] = vel
        coord, vel = new_coord, new_vel
        lnods = new_id[lnods].astype(np.int32)
    return QuadMesh(nx=nx, ny=ny, lnods=np.ascontiguousarray(lnods, dtype=np.int32),
                    coord=np.ascontiguousarray(coord, dtype=np.float64),
                    velocity=np.ascontiguousarray(vel, dtype=np.float64), rho=rho, mu=mu, dt=dt, name=name)


def config_cylinder2d() -> QuadMesh:
    """Stand-in for Cylinder 2D (1,200 elements, 1,280 points): 40 x 30 quadrilaterals, 1,271 points."""
    return make_quad_mesh(40, 30, jitter=True, permute=True, seed=11, name="quad40x30")


def config_venturi2d() -> QuadMesh:
    """Stand-in for Venturi 2D (4,200 elements, 4,371 points): 70 x 60 quadrilaterals, 4,331 points."""
    return make_quad_mesh(70, 60, jitter=True, permute=True, seed=12, name="quad70x60")


def config_quad2048() -> QuadMesh:
    """A 2-D throughput case: 2048 x 2048 quadrilaterals (4,194,304 elements), jittered, permuted then
    RCM-renumbered."""
    return make_quad_mesh(2048, jitter=True, permute=True, rcm=True, seed=13, rho=1.0, mu=1e-3, dt=5e-3,
                          name="quad2048_rcm")
