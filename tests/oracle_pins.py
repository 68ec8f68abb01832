"""Pins that tie the CPU oracle to facts fixed by the mathematics and by the documented reading
of the paper, independent of the oracle's own code.

Each pin takes a loaded oracle library handle and raises AssertionError on mismatch. They are
run against the real oracle (test_oracle_pins.py) and against copies with planted mistakes
(test_oracle_mutants.py), which must each fail at least one pin.

Independent routes used here:
  * hand-derived element entries on reference tetrahedra (tests/golden/element_worked_values.txt);
  * barycentric gradients from a LAPACK inverse of the 4x4 vertex matrix;
  * exact integration of products of linear fields with the barycentric-monomial formula
    int_K l^alpha = 6 V alpha! / (|alpha| + 3)!;
  * the degree-5 Grundmann-Moeller rule on the tetrahedron;
  * invariants of the weak form: rigid rotations in the kernel of the symmetric-gradient viscous
    and grad-div operators, constant-field row sums, the Galerkin skew pair (q, div u) / -(p, div v),
    symmetry without convection, the textbook P1 mass/stiffness when mu = 0 and a = 0 (the Kuhn
    cube's P1 Laplacian is the 7-point stencil times h), the discrete divergence theorem at
    interior nodes, and invariance under renumbering, rotation and translation.
"""
from __future__ import annotations

import itertools
import math
import os

import numpy as np

import oracle
from paper_2111_05651_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "element_worked_values.txt")
REF_TET = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])


# ------------------------------------------------------------------------------------------ #
# helpers (independent of the oracle)
# ------------------------------------------------------------------------------------------ #

def _safe_eval(expr: str) -> float:
    allowed = set("0123456789.+-*/() e")
    if not set(expr) <= allowed:
        raise ValueError(f"bad expression {expr!r}")
    return float(eval(expr, {"__builtins__": {}}, {}))  # numbers and operators only


def load_golden(path: str = GOLDEN):
    cases, entries = {}, []
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "case":
            kv = dict(t.split("=") for t in tok[2:])
            cases[tok[1]] = dict(scale=float(kv["scale"]), u=np.array([float(x) for x in kv["u"].split(",")]),
                                 rho=float(kv["rho"]), mu=float(kv["mu"]), dt=float(kv["dt"]))
        elif tok[1] == "A":
            entries.append((tok[0], "A", int(tok[2]), int(tok[3]), _safe_eval(" ".join(tok[4:]))))
        else:
            entries.append((tok[0], "b", int(tok[2]), None, _safe_eval(" ".join(tok[3:]))))
    return cases, entries


def bary_grad(X):
    """grad lambda_a [4][3] and volume, from the inverse of [[X_a, 1]]."""
    T = np.hstack([X, np.ones((4, 1))])
    Ti = np.linalg.inv(T)
    return Ti[:3, :].T.copy(), abs(np.linalg.det(T)) / 6.0


def random_tet(rng, scale=1.0, quality=0.3):
    while True:
        X = rng.normal(size=(4, 3)) * scale
        _, V = bary_grad(X)
        edges = [np.linalg.norm(X[i] - X[j]) for i in range(4) for j in range(i + 1, 4)]
        if V > quality * max(edges) ** 3 / (6 * math.sqrt(2)):
            return X


def monomial_integral(alpha, V):
    """int_K prod_k lambda_k^alpha_k = 6 V prod(alpha_k!) / (|alpha| + 3)!"""
    return 6.0 * V * np.prod([math.factorial(a) for a in alpha]) / math.factorial(sum(alpha) + 3)


def exact_product_integral(fields, V):
    """Exact integral over K of a product of linear fields given by their 4 nodal values."""
    total = 0.0
    for ks in itertools.product(range(4), repeat=len(fields)):
        alpha = [0, 0, 0, 0]
        coef = 1.0
        for f, k in zip(fields, ks):
            alpha[k] += 1
            coef *= f[k]
        if coef != 0.0:
            total += coef * monomial_integral(alpha, V)
    return total


def grundmann_moeller(s: int, n: int = 3):
    """Degree 2s+1 Grundmann-Moeller rule on the n-simplex of volume 1/n!:
    list of (barycentric point, weight)."""
    d = 2 * s + 1
    rule = []
    for i in range(s + 1):
        w = (-1) ** i * 2.0 ** (-2 * s) * (d + n - 2 * i) ** d / (math.factorial(i) * math.factorial(d + n - i))
        m = s - i
        for beta in itertools.product(range(m + 1), repeat=n + 1):
            if sum(beta) != m:
                continue
            rule.append((np.array([(2 * b + 1) / (d + n - 2 * i) for b in beta]), w))
    return rule


def gm_integral(f_of_lambda, V, s=2):
    rule = grundmann_moeller(s)
    return 6.0 * V * sum(w * f_of_lambda(p) for p, w in rule)


def _close(a, b, rtol, atol, what):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    if not np.allclose(a, b, rtol=rtol, atol=atol):
        err = np.max(np.abs(a - b))
        raise AssertionError(f"{what}: max |diff| {err:.3e}\n{a}\n{b}")


# ------------------------------------------------------------------------------------------ #
# element-level pins
# ------------------------------------------------------------------------------------------ #

def pin_golden(lib):
    cases, entries = load_golden()
    cache = {}
    for name, kind, r, c, want in entries:
        if name not in cache:
            cs = cases[name]
            X = REF_TET * cs["scale"]
            U = np.tile(cs["u"], (4, 1))
            cache[name] = oracle.element(X, U, cs["rho"], cs["mu"], cs["dt"], lib=lib)
        A, b = cache[name]
        got = A[r, c] if kind == "A" else b[r]
        if not math.isclose(got, want, rel_tol=1e-13, abs_tol=1e-15):
            raise AssertionError(f"golden {name} {kind}[{r}]{'' if c is None else f'[{c}]'}: "
                                 f"oracle {got!r} vs hand-derived {want!r}")


def pin_geometry(lib, ntet=20, seed=11):
    rng = np.random.default_rng(seed)
    for _ in range(ntet):
        X = random_tet(rng, scale=rng.uniform(0.01, 10.0))
        I = oracle.element_integrals(X, np.zeros((4, 3)), 1.0, 1e-3, 1e-2, lib=lib)
        G, V = bary_grad(X)
        _close(I["gpcar"], G, 1e-11, 1e-12 * np.abs(G).max(), "grad N vs LAPACK barycentric gradients")
        _close(I["V"], V, 1e-13, 0.0, "volume")
        _close(I["h"], (6 * V) ** (1 / 3), 1e-14, 0.0, "h = (6V)^(1/3)")
        _close(I["gpcar"].sum(axis=0), np.zeros(3), 0, 1e-12 * np.abs(G).max(), "sum_a grad N_a = 0")
        _close(X.T @ I["gpcar"], np.eye(3), 0, 1e-12, "sum_a X_a grad N_a^T = I")


def _integrals_exact(X, U):
    G, V = bary_grad(X)
    ag = U @ G.T            # ag[k][b] = U_k . G_b : nodal values of a.grad N_b
    N = np.eye(4)
    out = dict(mass=np.zeros((4, 4)), conv=np.zeros((4, 4)), aa=np.zeros((4, 4)), iag=np.zeros(4),
               un=np.zeros((4, 3)), au=np.zeros((4, 3)))
    for a in range(4):
        out["iag"][a] = exact_product_integral([ag[:, a]], V)
        for b in range(4):
            out["mass"][a, b] = exact_product_integral([N[a], N[b]], V)
            out["conv"][a, b] = exact_product_integral([N[a], ag[:, b]], V)
            out["aa"][a, b] = exact_product_integral([ag[:, a], ag[:, b]], V)
        for c in range(3):
            out["un"][a, c] = exact_product_integral([U[:, c], N[a]], V)
            out["au"][a, c] = exact_product_integral([ag[:, a], U[:, c]], V)
    return out, V


def pin_integrals_exact(lib, ntet=12, seed=12):
    rng = np.random.default_rng(seed)
    for _ in range(ntet):
        X = random_tet(rng, scale=rng.uniform(0.1, 3.0))
        U = rng.uniform(-2, 2, size=(4, 3))
        got = oracle.element_integrals(X, U, 1.0, 1e-3, 1e-2, lib=lib)
        want, V = _integrals_exact(X, U)
        _close(want["mass"], V / 20 * (1 + np.eye(4)), 1e-14, 0, "textbook P1 mass (self-check)")
        for k in want:
            scale = np.abs(want[k]).max() + 1e-300
            _close(got[k], want[k], 1e-12, 1e-13 * scale, f"exact integral {k}")


def pin_integrals_gm(lib, ntet=6, seed=13):
    rule = grundmann_moeller(2)
    assert abs(sum(w for _, w in rule) - 1 / 6) < 1e-15
    rng = np.random.default_rng(seed)
    for _ in range(ntet):
        X = random_tet(rng)
        U = rng.uniform(-2, 2, size=(4, 3))
        G, V = bary_grad(X)
        got = oracle.element_integrals(X, U, 1.0, 1e-3, 1e-2, lib=lib)
        u = lambda lam: lam @ U                      # velocity at barycentric point
        for a in range(4):
            for b in range(4):
                _close(got["conv"][a, b], gm_integral(lambda l: l[a] * (u(l) @ G[b]), V), 1e-12, 1e-13, "GM conv")
                _close(got["aa"][a, b], gm_integral(lambda l: (u(l) @ G[a]) * (u(l) @ G[b]), V), 1e-12, 1e-13, "GM aa")
                _close(got["mass"][a, b], gm_integral(lambda l: l[a] * l[b], V), 1e-12, 1e-14, "GM mass")
            for c in range(3):
                _close(got["au"][a, c], gm_integral(lambda l: (u(l) @ G[a]) * u(l)[c], V), 1e-12, 1e-13, "GM au")
                _close(got["un"][a, c], gm_integral(lambda l: u(l)[c] * l[a], V), 1e-12, 1e-13, "GM un")


def _blocks(A):
    idx_u = [4 * a + c for a in range(4) for c in range(3)]
    idx_p = [4 * a + 3 for a in range(4)]
    return (A[np.ix_(idx_u, idx_u)], A[np.ix_(idx_u, idx_p)], A[np.ix_(idx_p, idx_u)], A[np.ix_(idx_p, idx_p)])


def pin_element_invariants(lib, ntet=10, seed=14):
    rng = np.random.default_rng(seed)
    for _ in range(ntet):
        X = random_tet(rng)
        G, V = bary_grad(X)
        U = rng.uniform(-1, 1, size=(4, 3))
        rho, mu, dt = rng.uniform(0.5, 2), 10 ** rng.uniform(-4, -1), rng.uniform(1e-3, 1e-1)
        A, b = oracle.element(X, U, rho, mu, dt, lib=lib)
        Auu, Aup, Apu, App = _blocks(A)
        s = np.abs(A).max()
        abar = U.mean(axis=0)
        # tau1 from the worked form is pinned by the golden file; here only consistency:
        I = oracle.element_integrals(X, U, rho, mu, dt, lib=lib)
        t1 = I["tau1"]
        # constant trial field: sum over columns b of each block row
        for a in range(4):
            for c in range(3):
                for cp in range(3):
                    rs = sum(Auu[3 * a + c, 3 * bb + cp] for bb in range(4))
                    want = (rho / dt * V / 4 + t1 * rho * rho / dt * V * (abar @ G[a])) if c == cp else 0.0
                    _close(rs, want, 1e-10, 1e-12 * s, "Auu constant-field row sum")
                _close(Aup[3 * a + c].sum(), -V * G[a, c], 1e-10, 1e-12 * s, "Aup row sum = -V G_a")
            for cp in range(3):
                rs = sum(Apu[a, 3 * bb + cp] for bb in range(4))
                _close(rs, t1 * rho / dt * V * G[a, cp], 1e-10, 1e-12 * s, "Apu constant-field row sum")
            _close(App[a].sum(), 0.0, 0, 1e-12 * s, "App row sum")
        # Galerkin skew pair: Apu + Aup^T = PSPG + SUPG pressure parts
        for a in range(4):
            for bb in range(4):
                for cp in range(3):
                    want = t1 * G[a, cp] * (2 * rho * V * (abar @ G[bb]) + rho / dt * V / 4)
                    _close(Apu[a, 3 * bb + cp] + Aup[3 * bb + cp, a], want, 1e-10, 1e-12 * s, "Apu + Aup^T")
        # no convection: Auu and App symmetric
        A0, _ = oracle.element(X, np.zeros((4, 3)), rho, mu, dt, lib=lib)
        Auu0, _, _, App0 = _blocks(A0)
        _close(Auu0, Auu0.T, 0, 1e-13 * np.abs(Auu0).max(), "Auu symmetric when a = 0")
        _close(App0, App0.T, 0, 1e-13 * np.abs(App0).max(), "App symmetric when a = 0")
        # mu = 0, a = 0: textbook P1 consistent mass and stiffness (tau1 = dt/rho, tau2 = 0)
        A1, b1 = oracle.element(X, np.zeros((4, 3)), rho, 0.0, dt, lib=lib)
        Auu1, Aup1, Apu1, App1 = _blocks(A1)
        M = V / 20 * (1 + np.eye(4))
        _close(Auu1, np.kron(rho / dt * M, np.eye(3)), 1e-12, 1e-14, "mu=0,a=0: (rho/dt) mass x I3")
        _close(App1, dt / rho * V * G @ G.T, 1e-12, 1e-16, "mu=0,a=0: (dt/rho) P1 stiffness")
        _close(Aup1, -V / 4 * np.repeat(G.reshape(12, 1), 4, axis=1), 1e-12, 1e-16, "mu=0,a=0: -(p, div v)")
        want_pu = np.zeros((4, 12))
        for a in range(4):
            for bb in range(4):
                want_pu[a, 3 * bb:3 * bb + 3] = V / 4 * (G[bb] + G[a])
        _close(Apu1, want_pu, 1e-12, 1e-16, "mu=0,a=0: (q, div u) + PSPG mass")
        _close(b1, np.zeros(16), 0, 0, "zero velocity: zero RHS")


def pin_viscous_kernel(lib, ntet=8, seed=15):
    """With rho = 0 only the viscous, grad-div and PSPG-Laplacian terms survive: rigid rotations
    are in the kernel of the symmetric-gradient and grad-div operators; a pure dilatation
    u = x gives 2 mu V G_a + 3 tau2 V G_a (tau2 = mu when rho = 0)."""
    rng = np.random.default_rng(seed)
    for _ in range(ntet):
        X = random_tet(rng)
        G, V = bary_grad(X)
        U = rng.uniform(-1, 1, size=(4, 3))
        mu = 10 ** rng.uniform(-3, 0)
        A, _ = oracle.element(X, U, 0.0, mu, 1e-2, lib=lib)
        Auu, Aup, Apu, App = _blocks(A)
        w = rng.normal(size=3)
        urot = np.cross(w, X).reshape(12)
        s = np.abs(Auu).max() * np.abs(urot).max()
        _close(Auu @ urot, np.zeros(12), 0, 1e-12 * s, "rigid rotation in kernel of viscous + grad-div")
        _close(Apu @ urot, np.zeros(4), 0, 1e-12 * s, "div of a rigid rotation")
        udil = X.reshape(12)
        _close(Auu @ udil, (5 * mu * V * G).reshape(12), 1e-10, 1e-13 * s, "dilatation: (2 mu + 3 tau2) V G_a")


def pin_rotation_translation(lib, ntet=6, seed=16):
    rng = np.random.default_rng(seed)
    for _ in range(ntet):
        X = random_tet(rng)
        U = rng.uniform(-1, 1, size=(4, 3))
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        if np.linalg.det(Q) < 0:
            Q[:, 0] = -Q[:, 0]
        t = rng.normal(size=3) * 5
        A, b = oracle.element(X, U, 1.0, 1e-3, 1e-2, lib=lib)
        Ar, br = oracle.element(X @ Q.T + t, U @ Q.T, 1.0, 1e-3, 1e-2, lib=lib)
        R = np.zeros((16, 16))
        for a in range(4):
            R[4 * a:4 * a + 3, 4 * a:4 * a + 3] = Q
            R[4 * a + 3, 4 * a + 3] = 1.0
        s = np.abs(A).max()
        _close(Ar, R @ A @ R.T, 0, 1e-12 * s, "rotation covariance of the element matrix")
        _close(br, R @ b, 0, 1e-12 * np.abs(b).max(), "rotation covariance of the RHS")


# ------------------------------------------------------------------------------------------ #
# mesh-level pins
# ------------------------------------------------------------------------------------------ #

def brute_pattern(npoin, lnods):
    rows = [set() for _ in range(npoin)]
    for e in lnods:
        for a in e:
            rows[a].update(int(x) for x in e)
    bptr = np.zeros(npoin + 1, dtype=np.int64)
    bcol = []
    for i in range(npoin):
        cols = sorted(rows[i])
        bcol.extend(cols)
        bptr[i + 1] = bptr[i] + len(cols)
    bcol = np.array(bcol, dtype=np.int32)
    emap = np.zeros((len(lnods), 4, 4), dtype=np.int32)
    for e, nodes in enumerate(lnods):
        for a in range(4):
            lo, hi = bptr[nodes[a]], bptr[nodes[a] + 1]
            for bb in range(4):
                emap[e, a, bb] = lo + int(np.searchsorted(bcol[lo:hi], nodes[bb]))
    return bptr, bcol, emap


def pin_pattern(lib):
    for n in (1, 2, 3):
        m = inputs.make_mesh(n, jitter=True, permute=True, seed=n)
        bptr, bcol, emap = oracle.pattern(m.npoin, m.lnods, lib=lib)
        wb, wc, we = brute_pattern(m.npoin, m.lnods)
        assert np.array_equal(bptr, wb) and np.array_equal(bcol, wc) and np.array_equal(emap, we), \
            f"pattern differs from the set-based brute force at n={n}"
        assert int(bptr[-1]) == inputs.cube_counts(n)[3], "nnzb != npoin + 2 * edges"


def dense(npoin, bptr, bcol, values):
    D = np.zeros((4 * npoin, 4 * npoin))
    for i in range(npoin):
        for k in range(bptr[i], bptr[i + 1]):
            j = bcol[k]
            D[4 * i:4 * i + 4, 4 * j:4 * j + 4] = values[k]
    return D


def pin_kuhn_stencil(lib, n=4):
    """mu = 0, a = 0 on the unjittered Kuhn cube: App = (dt/rho) P1 stiffness, whose interior rows
    are the 7-point Laplacian h (6, -1 x 6) with exact zeros at the other Kuhn neighbours; the
    velocity diagonal sums to (rho/dt) times the cube volume."""
    m = inputs.make_mesh(n, velocity="zero", seed=0)
    rho, dt, h = 1.5, 2e-2, 1.0 / n
    pat = oracle.pattern(m.npoin, m.lnods, lib=lib)
    values, rhs = oracle.assemble(m, pat, lib=lib, rho=rho, mu=0.0, dt=dt)
    bptr, bcol, _ = pat
    M = n + 1
    for k in range(1, n):
        for j in range(1, n):
            for i in range(1, n):
                node = i + M * (j + M * k)
                for q in range(bptr[node], bptr[node + 1]):
                    col = bcol[q]
                    ci, cj, ck = col % M, (col // M) % M, col // (M * M)
                    off = abs(ci - i) + abs(cj - j) + abs(ck - k)
                    want = 6 * h if off == 0 else (-h if off == 1 else 0.0)
                    got = values[q][3, 3] * rho / dt
                    if abs(got - want) > 1e-13:
                        raise AssertionError(f"stencil at node {node} col {col}: {got} vs {want}")
    for c in range(3):
        tot = values[:, c, c].sum()
        _close(tot, rho / dt, 1e-12, 0, "sum of the velocity mass = (rho/dt) * volume")


def pin_divergence_theorem(lib, n=4):
    """Sum over the columns of an interior row of the velocity-pressure coupling is
    -int grad N_i = 0 (the SUPG part vanishes because sum_b grad N_b = 0)."""
    m = inputs.make_mesh(n, jitter=True, permute=True, velocity="uniform", seed=21)
    pat = oracle.pattern(m.npoin, m.lnods, lib=lib)
    values, _ = oracle.assemble(m, pat, lib=lib)
    bptr = pat[0]
    eps = 1e-9
    interior = np.all((m.coord > 0.2 / n + eps) & (m.coord < 1 - 0.2 / n - eps), axis=1)
    # jitter moves a node by at most 0.2 h, so grid-interior nodes are exactly those kept here
    assert interior.sum() == (n - 1) ** 3
    s = np.abs(values[:, :3, 3]).max()
    for i in np.nonzero(interior)[0]:
        rs = values[bptr[i]:bptr[i + 1], :3, 3].sum(axis=0)
        _close(rs, np.zeros(3), 0, 1e-12 * s, f"interior Aup row sum at node {i}")


def pin_renumbering(lib, n=3, seed=22):
    m = inputs.make_mesh(n, jitter=True, velocity="uniform", seed=seed)
    pat = oracle.pattern(m.npoin, m.lnods, lib=lib)
    v0, r0 = oracle.assemble(m, pat, lib=lib)
    D0 = dense(m.npoin, pat[0], pat[1], v0)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(m.npoin)                  # new id of old node
    eperm = rng.permutation(m.nelem)
    ln = perm[m.lnods][eperm]
    for e in range(ln.shape[0]):
        ln[e] = ln[e][rng.permutation(4)]            # local vertex order (orientation may flip)
    m2 = inputs.Mesh(n=n, lnods=ln.astype(np.int32), coord=np.empty_like(m.coord),
                     velocity=np.empty_like(m.velocity), rho=m.rho, mu=m.mu, dt=m.dt)
    m2.coord[perm] = m.coord
    m2.velocity[perm] = m.velocity
    pat2 = oracle.pattern(m2.npoin, m2.lnods, lib=lib)
    v2, r2 = oracle.assemble(m2, pat2, lib=lib)
    D2 = dense(m2.npoin, pat2[0], pat2[1], v2)
    P = np.zeros((4 * m.npoin,), dtype=np.int64)     # dof map old -> new
    for i in range(m.npoin):
        P[4 * i:4 * i + 4] = 4 * perm[i] + np.arange(4)
    s = np.abs(D0).max()
    _close(D2[np.ix_(P, P)], D0, 0, 1e-12 * s, "renumbering invariance of the assembled matrix")
    _close(r2[perm], r0, 0, 1e-12 * np.abs(r0).max(), "renumbering invariance of the RHS")


def pin_residual_uniform_flow(lib, n=3, seed=23):
    """Explicit residual: a uniform velocity field leaves no residual at any node. With U_b = u for
    every node, sum_b grad N_b = 0 removes the convective, viscous, grad-div and SUPG-convective
    parts of A_uu u, and what is left, (rho/dt) V/4 u + tau1 rho (rho/dt) V (u . grad N_a) u, is the
    element RHS term by term."""
    m = inputs.make_mesh(n, jitter=True, permute=True, seed=seed, rho=1.3, mu=2e-3, dt=4e-3)
    for ubar in (np.array([0.7, -0.4, 0.25]), np.array([0.0, 0.0, 2.0])):
        U = np.tile(ubar, (m.npoin, 1))
        rhsid, _, _ = oracle.residual(m, lib=lib, velocity=U)
        _, rhs = oracle.assemble(m, lib=lib, velocity=U)
        _close(rhsid, np.zeros_like(rhsid), 0, 1e-12 * np.abs(rhs[:, :3]).max(), "uniform-flow residual")


def pin_residual_csr_route(lib, n=3, seed=24):
    """Explicit residual against a second route: the assembled block-CSR matrix applied to the
    nodal velocities (pressure zero), subtracted from the assembled RHS."""
    m = inputs.make_mesh(n, jitter=True, permute=True, velocity="uniform", seed=seed)
    pat = oracle.pattern(m.npoin, m.lnods, lib=lib)
    values, rhs = oracle.assemble(m, pat, lib=lib)
    bptr, bcol, _ = pat
    rows = np.repeat(np.arange(m.npoin), np.diff(bptr))
    av = np.zeros((m.npoin, 3))
    np.add.at(av, rows, np.einsum("kij,kj->ki", values[:, :3, :3], m.velocity[bcol]))
    want = rhs[:, :3] - av
    rhsid, _, _ = oracle.residual(m, lib=lib)
    _close(rhsid, want, 0, 1e-12 * np.abs(want).max(), "residual vs rhs - A u")


def pin_residual_lumped(lib, n=3, seed=25):
    """Lumped masses: mass_rho at node i is rho sum_{e ni i} V_e / 4 with V_e = |det| / 6 from NumPy;
    their total is rho times the mesh volume; dt_rho at node i is sum_{e ni i} tau1_e V_e / 4 with
    tau1_e and V_e of the (pinned) element routine."""
    m = inputs.make_mesh(n, jitter=True, permute=True, velocity="vortex", seed=seed, rho=0.8, mu=5e-3, dt=2e-3)
    _, dt_rho, mass_rho = oracle.residual(m, lib=lib)
    X = m.coord[m.lnods]
    vol = np.abs(np.linalg.det(X[:, 1:, :] - X[:, :1, :])) / 6.0
    want = np.zeros(m.npoin)
    np.add.at(want, m.lnods.ravel(), np.repeat(m.rho * vol / 4.0, 4))
    _close(mass_rho, want, 0, 1e-14 * want.max(), "rho-weighted lumped mass")
    _close(np.array([mass_rho.sum()]), np.array([m.rho * vol.sum()]), 0, 1e-13, "total rho-weighted mass")
    w = np.zeros(m.npoin)
    for e in range(m.nelem):
        it = oracle.element_integrals(m.coord[m.lnods[e]], m.velocity[m.lnods[e]], m.rho, m.mu, m.dt, lib=lib)
        w[m.lnods[e]] += it["tau1"] * it["V"] / 4.0
    _close(dt_rho, w, 0, 1e-14 * w.max(), "tau-weighted lumped mass")


def pin_assemble_rows(lib):
    """The row-by-row route (used to check meshes too large to assemble whole) against the whole-mesh
    route: for every row of small jittered / permuted / RCM meshes, a mesh with nodes in no element
    and a hub node in 128 elements, and for a sample of the rows of a larger one, the rebuilt
    column set equals the row of the set-based pattern and the summed blocks and RHS are bit-for-bit
    those of the whole-mesh assembly (same element values, same element order)."""
    meshes = [inputs.make_mesh(3, jitter=True, permute=True, velocity="vortex", seed=41),
              inputs.make_mesh(4, jitter=True, permute=True, rcm=True, sort_elements=True, seed=42),
              inputs.hub_mesh(2, seed=43)]
    iso = inputs.make_mesh(2, jitter=True, seed=44)
    ln = iso.lnods.copy()
    ln[ln >= 5] += 2   # nodes 5 and 6 in no element
    coord = np.vstack([iso.coord[:5], [[3.0, 3, 3], [4.0, 4, 4]], iso.coord[5:]])
    vel = np.vstack([iso.velocity[:5], [[1.0, 2, 3], [4.0, 5, 6]], iso.velocity[5:]])
    meshes.append(inputs.Mesh(n=2, lnods=ln, coord=coord, velocity=vel, rho=iso.rho, mu=iso.mu, dt=iso.dt))
    big = inputs.make_mesh(8, jitter=True, permute=True, velocity="vortex", seed=45)
    rng = np.random.default_rng(46)
    cases = [(m, np.arange(m.npoin)) for m in meshes]
    cases.append((big, np.unique(np.concatenate([rng.choice(big.npoin, 60, replace=False), [0, big.npoin - 1]]))))
    for m, rows in cases:
        bptr, bcol, emap = oracle.pattern(m.npoin, m.lnods, lib=lib)
        values, rhs = oracle.assemble(m, (bptr, bcol, emap), lib=lib)
        maxdeg = int(np.diff(bptr).max())
        cols, deg, vals, rr = oracle.assemble_rows(m, rows, maxdeg=maxdeg, lib=lib)
        for s, i in enumerate(rows):
            lo, hi = bptr[i], bptr[i + 1]
            assert deg[s] == hi - lo, f"row {i}: {deg[s]} columns, pattern has {hi - lo}"
            assert np.array_equal(cols[s, :deg[s]], bcol[lo:hi]), f"row {i} columns"
            assert np.all(cols[s, deg[s]:] == -1)
            assert np.array_equal(vals[s, :deg[s]], values[lo:hi]), f"row {i} blocks"
            assert not np.any(vals[s, deg[s]:]), f"row {i} padding"
            assert np.array_equal(rr[s], rhs[i]), f"row {i} RHS"


ALL_PINS = [pin_golden, pin_geometry, pin_integrals_exact, pin_integrals_gm, pin_element_invariants,
            pin_viscous_kernel, pin_rotation_translation, pin_pattern, pin_kuhn_stencil,
            pin_divergence_theorem, pin_renumbering, pin_residual_uniform_flow, pin_residual_csr_route,
            pin_residual_lumped, pin_assemble_rows]
