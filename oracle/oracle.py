"""ctypes marshalling for the C oracle (TEST INFRASTRUCTURE ONLY; see nsa_oracle.c)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nsa_oracle.c")
Q1_SRC = os.path.join(HERE, "nsa_oracle_q1.c")  # the 2-D quadrilateral family
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11"]

OR_OK, OR_EINVAL, OR_ERANGE, OR_EDEGENERATE, OR_ENOMEM = 0, -1, -2, -3, -4

_lib = None


LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def build(src: str = SRC, out: str = LIB, q1_src: str = Q1_SRC) -> str:
    """Compile the oracle with gcc (always rebuilds): the serial build the tests pin, and the OpenMP
    build of the same sources that only times the CPU baseline."""
    tmp = out + ".tmp"
    subprocess.run(["gcc", *CFLAGS, "-Wno-unknown-pragmas", "-o", tmp, src, q1_src, "-lm"], check=True)
    os.replace(tmp, out)
    if out == LIB:
        build_flops()
        tmp = LIB_OMP + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-fopenmp", "-o", tmp, src, q1_src, "-lm"], check=True)
        os.replace(tmp, LIB_OMP)
    return out


LIB_FLOPS = os.path.join(HERE, "liboracle_flops.so")
FLOPS_SRC = os.path.join(HERE, "flops.cpp")


def build_flops() -> str:
    """The operation-counting build of the same source (flops.cpp)."""
    tmp = LIB_FLOPS + ".tmp"
    subprocess.run(["g++", "-O1", "-ffp-contract=off", "-std=c++17", "-fpermissive", "-w", "-fPIC", "-shared", "-o", tmp,
                    FLOPS_SRC],
                   check=True)
    os.replace(tmp, LIB_FLOPS)
    return LIB_FLOPS


def flops(mesh, kind="residual", pat=None):
    """Floating-point operations of the oracle's routine over the mesh (kind "residual": the
    explicit-residual outputs; "assemble": matrix and RHS), counted by the instrumented build, and
    the outputs it computed: (count, outputs)."""
    if not os.path.exists(LIB_FLOPS):
        build_flops()
    lib = C.CDLL(LIB_FLOPS)
    d, i64, P = C.c_double, C.c_int64, C.c_void_p
    ln = np.ascontiguousarray(mesh.lnods, dtype=np.int32)
    co, ve = _f64(mesh.coord), _f64(mesh.velocity)
    st = C.c_int(0)
    if kind == "residual":
        f = lib.oracle_flops_residual
        f.argtypes = [i64, i64, P, P, P, d, d, d, P, P, P, P]
        f.restype = C.c_longlong
        out = (np.zeros((mesh.npoin, 3)), np.zeros(mesh.npoin), np.zeros(mesh.npoin))
        n = f(mesh.npoin, mesh.nelem, _p(ln), _p(co), _p(ve), mesh.rho, mesh.mu, mesh.dt, *[_p(o) for o in out],
              C.byref(st))
    else:
        if pat is None:
            pat = pattern(mesh.npoin, mesh.lnods)
        bptr, _, emap = pat
        f = lib.oracle_flops_assemble
        f.argtypes = [i64, i64, P, P, P, d, d, d, i64, P, P, P, P]
        f.restype = C.c_longlong
        out = (np.zeros((int(bptr[-1]), 4, 4)), np.zeros((mesh.npoin, 4)))
        em = np.ascontiguousarray(emap, dtype=np.int32)
        n = f(mesh.npoin, mesh.nelem, _p(ln), _p(co), _p(ve), mesh.rho, mesh.mu, mesh.dt, int(bptr[-1]), _p(em),
              *[_p(o) for o in out], C.byref(st))
    if st.value != OR_OK:
        raise ValueError(f"oracle flops status {st.value}")
    return int(n), out


def load_omp():
    """The OpenMP build (all host threads; for timing the CPU baseline, never for parity)."""
    if not os.path.exists(LIB_OMP):
        build()
    lib = _bind(C.CDLL(LIB_OMP))
    return lib


def _bind(lib):
    d, i32, i64 = C.c_double, C.c_int32, C.c_int64
    P = C.c_void_p
    lib.oracle_element.argtypes = [P, P, d, d, d, P, P]
    lib.oracle_element.restype = C.c_int
    lib.oracle_element_integrals.argtypes = [P, P, d, d, d, P, P, P, P, P, P, P, P]
    lib.oracle_element_integrals.restype = C.c_int
    lib.oracle_validate.argtypes = [i64, i64, P, P, P]
    lib.oracle_validate.restype = C.c_int
    lib.oracle_pattern.argtypes = [i64, i64, P, P, P, P]
    lib.oracle_pattern.restype = i64
    lib.oracle_assemble.argtypes = [i64, i64, P, P, P, d, d, d, i64, P, P, P]
    lib.oracle_assemble.restype = C.c_int
    lib.oracle_assemble_rows.argtypes = [i64, i64, P, P, P, d, d, d, i64, P, i32, P, P, P, P]
    lib.oracle_assemble_rows.restype = C.c_int
    lib.oracle_residual.argtypes = [i64, i64, P, P, P, d, d, d, P, P, P]
    lib.oracle_residual.restype = C.c_int
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = C.c_int
    lib.oracle_q1_element_rule.argtypes = [P, P, d, d, d, C.c_int, P, P]
    lib.oracle_q1_element_rule.restype = C.c_int
    lib.oracle_q1_element.argtypes = [P, P, d, d, d, P, P]
    lib.oracle_q1_element.restype = C.c_int
    lib.oracle_q1_element_integrals.argtypes = [P, P, d, d, d, P, P, P, P, P]
    lib.oracle_q1_element_integrals.restype = C.c_int
    lib.oracle_q1_validate.argtypes = [i64, i64, P, P, P]
    lib.oracle_q1_validate.restype = C.c_int
    lib.oracle_q1_assemble.argtypes = [i64, i64, P, P, P, d, d, d, i64, P, P, P]
    lib.oracle_q1_assemble.restype = C.c_int
    return lib


def load(path: str | None = None):
    """Load the oracle library (building it first if it is not there)."""
    global _lib
    if path is not None:
        return _bind(C.CDLL(path))
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _bind(C.CDLL(LIB))
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def element(X, U, rho, mu, dt, lib=None):
    """Element matrix A [16][16] (rows test (a,c), cols trial (b,c'), dof 4a+c) and RHS [16]."""
    lib = lib or load()
    X, U = _f64(X, (4, 3)), _f64(U, (4, 3))
    A = np.zeros((16, 16))
    b = np.zeros(16)
    st = lib.oracle_element(_p(X), _p(U), rho, mu, dt, _p(A), _p(b))
    if st != OR_OK:
        raise ValueError(f"oracle_element status {st}")
    return A, b


def element_integrals(X, U, rho, mu, dt, lib=None):
    """Gauss-rule integrals and element scalars (see oracle_element_integrals)."""
    lib = lib or load()
    X, U = _f64(X, (4, 3)), _f64(U, (4, 3))
    out = dict(scal=np.zeros(4), gpcar=np.zeros((4, 3)), mass=np.zeros((4, 4)), conv=np.zeros((4, 4)),
               aa=np.zeros((4, 4)), iag=np.zeros(4), un=np.zeros((4, 3)), au=np.zeros((4, 3)))
    st = lib.oracle_element_integrals(_p(X), _p(U), rho, mu, dt, *[_p(out[k]) for k in
                                      ("scal", "gpcar", "mass", "conv", "aa", "iag", "un", "au")])
    if st != OR_OK:
        raise ValueError(f"oracle_element_integrals status {st}")
    s = out.pop("scal")
    out.update(V=s[0], h=s[1], tau1=s[2], tau2=s[3])
    return out


def validate(npoin, lnods, coord, lib=None):
    """(status, first bad element or -1)."""
    lib = lib or load()
    ln = np.ascontiguousarray(lnods, dtype=np.int32)
    co = _f64(coord)
    bad = np.zeros(1, dtype=np.int64)
    st = lib.oracle_validate(int(npoin), int(ln.shape[0]), _p(ln), _p(co), _p(bad))
    return st, int(bad[0])


def pattern(npoin, lnods, lib=None):
    """Block-CSR pattern of the node graph: (bptr int64 [npoin+1], bcol int32 [nnzb],
    emap int32 [nelem][4][4])."""
    lib = lib or load()
    ln = np.ascontiguousarray(lnods, dtype=np.int32)
    nelem = ln.shape[0]
    bptr = np.zeros(npoin + 1, dtype=np.int64)
    bcol = np.zeros(max(16 * nelem, 1), dtype=np.int32)
    emap = np.zeros((nelem, 4, 4), dtype=np.int32)
    nnzb = lib.oracle_pattern(int(npoin), int(nelem), _p(ln), _p(bptr), _p(bcol), _p(emap))
    if nnzb < 0:
        raise ValueError(f"oracle_pattern status {nnzb}")
    return bptr, bcol[:nnzb].copy(), emap


def assemble(mesh, pat=None, lib=None, rho=None, mu=None, dt=None, velocity=None):
    """Global BSR values [nnzb][4][4] and RHS [npoin][4] for a Mesh (inputs.Mesh)."""
    lib = lib or load()
    if pat is None:
        pat = pattern(mesh.npoin, mesh.lnods, lib=lib)
    bptr, bcol, emap = pat
    nnzb = int(bptr[-1])
    ln = np.ascontiguousarray(mesh.lnods, dtype=np.int32)
    co = _f64(mesh.coord)
    ve = _f64(mesh.velocity if velocity is None else velocity)
    em = np.ascontiguousarray(emap, dtype=np.int32)
    values = np.zeros((nnzb, 4, 4))
    rhs = np.zeros((mesh.npoin, 4))
    st = lib.oracle_assemble(mesh.npoin, mesh.nelem, _p(ln), _p(co), _p(ve),
                             mesh.rho if rho is None else rho, mesh.mu if mu is None else mu,
                             mesh.dt if dt is None else dt, nnzb, _p(em), _p(values), _p(rhs))
    if st != OR_OK:
        raise ValueError(f"oracle_assemble status {st}")
    return values, rhs


def residual(mesh, lib=None, rho=None, mu=None, dt=None, velocity=None):
    """Explicit-residual outputs of Listing 2 for a Mesh: (rhsid [npoin][3], dt_rho [npoin],
    mass_rho [npoin])."""
    lib = lib or load()
    ln = np.ascontiguousarray(mesh.lnods, dtype=np.int32)
    co = _f64(mesh.coord)
    ve = _f64(mesh.velocity if velocity is None else velocity)
    rhsid = np.zeros((mesh.npoin, 3))
    dt_rho = np.zeros(mesh.npoin)
    mass_rho = np.zeros(mesh.npoin)
    st = lib.oracle_residual(mesh.npoin, mesh.nelem, _p(ln), _p(co), _p(ve),
                             mesh.rho if rho is None else rho, mesh.mu if mu is None else mu,
                             mesh.dt if dt is None else dt, _p(rhsid), _p(dt_rho), _p(mass_rho))
    if st != OR_OK:
        raise ValueError(f"oracle_residual status {st}")
    return rhsid, dt_rho, mass_rho


def assemble_rows(mesh, rows, maxdeg=64, lib=None, velocity=None, rho=None, mu=None, dt=None):
    """Assembly restricted to the given node rows: returns (cols [s][maxdeg] -1 padded,
    deg [s], vals [s][maxdeg][4][4], rhs [s][4])."""
    lib = lib or load()
    rows = np.asarray(rows, dtype=np.int64)
    slot = np.full(mesh.npoin, -1, dtype=np.int64)
    slot[rows] = np.arange(rows.size, dtype=np.int64)
    ns = rows.size
    cols = np.zeros((ns, maxdeg), dtype=np.int32)
    deg = np.zeros(ns, dtype=np.int32)
    vals = np.zeros((ns, maxdeg, 4, 4))
    rhs = np.zeros((ns, 4))
    ln = np.ascontiguousarray(mesh.lnods, dtype=np.int32)
    st = lib.oracle_assemble_rows(mesh.npoin, mesh.nelem, _p(ln), _p(_f64(mesh.coord)),
                                  _p(_f64(mesh.velocity if velocity is None else velocity)),
                                  mesh.rho if rho is None else rho, mesh.mu if mu is None else mu,
                                  mesh.dt if dt is None else dt, ns, _p(slot), maxdeg, _p(cols),
                                  _p(deg), _p(vals), _p(rhs))
    if st != OR_OK:
        raise ValueError(f"oracle_assemble_rows status {st}")
    return cols, deg, vals, rhs


# ---- 2-D quadrilateral family (nsa_oracle_q1.c) ----------------------------------------------

def q1_element(X, U, rho, mu, dt, rule=2, lib=None):
    """Element matrix A [12][12] (rows test (a,c), cols trial (b,c'), dof 3a+c, c = 2 pressure) and
    RHS [12] of a bilinear quadrilateral with the rule x rule Gauss-Legendre rule (2 is the method's)."""
    lib = lib or load()
    X, U = _f64(X, (4, 2)), _f64(U, (4, 2))
    A = np.zeros((12, 12))
    b = np.zeros(12)
    st = lib.oracle_q1_element_rule(_p(X), _p(U), rho, mu, dt, int(rule), _p(A), _p(b))
    if st != OR_OK:
        raise ValueError(f"oracle_q1_element status {st}")
    return A, b


def q1_element_integrals(X, U, rho, mu, dt, lib=None):
    """2x2-rule integrals of one quadrilateral: area, h, tau1, tau2, mass, stiffness, convection, aa."""
    lib = lib or load()
    X, U = _f64(X, (4, 2)), _f64(U, (4, 2))
    out = dict(scal=np.zeros(4), mass=np.zeros((4, 4)), stiff=np.zeros((4, 4)), conv=np.zeros((4, 4)),
               aa=np.zeros((4, 4)))
    st = lib.oracle_q1_element_integrals(_p(X), _p(U), rho, mu, dt, *[_p(out[k]) for k in
                                         ("scal", "mass", "stiff", "conv", "aa")])
    if st != OR_OK:
        raise ValueError(f"oracle_q1_element_integrals status {st}")
    s = out.pop("scal")
    out.update(area=s[0], h=s[1], tau1=s[2], tau2=s[3])
    return out


def q1_validate(npoin, lnods, coord, lib=None):
    lib = lib or load()
    ln = np.ascontiguousarray(lnods, dtype=np.int32)
    co = _f64(coord)
    bad = C.c_int64(-1)
    st = lib.oracle_q1_validate(int(npoin), ln.shape[0], _p(ln), _p(co), C.byref(bad))
    return st, bad.value


def q1_assemble(mesh, pat=None, lib=None, rho=None, mu=None, dt=None, velocity=None):
    """values [nnzb][3][3] and rhs [npoin][3] of a quadrilateral mesh (inputs.QuadMesh)."""
    lib = lib or load()
    if pat is None:
        pat = pattern(mesh.npoin, mesh.lnods, lib=lib)
    bptr, _, emap = pat
    nnzb = int(bptr[-1])
    ln = np.ascontiguousarray(mesh.lnods, dtype=np.int32)
    vel = _f64(mesh.velocity if velocity is None else velocity)
    values = np.zeros((nnzb, 3, 3))
    rhs = np.zeros((mesh.npoin, 3))
    st = lib.oracle_q1_assemble(mesh.npoin, mesh.nelem, _p(ln), _p(_f64(mesh.coord)), _p(vel),
                                mesh.rho if rho is None else rho, mesh.mu if mu is None else mu,
                                mesh.dt if dt is None else dt, nnzb, _p(np.ascontiguousarray(emap, dtype=np.int32)),
                                _p(values), _p(rhs))
    if st != OR_OK:
        raise ValueError(f"oracle_q1_assemble status {st}")
    return values, rhs
