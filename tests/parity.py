"""Parity metric: per block class X in {uu, up, pu, pp} and RHS class {u, p},
err_X = max |got - ref| / max |ref| over the entries of that class. (Per-entry relative error is
ill-posed here: on the unjittered Kuhn cube some Laplacian entries are exactly zero.)"""
import numpy as np

TOL_FP64 = 1e-12
TOL_MIXED = 1e-5


def class_errors(values, ref_values, rhs, ref_rhs, ndofn=4):
    """ndofn 4: tetrahedra (u, v, w, p); 3: quadrilaterals (u, v, p). Pressure is the last dof."""
    k = ndofn - 1
    v = np.asarray(values, dtype=np.float64).reshape(-1, ndofn, ndofn)
    r = np.asarray(ref_values, dtype=np.float64).reshape(-1, ndofn, ndofn)
    out = {}
    sl = {"uu": (slice(0, k), slice(0, k)), "up": (slice(0, k), slice(k, k + 1)),
          "pu": (slice(k, k + 1), slice(0, k)), "pp": (slice(k, k + 1), slice(k, k + 1))}
    for name, (i, j) in sl.items():
        ref = r[:, i, j]
        den = np.abs(ref).max() if ref.size else 0.0
        diff = np.abs(v[:, i, j] - ref).max() if ref.size else 0.0
        out[name] = float(diff / den) if den > 0 else float(diff)
    b = np.asarray(rhs, dtype=np.float64).reshape(-1, ndofn)
    rb = np.asarray(ref_rhs, dtype=np.float64).reshape(-1, ndofn)
    for name, sel in (("rhs_u", slice(0, k)), ("rhs_p", slice(k, k + 1))):
        ref = rb[:, sel]
        den = np.abs(ref).max() if ref.size else 0.0
        diff = np.abs(b[:, sel] - ref).max() if ref.size else 0.0
        out[name] = float(diff / den) if den > 0 else float(diff)
    return out


def assert_parity(values, ref_values, rhs, ref_rhs, tol, what="", ndofn=4):
    err = class_errors(values, ref_values, rhs, ref_rhs, ndofn)
    bad = {k: v for k, v in err.items() if not (v <= tol)}
    assert not bad, f"{what}: block-class errors above {tol:g}: {bad} (all: {err})"
    return err
