"""Parity metric: per block class X in {uu, up, pu, pp} and RHS class {u, p},
err_X = max |got - ref| / max |ref| over the entries of that class. (Per-entry relative error is
ill-posed here: on the unjittered Kuhn cube some Laplacian entries are exactly zero.)"""
import numpy as np

TOL_FP64 = 1e-12
TOL_MIXED = 1e-5


def class_errors(values, ref_values, rhs, ref_rhs):
    v = np.asarray(values, dtype=np.float64).reshape(-1, 4, 4)
    r = np.asarray(ref_values, dtype=np.float64).reshape(-1, 4, 4)
    out = {}
    sl = {"uu": (slice(0, 3), slice(0, 3)), "up": (slice(0, 3), slice(3, 4)),
          "pu": (slice(3, 4), slice(0, 3)), "pp": (slice(3, 4), slice(3, 4))}
    for k, (i, j) in sl.items():
        ref = r[:, i, j]
        den = np.abs(ref).max() if ref.size else 0.0
        diff = np.abs(v[:, i, j] - ref).max() if ref.size else 0.0
        out[k] = float(diff / den) if den > 0 else float(diff)
    b = np.asarray(rhs, dtype=np.float64).reshape(-1, 4)
    rb = np.asarray(ref_rhs, dtype=np.float64).reshape(-1, 4)
    for k, sel in (("rhs_u", slice(0, 3)), ("rhs_p", slice(3, 4))):
        ref = rb[:, sel]
        den = np.abs(ref).max() if ref.size else 0.0
        diff = np.abs(b[:, sel] - ref).max() if ref.size else 0.0
        out[k] = float(diff / den) if den > 0 else float(diff)
    return out


def assert_parity(values, ref_values, rhs, ref_rhs, tol, what=""):
    err = class_errors(values, ref_values, rhs, ref_rhs)
    bad = {k: v for k, v in err.items() if not (v <= tol)}
    assert not bad, f"{what}: block-class errors above {tol:g}: {bad} (all: {err})"
    return err
