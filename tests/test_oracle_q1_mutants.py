"""Planted mistakes in a copy of the 2-D oracle (nsa_oracle_q1.c) must each be caught by a pin of
oracle_q1_pins.py: a dropped term, a wrong sign, a transposed index, a wrong Gauss point or weight,
a wrong element length, a scatter slip. Same procedure as the tetrahedral mutants."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC3 = os.path.join(ROOT, "oracle", "nsa_oracle.c")
SRC = os.path.join(ROOT, "oracle", "nsa_oracle_q1.c")

MUTANTS = {
    "drop_mass": ("rdt * Na * Nb + rho * Na * agb", "rho * Na * agb"),
    "convection_transposed": ("rho * Na * agb + t1", "rho * Nb * aga + t1"),
    "viscous_transposed": ("mu * E->gpcar[g][a][cp] * E->gpcar[g][b][c]", "mu * E->gpcar[g][a][c] * E->gpcar[g][b][cp]"),
    "graddiv_dropped": ("+ E->tau2 * E->gpcar[g][a][c] * E->gpcar[g][b][cp]", "+ 0.0"),
    "pressure_sign": ("(-Nb * E->gpcar[g][a][c]", "(Nb * E->gpcar[g][a][c]"),
    "continuity_wrong_node": ("(Na * E->gpcar[g][b][c]", "(Na * E->gpcar[g][a][c]"),
    "pspg_no_transient": ("(rdt * Nb + rho * agb)", "(rho * agb)"),
    "pp_wrong_tau": ("w * E->tau1 * E->wgrgr[g][a][b]", "w * E->tau2 * E->wgrgr[g][a][b]"),
    "gauss_point": ("x[0] = -1.0 / sqrt(3.0); x[1] = 1.0 / sqrt(3.0);", "x[0] = -0.5; x[1] = 0.5;"),
    "jacobian_transposed": ("J[r][s] += E->elcod[a][r] * deriv[a][s]", "J[r][s] += E->elcod[a][s] * deriv[a][r]"),
    "inverse_sign": ("{{J[1][1] / det, -J[0][1] / det}", "{{J[1][1] / det, J[0][1] / det}"),
    "shape_derivative": ("deriv[a][1] = 0.25 * ETA[a] * (1.0 + XI[a] * xi);", "deriv[a][1] = 0.25 * ETA[a] * (1.0 + XI[a] * eta);"),
    "hleng_area": ("E->hleng = sqrt(E->area);", "E->hleng = E->area;"),
    "rhs_supg_sign": ("+ t1 * rho * rdt * aga * E->gpvel[g][c]", "- t1 * rho * rdt * aga * E->gpvel[g][c]"),
    "scatter_transposed": ("blk[3 * c + cp] += E.elauu[3 * a + c][3 * b + cp]", "blk[3 * c + cp] += E.elauu[3 * a + cp][3 * b + c]"),
}

DRIVER = """
import sys
sys.path.insert(0, {root!r})
import oracle
from tests import oracle_q1_pins as P
lib = oracle.load({lib!r})
failed = []
for pin in P.ALL_PINS:
    try:
        pin(lib)
    except Exception as exc:
        failed.append(pin.__name__)
print("FAILED_PINS", ",".join(failed))
"""


def _run_mutant(name, tmp):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutant {name}: snippet found {src.count(old)} times"
    path = os.path.join(tmp, f"{name}.c")
    lib = os.path.join(tmp, f"lib{name}.so")
    open(path, "w").write(src.replace(old, new))
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", "-Wno-unknown-pragmas", "-o", lib,
                    SRC3, path, "-lm"], check=True)
    r = subprocess.run([sys.executable, "-c", DRIVER.format(root=ROOT, lib=lib)], capture_output=True, text=True,
                       timeout=300)
    if r.returncode != 0:
        return name, f"crashed rc={r.returncode}"
    line = [l for l in r.stdout.splitlines() if l.startswith("FAILED_PINS")][-1]
    return name, line.split(" ", 1)[1] if " " in line else ""


def test_every_q1_mutant_is_caught():
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max_workers=6) as ex:
            results = dict(ex.map(lambda n: _run_mutant(n, tmp), sorted(MUTANTS)))
    survivors = [n for n, f in results.items() if not f]
    for n, f in sorted(results.items()):
        print(f"{n:24s} caught by: {f}")
    assert not survivors, f"mutants not caught by any pin: {survivors}"
