"""Planted mistakes in a copy of the oracle must each be caught by at least one pin.

Every mutant is a one-line textual change to a temporary copy of oracle/nsa_oracle.c (a dropped
term, a wrong sign, a transposed index, a wrong constant, a pattern or scatter slip). The copy
is compiled with the oracle's own flags and the pins of oracle_pins.py run against it in a
subprocess; the test fails if any mutant passes every pin.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nsa_oracle.c")

MUTANTS = {
    "drop_mass": ("rdt * Na * Nb + rho * Na * agb", "rho * Na * agb"),
    "convection_transposed": ("rho * Na * agb + t1", "rho * Nb * aga + t1"),
    "supg_no_transient": ("t1 * rho * aga * (rho * agb + rdt * Nb)", "t1 * rho * aga * (rho * agb)"),
    "viscous_transposed": ("mu * V * E->gpcar[a][cp] * E->gpcar[b][c]", "mu * V * E->gpcar[a][c] * E->gpcar[b][cp]"),
    "graddiv_transposed": ("E->tau2 * V * E->gpcar[a][c] * E->gpcar[b][cp]", "E->tau2 * V * E->gpcar[a][cp] * E->gpcar[b][c]"),
    "pressure_sign": ("(-Nb * E->gpcar[a][c]", "(Nb * E->gpcar[a][c]"),
    "continuity_wrong_node": ("(Na * E->gpcar[b][c]", "(Na * E->gpcar[a][c]"),
    "supg_pressure_wrong_node": ("t1 * rho * aga * E->gpcar[b][c]", "t1 * rho * agb * E->gpcar[b][c]"),
    "pspg_no_transient": ("(rdt * Nb + rho * agb)", "(rho * agb)"),
    "pp_wrong_tau": ("E->tau1 * V * E->wgrgr[a][b]", "E->tau2 * V * E->wgrgr[a][b]"),
    "rhs_supg_sign": ("+ t1 * rho * rdt * aga * E->gpvel[g][c]", "- t1 * rho * rdt * aga * E->gpvel[g][c]"),
    "rhs_galerkin_no_shape": ("rdt * E->gpvel[g][c] * Na +", "rdt * E->gpvel[g][c] +"),
    "rhs_pspg_no_tau": ("w * t1 * rdt * gdu", "w * rdt * gdu"),
    "tau1_no_transient": ("1.0 / (rho / dt + 4.0", "1.0 / (4.0"),
    "tau1_c1": ("4.0 * mu / (h * h)", "2.0 * mu / (h * h)"),
    "tau1_no_convective": ("+ 2.0 * rho * anorm / h)", ")"),
    "tau2_no_convective": ("E->tau2 = mu + 0.5 * rho * anorm * h;", "E->tau2 = mu;"),
    "anorm_squared": ("double anorm = sqrt(an2);", "double anorm = an2;"),
    "h_no_6": ("cbrt(6.0 * E->vol)", "cbrt(E->vol)"),
    "gauss_swapped": ("(a == g) ? alpha : beta", "(a == g) ? beta : alpha"),
    "gauss_alpha": ("(5.0 + 3.0 * sq5) / 20.0", "(5.0 + 3.0 * sq5) / 19.0"),
    "jacobian_transposed": ("J[r][s] = E->elcod[s + 1][r] - E->elcod[0][r];", "J[r][s] = E->elcod[r + 1][s] - E->elcod[0][s];"),
    "grad0_sign": ("E->gpcar[0][d] -= jinv[s][d];", "E->gpcar[0][d] += jinv[s][d];"),
    "inverse_transposed": ("jinv[s][d] = cof[d][s] / det;", "jinv[s][d] = cof[s][d] / det;"),
    "volume_factor": ("E->vol = fabs(det) / 6.0;", "E->vol = fabs(det) / 2.0;"),
    "drop_laplacian": ("if (c == cp) v += mu * V * E->wgrgr[a][b];", "if (c == cp) v += 0.0;"),
    "agrau_wrong_node": ("s += E->gpvel[g][d] * E->gpcar[a][d];", "s += E->gpvel[g][d] * E->gpcar[g][d];"),
    "gpvel_one_node": ("s += E->shape[g][a] * E->elvel[a][c];", "s += E->shape[g][a] * E->elvel[g][c];"),
    "scatter_block_transposed": ("                        blk[4 * c + cp] += E.elauu[4 * a + c][4 * b + cp];",
                                 "                        blk[4 * cp + c] += E.elauu[4 * a + c][4 * b + cp];"),
    "rhs_wrong_node": ("double *r = rhs + 4 * (size_t)lnods[4 * e + a];", "double *r = rhs + 4 * (size_t)lnods[4 * e + (a + 1) % 4];"),
    "pattern_keeps_duplicates": ("if (k == lo || pairs[k] != pairs[k - 1]) bcol[nnzb++] = pairs[k];", "bcol[nnzb++] = pairs[k];"),
    "emap_search_off": ("if (bcol[mid] < col) lo = mid + 1; else hi = mid;", "if (bcol[mid] <= col) lo = mid + 1; else hi = mid;"),
    "residual_sign": ("r -= E.elauu[4 * a + c][4 * b + cp] * E.elvel[b][cp];", "r += E.elauu[4 * a + c][4 * b + cp] * E.elvel[b][cp];"),
    "residual_transposed": ("r -= E.elauu[4 * a + c][4 * b + cp] * E.elvel[b][cp];", "r -= E.elauu[4 * b + cp][4 * a + c] * E.elvel[b][cp];"),
    "residual_with_pressure_column": ("for (int cp = 0; cp < NDIME; cp++) r -=", "for (int cp = 0; cp < NDOFN; cp++) r -="),
    "residual_wrong_velocity_node": ("E.elauu[4 * a + c][4 * b + cp] * E.elvel[b][cp];", "E.elauu[4 * a + c][4 * b + cp] * E.elvel[a][cp];"),
    "lumped_tau2": ("const double dtr = lump * E.tau1,", "const double dtr = lump * E.tau2,"),
    "lumped_no_shape": ("lump += E.gpvol[g] * E.shape[g][a];", "lump += E.gpvol[g];"),
    "rows_insert_after_equal": ("while (k < deg[s] && row[k] < col) k++;", "while (k < deg[s] && row[k] <= col) k++;"),
    "rows_keep_duplicates": ("if (k < deg[s] && row[k] == col) continue;", "if (0) continue;"),
    "rows_block_transposed": ("for (int cp = 0; cp < NDOFN; cp++) blk[4 * c + cp] +=",
                              "for (int cp = 0; cp < NDOFN; cp++) blk[4 * cp + c] +="),
    "rows_rhs_wrong_node": ("rhs_s[4 * s + c] += E.elrhs[4 * a + c];", "rhs_s[4 * s + c] += E.elrhs[4 * ((a + 1) % 4) + c];"),
    "rows_touched_first_vertex": ("touched |= rowslot[lnods[4 * e + a]] >= 0;", "touched |= rowslot[lnods[4 * e]] >= 0;"),
    "rows_next_block": ("double *blk = vals + 16 * ((size_t)s * maxdeg + k);",
                        "double *blk = vals + 16 * ((size_t)s * maxdeg + k + (k + 1 < deg[s]));"),
}

DRIVER = r"""
import sys
sys.path.insert(0, {root!r})
import oracle
from tests import oracle_pins as P
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
                    path, "-lm"], check=True)
    r = subprocess.run([sys.executable, "-c", DRIVER.format(root=ROOT, lib=lib)], capture_output=True,
                       text=True, timeout=300)
    if r.returncode != 0:   # a crash also counts as caught, but report it
        return name, f"crashed rc={r.returncode}"
    line = [l for l in r.stdout.splitlines() if l.startswith("FAILED_PINS")][-1]
    return name, line.split(" ", 1)[1] if " " in line else ""


def test_every_mutant_is_caught():
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max_workers=6) as ex:
            results = dict(ex.map(lambda n: _run_mutant(n, tmp), sorted(MUTANTS)))
    survivors = [n for n, f in results.items() if not f]
    for n, f in sorted(results.items()):
        print(f"{n:28s} caught by: {f}")
    assert not survivors, f"mutants not caught by any pin: {survivors}"
