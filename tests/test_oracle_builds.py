"""The oracle's two extra builds of the same C source, used for measurement only: the OpenMP build
that times the CPU baseline, and the operation-counting build that gives the method's flops per
element. Both must compute what the serial, pinned build computes; the flop count per element must be
the same on every mesh and equal to the figures the benchmark's roofline uses."""
import importlib.util
import os

import numpy as np
import pytest

import oracle
from paper_2111_05651_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def bench_module():
    spec = importlib.util.spec_from_file_location("bench_consts", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


MESHES = {
    "cube8": lambda: inputs.config_small(),
    "perm6": lambda: inputs.make_mesh(6, jitter=True, permute=True, seed=3),
    "soup": lambda: inputs.bad_element_soup(eps=(1e-2, 1e-4)),
    "hub2": lambda: inputs.hub_mesh(2, seed=2),
}


@pytest.mark.parametrize("name", sorted(MESHES))
def test_flop_count_per_element(name):
    m = MESHES[name]()
    b = bench_module()
    pat = oracle.pattern(m.npoin, m.lnods)
    n_res, out_res = oracle.flops(m, "residual")
    n_asm, out_asm = oracle.flops(m, "assemble", pat)
    assert n_res == b.METHOD_FLOPS_RESIDUAL * m.nelem
    assert n_asm == b.METHOD_FLOPS_ASSEMBLY * m.nelem
    # the counting build computes the serial oracle's values, bit for bit
    for a, e in zip(out_res, oracle.residual(m)):
        assert np.array_equal(a, e)
    for a, e in zip(out_asm, oracle.assemble(m, pat)):
        assert np.array_equal(a, e)


@pytest.mark.parametrize("name", ["cube8", "perm6", "hub2"])
def test_openmp_build_matches_serial(name):
    m = MESHES[name]()
    omp = oracle.load_omp()
    assert int(omp.oracle_threads()) >= 1
    pat = oracle.pattern(m.npoin, m.lnods)
    # atomic adds in any order: equal up to the rounding of the sums
    for a, e in zip(oracle.assemble(m, pat, lib=omp), oracle.assemble(m, pat)):
        scale = np.abs(e).max()
        assert np.abs(a - e).max() <= 1e-13 * scale
    for a, e in zip(oracle.residual(m, lib=omp), oracle.residual(m)):
        scale = np.abs(e).max()
        assert np.abs(a - e).max() <= 1e-13 * scale
