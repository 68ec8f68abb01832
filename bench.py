#!/usr/bin/env python3
"""Throughput of P1-tet incompressible Navier-Stokes assembly on one MI355X.

One step = one nsa_assemble call: every element of the mesh gathered, integrated and added into
the block-CSR matrix and RHS (values and RHS overwritten), inputs already resident in HBM.
Default workload: the 128^3 Kuhn cube (12,582,912 tets, 2,146,689 nodes, 31,802,497 4x4 blocks),
jittered, randomly permuted then RCM-renumbered, elements sorted by smallest node, Taylor-Green
velocity plus 1% noise, rho=1, mu=1e-3, dt=5e-3. The headline is the plain FP64 kernel; the mixed
form (FP64 geometry and accumulation, FP32 element integration) is timed beside it on the same GPU
with its block-class error against the FP64 result. Prints one JSON line.
"""
import argparse
import gc
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
KERNEL_SRCS = [os.path.join(ROOT, "paper_2111_05651_amd", "csrc", f)
               for f in ("nsa_kernels.hip", "nsa_device.h", "nsa_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(nelem, npoin, nnzb):
    """Bytes the method must move once: connectivity (16/elem), coordinates + velocity (48/node),
    every block written once (128/block), RHS (32/node)."""
    return 16 * nelem + 48 * npoin + 128 * nnzb + 32 * npoin


def source_digest():
    """Digest of the sources the tiled kernels are compiled from (counter figures are only valid
    for the code they were taken on)."""
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def make_workload(name):
    from paper_2111_05651_amd import inputs
    return {"cube128": inputs.config_128, "cube64": inputs.config_64, "cube8": inputs.config_small}[name]()


def time_steps(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for s, e in evs:
        s.record(stream)
        fn()
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [s.elapsed_time(e) for s, e in evs]
    total = evs[0][0].elapsed_time(evs[-1][1])
    return total / steps, per, wall


def timing_series(fn, stream, est_ms, seconds=1.0, cap=20000):
    """Per-launch device times over a series of at least `seconds` of launches (after the contract's
    K timed steps): count, total seconds, median, min and mean launch in ms."""
    import math
    import torch
    per = []
    n = max(20, min(cap, int(math.ceil(seconds * 1e3 / max(est_ms, 1e-3)))))
    while n > 0:
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        per += [a.elapsed_time(b) for a, b in evs]
        # the estimate includes host overhead between launches: top the series up to `seconds` of launches
        short = seconds * 1e3 - sum(per)
        n = min(cap - len(per), int(math.ceil(short / statistics.fmean(per))) + 1) if short > 0 else 0
    n = len(per)
    return {"launches": n, "total_s": sum(per) / 1e3, "median_ms": statistics.median(per), "min_ms": min(per),
            "mean_ms": statistics.fmean(per)}


def bandwidth_probes(gib=2.0):
    """What this device's HBM gives plain streams (the library's probe kernels, 16-byte accesses, one
    pass each): best of 10 launches of a read, a write and a copy of `gib` GiB (copy: read + write
    bytes)."""
    import torch
    from paper_2111_05651_amd import nsa
    n = int(gib * 2 ** 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    sink = torch.zeros(2, dtype=torch.float64, device="cuda:0")
    out = {"bytes": 8 * n}
    for name, kind, src, dst, nbytes in (("read", nsa.PROBE_READ, a, sink, 8 * n),
                                         ("write", nsa.PROBE_WRITE, None, b, 8 * n),
                                         ("copy", nsa.PROBE_COPY, a, b, 16 * n)):
        st = timing_series(lambda: nsa.bandwidth_probe(kind, src, dst), torch.cuda.current_stream(), 1.0,
                           seconds=0.0, cap=10)
        out[f"{name}_GBs"] = nbytes / (st["min_ms"] / 1e3) / 1e9
    del a, b, sink
    torch.cuda.empty_cache()
    return out


def host_description():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def class_diff(a_values, a_rhs, b_values, b_rhs, ndofn=4):
    """Per block class {uu, up, pu, pp} and RHS class {u, p}: max|a - b| / max|b| (pressure is the last
    of the ndofn dofs of a node: 4 for tetrahedra, 3 for quadrilaterals)."""
    q = ndofn - 1
    out = {}
    sl = {"uu": (slice(0, q), slice(0, q)), "up": (slice(0, q), slice(q, q + 1)), "pu": (slice(q, q + 1), slice(0, q)),
          "pp": (slice(q, q + 1), slice(q, q + 1))}
    for k, (i, j) in sl.items():
        ref = b_values[:, i, j]
        out[k] = float((a_values[:, i, j] - ref).abs().max() / ref.abs().max())
    for k, c in (("rhs_u", slice(0, q)), ("rhs_p", slice(q, q + 1))):
        ref = b_rhs[:, c]
        den = ref.abs().max()
        out[k] = float((a_rhs[:, c] - ref).abs().max() / den) if den > 0 else float((a_rhs[:, c] - ref).abs().max())
    return out


def cpu_baseline(m, nelem_sample):
    """The oracle on the first nelem_sample elements of the same mesh: its OpenMP build (the same C
    source, element loop on all host threads, atomic adds) and, beside it, the serial build the tests
    pin. FP64, pattern build untimed."""
    import oracle
    from paper_2111_05651_amd import inputs
    sub = inputs.Mesh(n=m.n, lnods=m.lnods[:nelem_sample].copy(), coord=m.coord, velocity=m.velocity,
                      rho=m.rho, mu=m.mu, dt=m.dt)
    pat = oracle.pattern(sub.npoin, sub.lnods)
    omp = oracle.load_omp()
    t0 = time.perf_counter()
    oracle.assemble(sub, pat, lib=omp)
    t_omp = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.assemble(sub, pat)
    t_ser = time.perf_counter() - t0
    threads = int(omp.oracle_threads())
    return {"value": nelem_sample / t_omp, "unit": "elements/s", "cores": threads, "kind": "oracle",
            "sample": f"first {nelem_sample} elements of the same mesh, FP64 C oracle built with OpenMP on "
                      f"{threads} threads ({t_omp:.1f} s); pattern build untimed",
            "serial": {"value": nelem_sample / t_ser, "cores": 1, "seconds": t_ser}, **host_description()}


def cpu_baseline_residual(m):
    """The oracle's explicit-residual routine on the whole mesh: its OpenMP build on all host threads
    and, beside it, the serial build the tests pin. FP64."""
    import oracle
    omp = oracle.load_omp()
    t0 = time.perf_counter()
    oracle.residual(m, lib=omp)
    t_omp = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.residual(m)
    t_ser = time.perf_counter() - t0
    threads = int(omp.oracle_threads())
    return {"value": m.nelem / t_omp, "unit": "elements/s", "cores": threads, "kind": "oracle",
            "sample": f"all {m.nelem} elements of the same mesh, FP64 C oracle (residual outputs) built with "
                      f"OpenMP on {threads} threads ({t_omp:.1f} s)",
            "serial": {"value": m.nelem / t_ser, "cores": 1, "seconds": t_ser}, **host_description()}


FLOPS_FILE = os.path.join(ROOT, "profiles", "residual_flops.json")
PEAK_FP64_TFLOPS = 78.6        # MI355X FP64 vector, published
PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector, published (counts packed FP32 instructions)
FP32_NO_PACKED_TFLOPS = 78.6   # 256 CUs x 64 FP32 lanes per clock x 2 (FMA) x 2.4 GHz: the library is
                               # built without packed FP32 instructions
# Floating-point operations per element of the method in the order of Listing 1, Gauss-point loops
# included, as counted by the oracle's instrumented build (the same count on every mesh; a CPU test
# checks both figures): the explicit-residual outputs, and the matrix and RHS.
METHOD_FLOPS_RESIDUAL = 6913
METHOD_FLOPS_ASSEMBLY = 6837


def residual_flops(kernel_key):
    """VALU flops per element (FP64, FP32) of the residual kernel from the committed counter
    summary, if it was taken on this kernel source."""
    try:
        with open(FLOPS_FILE) as f:
            rec = json.load(f).get(kernel_key)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha256") != source_digest():
        return None
    return rec


def run_residual(args, m, prec):
    """The explicit-residual outputs of Listing 2 (rhsid, dt_rho_nsi, mass_rho_nsi), no matrix."""
    import torch
    from paper_2111_05651_amd import nsa
    cached = args.residual_geometry == "precomputed"
    mesh = nsa.Mesh.from_inputs(m, tile_blocks=0, tile_blocks_colour=0, tile_rows_residual=args.tile_rows_residual,
                                keep_direct=False, residual_geometry=cached)
    mesh.upload("cuda:0")
    info = mesh.info
    log(f"mesh registered: residual tiles={info.residual_ntiles} geometry {args.residual_geometry} records/nelem="
        f"{info.residual_records / max(m.nelem, 1):.2f} lds={info.residual_lds_bytes}")
    vel = torch.from_numpy(m.velocity).to("cuda:0")
    r = torch.empty((m.npoin, 3), dtype=torch.float64, device="cuda:0")
    t = torch.empty(m.npoin, dtype=torch.float64, device="cuda:0")
    w = torch.empty_like(t)
    stream = torch.cuda.current_stream()

    def step(p=prec):
        nsa.assemble_residual(mesh, vel, m.rho, m.mu, m.dt, precision=p, rhsid=r, dt_rho=t, mass_rho=w, stream=stream)

    est, _, _ = time_steps(step, 3, 1, stream)
    series = timing_series(step, stream, est, seconds=args.series_seconds)
    log(f"timing series: {series['launches']} launches over {series['total_s']:.2f} s, median "
        f"{series['median_ms']:.4f} ms, min {series['min_ms']:.4f} ms")
    ms, per, wall = time_steps(step, args.steps, args.warmup, stream)
    log(f"timed {args.steps} steps: {ms:.4f} ms/step (wall {wall:.3f} s)")
    beside = None
    if not args.no_beside:
        other = nsa.FP64 if prec == nsa.MIXED else nsa.MIXED
        first = [x.clone() for x in (r, t, w)]
        ms_o, _, _ = time_steps(lambda: step(other), args.steps, args.warmup, stream)
        series_o = timing_series(lambda: step(other), stream, ms_o, seconds=args.series_seconds)
        f64, mix = (first, (r, t, w)) if other == nsa.MIXED else ((r, t, w), first)
        err = {n: float((a - b).abs().max() / b.abs().max()) for n, a, b in zip(("rhsid", "dt_rho", "mass_rho"), mix, f64)}
        beside = {"precision": "mixed" if other == nsa.MIXED else "fp64", "value": m.nelem / (ms_o / 1e3),
                  "ms_per_step": ms_o, "unit": "elements/s", "same_gpu": True, "timing": series_o,
                  "mixed_vs_fp64_error": err}
        log(f"{beside['precision']} beside it: {ms_o:.4f} ms/step; mixed vs FP64 errors {err}")
    launch_ms = series["mean_ms"]
    rt = "float" if prec == nsa.MIXED else "double"
    kname = f"k_residual<{rt},256>" if not cached else f"k_residual<{rt},256,precomputed geometry>"
    peak = PEAK_FP64_TFLOPS if prec == nsa.FP64 else PEAK_FP32_TFLOPS
    # Work counted once per element: the kernel's VALU flops (rocprofv3, this kernel source) divided by
    # the (element, tile) evaluations per element -- an element whose rows fall in several tiles is
    # integrated once per tile, and only one of those evaluations is the method's work.
    evals = info.residual_records / max(m.nelem, 1)
    fl = residual_flops(f"{kname}@{args.workload}/rows{args.tile_rows_residual}")
    roof = {"bound": "alu", "achieved": None, "peak": peak, "unit": "TFLOP/s", "frac": None, "traffic": None,
            "kernel": kname, "evaluations_per_element": evals,
            "method_flops_per_element_listing1": METHOD_FLOPS_RESIDUAL,
            "method_flops_basis": "the method's floating-point operations per element in the order of Listing 1 "
                                  "(Gauss-point loops included), counted by the oracle's instrumented build; "
                                  "context only -- the kernel's closed forms for linear tetrahedra take fewer",
            "avg_launch_ms": launch_ms,
            "launch_ms_basis": f"mean of the {series['launches']} launches of the timing series"}
    if fl:
        valu = fl["fp64_flops_per_element"] + fl["fp32_flops_per_element"]
        per_elem = valu / evals
        achieved = per_elem * m.nelem / (launch_ms / 1e3) / 1e12
        roof.update({"achieved": achieved, "frac": achieved / peak, "flops_per_element": per_elem,
                     "flops_basis": "VALU flops per element evaluation counted by rocprofv3 on this kernel "
                                    "source, once per element",
                     "valu_flops_per_element_all_evaluations": valu,
                     "valu_TFLOPs_all_evaluations": valu * m.nelem / (launch_ms / 1e3) / 1e12})
        if prec == nsa.MIXED:
            roof["peak_fp32_without_packed"] = FP32_NO_PACKED_TFLOPS
            roof["frac_vs_fp32_without_packed"] = achieved / FP32_NO_PACKED_TFLOPS
    else:
        roof["note"] = "no VALU counter record for this kernel source in profiles/residual_flops.json"
    nbytes = 16 * m.nelem + 48 * m.npoin + 40 * m.npoin
    line = {
        "metric": "elements assembled/s (explicit-residual outputs)", "value": m.nelem / (ms / 1e3),
        "unit": "elements/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == nsa.MIXED else "f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {m.name}", "path": "residual", "nelem": m.nelem, "npoin": m.npoin,
                   "precision": args.precision, "rows_per_tile": args.tile_rows_residual, "rho": m.rho, "mu": m.mu,
                   "dt": m.dt, "geometry": args.residual_geometry},
        "hbm_GBs": nbytes / (launch_ms / 1e3) / 1e9, "algorithmic_bytes_per_launch": nbytes,
        "timing": series, "roofline": roof, "beside": beside,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle residual on the whole mesh ...")
        line["cpu_baseline"] = cpu_baseline_residual(m)
    print(json.dumps(line), flush=True)


def run_quads(args, prec):
    """The 2-D family: bilinear quadrilaterals (block-CSR with 3x3 blocks plus RHS)."""
    import torch
    import oracle
    from paper_2111_05651_amd import inputs, nsa
    t0 = time.perf_counter()
    m = {"quad2048": inputs.config_quad2048, "cylinder2d": inputs.config_cylinder2d,
         "venturi2d": inputs.config_venturi2d}[args.workload]()
    log(f"workload {args.workload}: {m.nelem} quadrilaterals, {m.npoin} nodes ({time.perf_counter() - t0:.1f} s)")
    scat = {"atomic": nsa.ATOMIC, "colour": nsa.COLOUR}[args.scatter]
    mesh = nsa.Mesh.from_quads(m).upload("cuda:0")
    info = mesh.info
    log(f"mesh registered: nnzb={info.nnzb} ntiles={info.ntiles[scat]} records/nelem="
        f"{info.tile_runs[scat] / max(m.nelem, 1):.2f} lds={info.tile_lds_bytes[scat]}")
    vel = torch.from_numpy(m.velocity).to("cuda:0")
    values, rhs = mesh.alloc_outputs("cuda:0")
    stream = torch.cuda.current_stream()

    def step(p=prec):
        nsa.assemble(mesh, vel, m.rho, m.mu, m.dt, precision=p, scatter=scat, values=values, rhs=rhs, stream=stream)

    est, _, _ = time_steps(step, 3, 1, stream)
    series = timing_series(step, stream, est, seconds=args.series_seconds)
    log(f"timing series: {series['launches']} launches, median {series['median_ms']:.4f} ms, min {series['min_ms']:.4f} ms")
    ms, _, _ = time_steps(step, args.steps, args.warmup, stream)
    beside = None
    if not args.no_beside:
        other = nsa.FP64 if prec == nsa.MIXED else nsa.MIXED
        fv, fr = values.clone(), rhs.clone()
        ms_o, _, _ = time_steps(lambda: step(other), args.steps, args.warmup, stream)
        series_o = timing_series(lambda: step(other), stream, ms_o, seconds=args.series_seconds)
        if other == nsa.MIXED:
            diff = class_diff(values, rhs, fv, fr, ndofn=3)
        else:
            diff = class_diff(fv, fr, values, rhs, ndofn=3)
        beside = {"precision": "mixed" if other == nsa.MIXED else "fp64", "value": m.nelem / (ms_o / 1e3),
                  "ms_per_step": ms_o, "unit": "elements/s", "same_gpu": True, "timing": series_o,
                  "mixed_vs_fp64_class_error": diff}
        log(f"{beside['precision']} beside it: {ms_o:.4f} ms/step; class errors {diff}")
    # what the method must move: connectivity, coordinates + velocity (2 + 2 doubles per node), every
    # 3x3 block written once, the RHS (3 doubles per node)
    nbytes = 16 * m.nelem + 32 * m.npoin + 72 * info.nnzb + 24 * m.npoin
    launch_ms = series["mean_ms"]
    achieved = nbytes / (launch_ms / 1e3) / 1e9
    rt = "float" if prec == nsa.MIXED else "double"
    roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
            "traffic": None, "kernel": f"k_q1<{rt},{info.tile_threads[scat]}>",
            "algorithmic_bytes_per_launch": nbytes, "avg_launch_ms": launch_ms,
            "launch_ms_basis": f"mean of the {series['launches']} launches of the timing series"}
    line = {"metric": "elements assembled/s", "value": m.nelem / (ms / 1e3), "unit": "elements/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64" if prec == nsa.MIXED else "f64",
            "data": "synthetic",
            "config": {"workload": f"{args.workload}: {m.name}", "family": "bilinear quadrilaterals",
                       "nelem": m.nelem, "npoin": m.npoin, "nnzb": info.nnzb, "precision": args.precision,
                       "scatter": args.scatter, "rho": m.rho, "mu": m.mu, "dt": m.dt},
            "hbm_GBs": achieved, "timing": series, "roofline": roof, "beside": beside}
    if not args.no_cpu_baseline:
        # whole passes over the mesh (or its first --cpu-sample elements) until about 10 s of CPU work
        nsample = min(m.nelem, args.cpu_sample or m.nelem)
        sub = inputs.QuadMesh(nx=m.nx, ny=m.ny, lnods=m.lnods[:nsample].copy(), coord=m.coord, velocity=m.velocity,
                              rho=m.rho, mu=m.mu, dt=m.dt)
        pat = oracle.pattern(sub.npoin, sub.lnods)
        passes, t = 0, 0.0
        while t < 10.0:
            t0 = time.perf_counter()
            oracle.q1_assemble(sub, pat)
            t += time.perf_counter() - t0
            passes += 1
        line["cpu_baseline"] = {"value": passes * nsample / t, "unit": "elements/s", "cores": 1, "kind": "oracle",
                                "sample": f"{passes} pass(es) over {'the whole mesh' if nsample == m.nelem else f'the first {nsample} elements'}"
                                          f" ({nsample} elements), serial FP64 C oracle (nsa_oracle_q1.c, {t:.1f} s); "
                                          "pattern build untimed",
                                **host_description()}
    print(json.dumps(line), flush=True)


def traffic_for(kernel_key, launches_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on this
    exact kernel source and configuration; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    rec = t.get(kernel_key)
    if not rec or rec.get("source_sha256") != source_digest():
        return None
    return rec.get("hbm_bytes_per_launch")


def run_batch(args):
    """64 independent jittered cubes (n ~ U{8..48}): one graph-captured launch of the
    tiled kernel over all of them (mixed precision by default), autotuned; beside it the same 64
    meshes as 64 plain FP64 launches on the same GPU."""
    import torch
    from paper_2111_05651_amd import autotune, inputs, nsa
    prec = {"mixed": nsa.MIXED, "fp64": nsa.FP64}[args.precision]
    if args.workload in ("quad2048", "cylinder2d", "venturi2d"):
        return run_quads(args, prec)
    scat = {"atomic": nsa.ATOMIC, "colour": nsa.COLOUR}[args.scatter]
    t0 = time.perf_counter()
    ms_ = inputs.config_batch()
    nelem = sum(m.nelem for m in ms_)
    log(f"batch of {len(ms_)} meshes, {nelem} tets ({time.perf_counter() - t0:.1f} s)")
    tuned = autotune.tune_batch(ms_, scat, prec, cache=None, log=log,
                                tile_candidates=(336, 384, 512) if scat == nsa.ATOMIC else (128, 160, 256))
    log(f"autotuned: {({k: tuned[k] for k in ('tile_blocks', 'block_threads', 'grid_wgs', 'ms')})}")
    handles, b, vels, outs = autotune.build_batch(ms_, tuned["tile_blocks"], scat)
    nt = tuned["block_threads"] if scat == nsa.ATOMIC else 0
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        b.assemble(prec, grid_wgs=tuned["grid_wgs"], block_threads=nt)
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        b.assemble(prec, grid_wgs=tuned["grid_wgs"], block_threads=nt)
    cur = torch.cuda.current_stream()
    ms, per, wall = time_steps(graph.replay, args.steps, args.warmup, cur)
    ms_direct, _, _ = time_steps(lambda: b.assemble(prec, grid_wgs=tuned["grid_wgs"], block_threads=nt),
                                 args.steps, args.warmup, cur)
    log(f"batched: graph replay {ms:.4f} ms, direct launch {ms_direct:.4f} ms")

    def solo_all():
        for m, h, v, (vv, rr) in zip(ms_, handles, vels, outs):
            nsa.assemble(h, v, m.rho, m.mu, m.dt, precision=nsa.FP64, scatter=scat, kernel=nsa.KERNEL_TILED,
                         values=vv, rhs=rr)
    ms64, _, _ = time_steps(solo_all, args.steps, args.warmup, cur)
    log(f"64 plain FP64 launches: {ms64:.4f} ms")
    nbytes = sum(algorithmic_bytes(m.nelem, m.npoin, h.nnzb) for m, h in zip(ms_, handles))
    launch_ms = statistics.fmean(per)
    achieved = nbytes / (launch_ms / 1e3) / 1e9
    line = {
        "metric": "elements assembled/s", "value": nelem / (ms / 1e3), "unit": "elements/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if prec == nsa.MIXED else "f64", "data": "synthetic",
        "config": {"workload": "batch64: 64 jittered permuted cubes, n ~ U{8..48}, per-mesh rho/mu/dt",
                   "nelem": nelem, "nmesh": len(ms_), "precision": args.precision, "scatter": args.scatter,
                   "kernel": "tiled, one launch over all meshes, hipGraph-captured", "tile_blocks": tuned["tile_blocks"],
                   "block_threads": tuned["block_threads"], "grid_wgs": tuned["grid_wgs"]},
        "hbm_GBs": achieved,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": None, "kernel": "k_tiled_batch",
                     "algorithmic_bytes_per_launch": nbytes, "avg_launch_ms": launch_ms},
        "direct_launch_ms": ms_direct,
        "fp64_plain_launches": {"value": nelem / (ms64 / 1e3), "ms_per_step": ms64, "unit": "elements/s",
                                "launches": len(ms_), "dtype": "f64"},
        "autotune_trials": tuned["trials"],
    }
    print(json.dumps(line), flush=True)


def serve_run(executor, sizes, mean_elems, rate_ref, frac, seed, seconds, args):
    """One load level: Poisson arrivals at frac * rate_ref elements/s for `seconds` through a Server over
    `executor`; p50/p99 latency (arrival to results ready), throughput and the scheduler's figures."""
    import threading
    import torch
    from paper_2111_05651_amd import inputs
    from paper_2111_05651_amd.serve import DONE, Server
    lam = frac * rate_ref / mean_elems
    nreq = max(1, int(math.ceil(lam * seconds)))
    stream = inputs.served_requests(nreq, len(sizes), rate=lam, seed=seed)
    srv = Server(executor, budget_bytes=int(args.serve_budget_gb * 2 ** 30), timeout=60.0,
                 max_launch_elems=args.serve_launch_elems)
    executor.intervals.clear()
    reqs = []
    gc.collect()
    pauses, t_gc = [], [0.0]

    def on_gc(phase, info):
        if phase == "start":
            t_gc[0] = time.perf_counter()
        else:
            pauses.append(time.perf_counter() - t_gc[0])
    gc.callbacks.append(on_gc)
    if args.serve_gc == "paused":
        # the load generator's own policy: long-lived objects frozen, the cyclic collector off
        # during the arrival window (reference counting still frees everything)
        gc.freeze()
        gc.disable()
    mem0 = torch.cuda.memory_stats()
    with srv:
        start = time.perf_counter() + 0.05

        def client():
            for q in stream:
                wait = start + q["t"] - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
                reqs.append(srv.submit(q["mesh"], q["rho"], q["mu"], q["dt"], vel_seed=q["vel_seed"],
                                       arrival=start + q["t"]))
        th = threading.Thread(target=client)
        th.start()
        th.join()
        for r in reqs:
            r.wait(120.0)
    gc.enable()
    gc.unfreeze()
    gc.callbacks.remove(on_gc)
    mem1 = torch.cuda.memory_stats()
    st = srv.stats(t_start=start)
    ov = executor.device_overlap()
    done = [r for r in reqs if r.status == DONE]
    wait = [r.t_launch - r.t_arrival for r in done]
    service = [r.t_done - r.t_launch for r in done]

    def pct(x, q):
        return float(statistics.quantiles(x, n=100)[q - 1]) * 1e3 if len(x) > 1 else float("nan")
    nbytes = sum(algorithmic_bytes(*sizes[r.mesh_id]) for r in done)
    busy = ov.get("busy_ms", 0.0)
    out = {"load": frac, "rate_per_s": lam, "requests": nreq, "done": len(done),
           "p50_ms": st.get("p50", float("nan")) * 1e3, "p99_ms": st.get("p99", float("nan")) * 1e3,
           "mean_ms": st.get("mean", float("nan")) * 1e3, "elements_per_s": st.get("elements_per_s"),
           "offered_elements_per_s": lam * mean_elems, "launches": st["launches"],
           "mean_launch_requests": st["mean_launch_requests"], "max_inflight": st["max_inflight"],
           "peak_reserved_GB": st["peak_reserved_bytes"] / 1e9, "rejected": st["rejected"],
           "timeouts": st["timeout"], "device_busy_ms": busy,
           "device_overlapping_launches": ov.get("overlapping", 0),
           "hbm_GBs_while_busy": nbytes / (busy / 1e3) / 1e9 if busy > 0 else None,
           "wait_ms_p50_p99": [pct(wait, 50), pct(wait, 99)],
           "service_ms_p50_p99": [pct(service, 50), pct(service, 99)],
           "gc_pauses": len(pauses), "gc_max_pause_ms": max(pauses, default=0.0) * 1e3,
           "device_mallocs": mem1.get("num_device_alloc", 0) - mem0.get("num_device_alloc", 0),
           "device_frees": mem1.get("num_device_free", 0) - mem0.get("num_device_free", 0)}
    log(f"{'batched' if executor.mode == 'batched' else 'plain FP64'} at {frac:.0%}: "
        f"{json.dumps({k: (round(v, 4) if isinstance(v, float) else v) for k, v in out.items()})}")
    return out



def served_leg(args):
    """Compact served leg of the default run: `--served-leg-meshes` resident jittered cubes (tets
    log-uniform in [1e3, 5e6]), Poisson arrivals for `--served-leg-seconds` at `--served-leg-load` of
    the batched form's throughput over those same meshes (one launch over all of them, measured
    first), continuous batching in mixed precision; beside it plain FP64 launches served one at a
    time on the same resident meshes and the same arrival stream."""
    import torch
    from paper_2111_05651_amd import inputs, nsa
    from paper_2111_05651_amd.serve import GpuExecutor
    t0 = time.perf_counter()
    meshes = inputs.config_served(nmesh=args.served_leg_meshes)
    ex = GpuExecutor(meshes, scatter=nsa.ATOMIC, precision=nsa.MIXED, slots=args.serve_slots, trace=True)
    sizes = [(h.nelem, h.npoin, h.nnzb) for h in ex.meshes]
    del meshes
    log(f"served leg: {len(sizes)} resident meshes, {sum(x[0] for x in sizes)} tets, "
        f"{ex.resident_bytes / 1e9:.2f} GB ({time.perf_counter() - t0:.1f} s)")
    # reference rate: one batched mixed-precision launch over every resident mesh
    b = nsa.Batch(ex.meshes, nsa.ATOMIC)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(11)
    vels = [torch.rand((h.npoin, 3), dtype=torch.float64, device="cuda:0", generator=g) - 0.5 for h in ex.meshes]
    outs = b.alloc_outputs()
    b.set_inputs(vels, [1.0] * len(vels), [1e-3] * len(vels), [1e-2] * len(vels), outs)
    ms_b, _, _ = time_steps(lambda: b.assemble(nsa.MIXED), 10, 3, torch.cuda.current_stream())
    rate = sum(x[0] for x in sizes) / (ms_b / 1e3)
    log(f"served leg: batched launch over all meshes {ms_b:.3f} ms, {rate:.4g} elements/s")
    del b, vels, outs
    torch.cuda.empty_cache()
    mean_elems = sum(x[0] for x in sizes) / len(sizes)
    served = serve_run(ex, sizes, mean_elems, rate, args.served_leg_load, 60, args.served_leg_seconds, args)
    plain = GpuExecutor(None, scatter=nsa.ATOMIC, precision=nsa.FP64, mode="plain", trace=True, resident=ex.meshes)
    base = serve_run(plain, sizes, mean_elems, rate, args.served_leg_load, 60, args.served_leg_seconds, args)
    out = {"workload": f"{len(sizes)} resident jittered cubes, tets log-uniform in [1e3, 5e6], "
                       f"{sum(x[0] for x in sizes)} tets; Poisson arrivals for {args.served_leg_seconds:g} s at "
                       f"{args.served_leg_load:.0%} of the batched throughput over the same meshes",
           "reference_batched_ms": ms_b, "reference_batched_elements_per_s": rate,
           "continuous_batching": served, "plain_fp64_one_at_a_time": base}
    del ex, plain
    torch.cuda.empty_cache()
    return out


def run_serve(args):
    """Served load: 200 resident jittered cubes (tets log-uniform in [1e3, 5e6]), open-loop Poisson
    arrivals, one request = one assembly of a uniformly chosen mesh with a velocity drawn on the
    device from the request's seed and its own rho, mu, dt. The arrival rate is set to a fraction of
    the batched form's throughput on the 64-mesh batch (measured first, same run). The server runs
    continuous batching (mixed precision); beside it, plain FP64 launches served one at a time on
    the same meshes (resident with the FP64 kernel's own plan) and the same arrival stream."""
    import math
    import threading
    import torch
    from paper_2111_05651_amd import inputs, nsa
    from paper_2111_05651_amd.serve import DONE, GpuExecutor, Server, default_tile_blocks
    scat = {"atomic": nsa.ATOMIC, "colour": nsa.COLOUR}[args.scatter]
    prec = {"mixed": nsa.MIXED, "fp64": nsa.FP64}[args.precision]
    # reference rate: the 64-mesh batch, one launch, with the plan the served meshes use
    t0 = time.perf_counter()
    c4 = inputs.config_batch()
    tb = default_tile_blocks(scat, prec)
    hs = [nsa.Mesh.from_inputs(m, tile_blocks=tb if scat == nsa.ATOMIC else 0,
                               tile_blocks_colour=0 if scat == nsa.ATOMIC else tb).upload() for m in c4]
    b = nsa.Batch(hs, scat)
    vels = [torch.from_numpy(m.velocity).cuda() for m in c4]
    outs = b.alloc_outputs()
    b.set_inputs(vels, [m.rho for m in c4], [m.mu for m in c4], [m.dt for m in c4], outs)
    ms4, _, _ = time_steps(lambda: b.assemble(prec), 10, 3, torch.cuda.current_stream())
    rate4 = sum(m.nelem for m in c4) / (ms4 / 1e3)
    log(f"64-mesh batch: {ms4:.3f} ms, {rate4:.4g} elements/s ({time.perf_counter() - t0:.1f} s)")
    del c4, hs, b, vels, outs
    torch.cuda.empty_cache()
    # resident meshes
    t0 = time.perf_counter()
    meshes = inputs.config_served(nmesh=args.serve_meshes)
    log(f"{len(meshes)} served meshes generated, {sum(m.nelem for m in meshes)} tets "
        f"({time.perf_counter() - t0:.1f} s)")
    ex = GpuExecutor(meshes, scatter=scat, precision=prec, slots=args.serve_slots, trace=True, log=log)
    sizes = [(h.nelem, h.npoin, h.nnzb) for h in ex.meshes]
    log(f"resident: {ex.resident_bytes / 1e9:.2f} GB ({time.perf_counter() - t0:.1f} s)")
    # the plain FP64 comparison keeps meshes of its own when the served plan is not the FP64 kernel's
    if default_tile_blocks(scat, prec) == default_tile_blocks(scat, nsa.FP64, "plain"):
        plain = GpuExecutor(None, scatter=scat, precision=nsa.FP64, mode="plain", trace=True, resident=ex.meshes)
    else:
        plain = GpuExecutor(meshes, scatter=scat, precision=nsa.FP64, mode="plain", trace=True, log=log)
        log(f"plain comparison: own resident meshes, {plain.resident_bytes / 1e9:.2f} GB "
            f"({time.perf_counter() - t0:.1f} s)")
    del meshes
    mean_elems = sum(x[0] for x in sizes) / len(sizes)

    loads = [float(x) for x in args.serve_loads.split(",")]
    served = [serve_run(ex, sizes, mean_elems, rate4, f, 60 + k, args.serve_seconds, args) for k, f in enumerate(loads)]
    base = [serve_run(plain, sizes, mean_elems, rate4, f, 60 + k, args.serve_seconds, args) for k, f in enumerate(loads)]
    head = served[-1]
    hbm = head["hbm_GBs_while_busy"]
    line = {
        "metric": "elements assembled/s under served load (p50/p99 latency)", "value": head["elements_per_s"],
        "unit": "elements/s", "n_gpus": 1, "steps": head["requests"], "warmup": 0, "ms_per_step": head["mean_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == nsa.MIXED else "f64", "data": "synthetic",
        "config": {"workload": f"served: {len(sizes)} resident jittered cubes, tets log-uniform in [1e3, 5e6]; "
                               f"Poisson arrivals at {head['load']:.0%} of the 64-mesh batched throughput",
                   "nmesh": len(sizes), "resident_elements": int(sum(x[0] for x in sizes)),
                   "budget_GB": args.serve_budget_gb, "slots": args.serve_slots, "scatter": args.scatter,
                   "precision": args.precision, "reference_batched_elements_per_s": rate4,
                   "seconds_of_arrivals": args.serve_seconds, "launch_elems_cap": args.serve_launch_elems,
                   "python_gc": args.serve_gc},
        "latency_ms": {"p50": head["p50_ms"], "p99": head["p99_ms"]},
        "roofline": {"bound": "hbm", "achieved": hbm, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": hbm / PEAK_HBM_GBS if hbm else None, "traffic": None, "kernel": "k_tiled_batch",
                     "note": "algorithmic bytes of the completed requests over the device-busy time"},
        "cpu_baseline": None,
        "loads": served,
        "plain_fp64_one_at_a_time": base,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cube128",
                    choices=["cube128", "cube64", "cube8", "batch64", "serve", "quad2048", "cylinder2d", "venturi2d"])
    ap.add_argument("--precision", default=None, choices=["mixed", "fp64"],
                    help="default: fp64 for the single-mesh workloads (mixed timed beside), mixed for batch64 "
                         "and serve (compared against plain FP64 launches)")
    ap.add_argument("--scatter", default="atomic", choices=["atomic", "colour"])
    ap.add_argument("--kernel", default="tiled", choices=["tiled", "direct", "auto", "gather"])
    ap.add_argument("--tile-blocks-gather", type=int, default=512, help="blocks per tile of the gather plan")
    ap.add_argument("--path", default="matrix", choices=["matrix", "residual"],
                    help="matrix: block-CSR values + RHS; residual: the explicit-residual outputs (no matrix)")
    ap.add_argument("--tile-rows-residual", type=int, default=256, help="rows per tile of the residual plan")
    ap.add_argument("--residual-geometry", default="formed", choices=["formed", "precomputed"],
                    help="residual path: element geometry formed from the coordinates in the kernel, or read "
                         "from a per-element table stored at upload (nsa_mesh_set_residual_geometry)")
    ap.add_argument("--block-threads", type=int, default=0, help="workgroup size override (0 = the plan's)")
    ap.add_argument("--tile-blocks", type=int, default=512, help="tile size of the atomic-mode plan")
    ap.add_argument("--tile-threads", type=int, default=0, help="workgroup size of the atomic-mode plan (0 = default)")
    ap.add_argument("--tile-blocks-colour", type=int, default=128, help="tile size of the colour-mode plan")
    ap.add_argument("--no-beside", action="store_true",
                    help="skip timing the other precision beside (mixed beside FP64, or FP64 beside mixed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true", help="skip the HBM bandwidth probes")
    ap.add_argument("--series-seconds", type=float, default=1.0,
                    help="length of the per-launch timing series after the K timed steps")
    ap.add_argument("--no-served-leg", dest="served_leg", action="store_false",
                    help="skip the compact served leg of the default cube128 run")
    ap.add_argument("--served-leg-meshes", type=int, default=40)
    ap.add_argument("--served-leg-seconds", type=float, default=2.0)
    ap.add_argument("--served-leg-load", type=float, default=0.8)
    ap.add_argument("--cpu-sample", type=int, default=0, help="elements for the CPU baseline (0 = the whole mesh)")
    ap.add_argument("--serve-meshes", type=int, default=200)
    ap.add_argument("--serve-seconds", type=float, default=4.0, help="seconds of arrivals per load level")
    ap.add_argument("--serve-loads", default="0.5,0.8", help="arrival rates as fractions of the batched rate")
    ap.add_argument("--serve-slots", type=int, default=3)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-launch-elems", type=int, default=4_000_000, help="element cap of one served launch")
    ap.add_argument("--serve-gc", default="paused", choices=["paused", "default"],
                    help="Python's cyclic collector during the arrival window")
    ap.add_argument("--copy-probe", type=float, default=0.0, metavar="GIB",
                    help="instead: time a plain device copy of this many GiB (counter calibration)")
    args = ap.parse_args()
    if args.precision is None:
        args.precision = "mixed" if args.workload in ("batch64", "serve") else "fp64"
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU design is "
              "documented but not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2111_05651_amd import nsa
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    nsa.load()
    if args.copy_probe > 0:
        n = int(args.copy_probe * 2 ** 30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        ms, per, _ = time_steps(lambda: dst.copy_(src), args.steps, args.warmup, torch.cuda.current_stream())
        print(json.dumps({"copy_probe_bytes_read": 8 * n, "copy_probe_bytes_written": 8 * n, "ms": ms,
                          "GBs_read_plus_write": 16 * n / (ms / 1e3) / 1e9}), flush=True)
        return
    if args.workload == "batch64":
        return run_batch(args)
    if args.workload == "serve":
        return run_serve(args)
    prec = {"mixed": nsa.MIXED, "fp64": nsa.FP64}[args.precision]
    if args.workload in ("quad2048", "cylinder2d", "venturi2d"):
        return run_quads(args, prec)
    scat = {"atomic": nsa.ATOMIC, "colour": nsa.COLOUR}[args.scatter]
    kern = {"tiled": nsa.KERNEL_TILED, "direct": nsa.KERNEL_DIRECT, "auto": nsa.KERNEL_AUTO,
            "gather": nsa.KERNEL_GATHER}[args.kernel]

    probe = None
    if not args.no_probe:
        probe = bandwidth_probes()
        log(f"bandwidth probes: read {probe['read_GBs']:.0f} GB/s, write {probe['write_GBs']:.0f} GB/s, "
            f"copy {probe['copy_GBs']:.0f} GB/s (read + write)")
    t0 = time.perf_counter()
    m = make_workload(args.workload)
    log(f"workload {args.workload}: {m.nelem} tets, {m.npoin} nodes ({time.perf_counter() - t0:.1f} s)")
    if args.path == "residual":
        return run_residual(args, m, prec)
    gather = kern == nsa.KERNEL_GATHER
    # set-up, once per mesh and outside the timed region: the pattern, element-to-block map and global
    # colouring (nsa_mesh_create), the tile plans (built on first need), the device upload
    t0 = time.perf_counter()
    mesh = nsa.Mesh.from_inputs(m, tile_blocks=0 if gather else args.tile_blocks,
                                tile_blocks_colour=0 if gather else args.tile_blocks_colour,
                                tile_blocks_gather=args.tile_blocks_gather if gather else 0,
                                keep_direct=kern in (nsa.KERNEL_DIRECT, nsa.KERNEL_AUTO),
                                tile_threads=args.tile_threads or None)
    info = mesh.info
    t2 = time.perf_counter()
    mesh.upload("cuda:0")
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    setup = {"mesh_and_plans_s": t2 - t0, "upload_s": t3 - t2, "workspace_GB": info.ws_bytes / 1e9,
             "host_threads": os.cpu_count(),
             "note": "once per mesh, untimed in the throughput figures: pattern, element-to-block map, global "
                     "colouring and the tile plans (host, multithreaded); device upload"}
    log(f"set-up: mesh and plans {t2 - t0:.2f} s, upload {t3 - t2:.2f} s")
    info = mesh.info
    if gather:
        log(f"mesh registered: nnzb={info.nnzb} gather tiles={info.gather_ntiles} records/nelem="
            f"{info.gather_records / max(m.nelem, 1):.2f} lds={list(info.gather_lds_bytes)}")
    else:
        log(f"mesh registered: nnzb={info.nnzb} ntiles={info.ntiles[scat]} runs={info.tile_runs[scat]} "
            f"(pairs per run {4 * m.nelem / max(info.tile_runs[scat], 1):.2f}) max runs per tile "
            f"{info.tile_max_runs[scat]} lds={info.tile_lds_bytes[scat]}")
    vel = torch.from_numpy(m.velocity).to("cuda:0")
    values, rhs = mesh.alloc_outputs("cuda:0")
    stream = torch.cuda.current_stream()

    def step(p=prec):
        nsa.assemble(mesh, vel, m.rho, m.mu, m.dt, precision=p, scatter=scat, kernel=kern, values=values,
                     rhs=rhs, stream=stream, block_threads=args.block_threads)

    # the per-launch series (at least --series-seconds of launches) comes first, then the warmup and
    # the K timed steps of the contract
    est, _, _ = time_steps(step, 3, 1, stream)
    series = timing_series(step, stream, est, seconds=args.series_seconds)
    log(f"timing series: {series['launches']} launches over {series['total_s']:.2f} s, median "
        f"{series['median_ms']:.4f} ms, min {series['min_ms']:.4f} ms")
    ms, per, wall = time_steps(step, args.steps, args.warmup, stream)
    log(f"timed {args.steps} steps: {ms:.4f} ms/step (wall {wall:.3f} s)")
    beside = None
    if not args.no_beside and kern != nsa.KERNEL_DIRECT:
        other = nsa.FP64 if prec == nsa.MIXED else nsa.MIXED
        first_v, first_r = values.clone(), rhs.clone()
        ms_o, _, _ = time_steps(lambda: step(other), args.steps, args.warmup, stream)
        series_o = timing_series(lambda: step(other), stream, ms_o, seconds=args.series_seconds)
        # block-class error of the mixed result against the FP64 one (the FP64 kernel meets the
        # oracle to 1e-12 in the parity tests)
        if other == nsa.MIXED:
            diff = class_diff(values, rhs, first_v, first_r)
        else:
            diff = class_diff(first_v, first_r, values, rhs)
        del first_v, first_r
        # the library's own report (nsa_options.err_out): sampled element blocks, mixed against FP64
        err = torch.zeros(12, dtype=torch.float64, device="cuda:0")
        nsa.assemble(mesh, vel, m.rho, m.mu, m.dt, precision=nsa.MIXED, scatter=scat, kernel=kern, values=values,
                     rhs=rhs, stream=stream, err_out=err)
        lib_err = nsa.error_report(err)
        beside = {"precision": "mixed" if other == nsa.MIXED else "fp64", "value": m.nelem / (ms_o / 1e3),
                  "ms_per_step": ms_o, "unit": "elements/s", "dtype": "f32+f64" if other == nsa.MIXED else "f64",
                  "same_gpu": True, "timing": series_o, "mixed_vs_fp64_class_error": diff,
                  "library_error_report": lib_err}
        log(f"{beside['precision']} kernel beside it: {ms_o:.4f} ms/step (series median {series_o['median_ms']:.4f}); "
            f"mixed vs FP64 class errors {diff}")

    nbytes = algorithmic_bytes(m.nelem, m.npoin, info.nnzb)
    launch_ms = series["mean_ms"]
    achieved = nbytes / (launch_ms / 1e3) / 1e9
    rt = "float" if prec == nsa.MIXED else "double"
    if gather:
        nthreads = args.block_threads or info.gather_threads
        kname = f"k_gather<{rt},{nthreads}>"
        tb = args.tile_blocks_gather
    else:
        nthreads = args.block_threads or info.tile_threads[scat]
        kname = f"k_tiled<{rt},{nthreads}>"
        tb = args.tile_blocks if scat == nsa.ATOMIC else args.tile_blocks_colour
    key = f"{kname}@{args.workload}/tile{tb}"
    traffic = traffic_for(key, nbytes) if kern in (nsa.KERNEL_TILED, nsa.KERNEL_GATHER) else None
    roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "kernel": kname,
            "algorithmic_bytes_per_launch": nbytes, "avg_launch_ms": launch_ms,
            "launch_ms_basis": f"mean of the {series['launches']} launches of the timing series"}
    if probe:
        roof.update({"probe_read_GBs": probe["read_GBs"], "probe_write_GBs": probe["write_GBs"],
                     "probe_copy_GBs": probe["copy_GBs"], "frac_vs_probe_write": achieved / probe["write_GBs"],
                     "frac_vs_probe_copy": achieved / probe["copy_GBs"]})
    line = {
        "metric": "elements assembled/s",
        "value": m.nelem / (ms / 1e3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == nsa.MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {m.name}", "nelem": m.nelem, "npoin": m.npoin,
                   "nnzb": info.nnzb, "precision": args.precision, "scatter": args.scatter,
                   "kernel": args.kernel, "tile_blocks": tb, "tile_threads": nthreads, "rho": m.rho, "mu": m.mu,
                   "dt": m.dt},
        "hbm_GBs": achieved,
        "timing": series,
        "roofline": roof,
        "beside": beside,
        "setup": setup,
    }
    del values, rhs, vel, mesh
    torch.cuda.empty_cache()
    if args.served_leg and args.workload == "cube128":
        line["served"] = served_leg(args)
        head = line["served"]["continuous_batching"]
        line["latency_ms"] = {"p50": head["p50_ms"], "p99": head["p99_ms"], "load": head["load"],
                              "workload": line["served"]["workload"]}
    if not args.no_cpu_baseline:
        ns = min(args.cpu_sample, m.nelem) if args.cpu_sample > 0 else m.nelem
        log(f"cpu baseline: oracle on {ns} elements ...")
        line["cpu_baseline"] = cpu_baseline(m, ns)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
