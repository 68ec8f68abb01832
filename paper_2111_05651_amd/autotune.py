"""Autotuner for the tiled kernel: picks the tile size (blocks per LDS tile), the workgroup size and
the grid (one workgroup per tile, or a persistent grid of a few workgroups per CU) for a batch of
meshes by timing the candidates on the device.

Every candidate runs the library's own kernel through the C-ABI on the real inputs; the search
rebuilds the tile plans once per tile size (host work) and times launch parameters on each. The
choice is cached in a JSON file keyed by the batch's shape, so a served process tunes once.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

from . import nsa

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "nsa_autotune.json")


def signature(meshes, scatter, precision) -> str:
    """Key of a batch: library version (plans change with it), sizes of its meshes, mode and precision."""
    h = hashlib.sha256()
    h.update(f"v{nsa.load().nsa_version()};".encode())
    for m in meshes:
        h.update(f"{m.nelem}:{m.npoin};".encode())
    h.update(f"s{scatter}p{precision}".encode())
    return h.hexdigest()[:24]


def _time(fn, reps, warmup=2):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def build_batch(meshes, tile_blocks, scatter, device="cuda"):
    """nsa meshes (tile plan of `scatter` at `tile_blocks`, the other mode's plan dropped), their
    batch, velocities and outputs, ready to launch."""
    import torch
    other = nsa.COLOUR if scatter == nsa.ATOMIC else nsa.ATOMIC
    handles = []
    for m in meshes:
        h = nsa.Mesh(m.lnods, m.coord)
        h.set_tiling(tile_blocks, scatter)
        h.set_tiling(0, other)
        handles.append(h.upload(device))
    b = nsa.Batch(handles, scatter, device=device)
    vels = [torch.from_numpy(m.velocity).to(device) for m in meshes]
    outs = b.alloc_outputs(device)
    b.set_inputs(vels, [m.rho for m in meshes], [m.mu for m in meshes], [m.dt for m in meshes], outs)
    return handles, b, vels, outs


def tune_batch(meshes, scatter=nsa.ATOMIC, precision=nsa.MIXED, tile_candidates=(336, 384, 512),
               thread_candidates=(128, 256), grid_per_cu=(0, 1, 2), reps=5, cache: str | None = DEFAULT_CACHE,
               log=None) -> dict:
    """Best (tile_blocks, block_threads, grid_wgs) for this batch; cached by signature(). A grid
    candidate g > 0 is a persistent grid of g workgroups per CU (4 g for the one-wavefront plan);
    g = 0 is one workgroup per tile (grid_wgs 0)."""
    import torch
    key = signature(meshes, scatter, precision)
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                hit = json.load(f).get(key)
            if hit:
                return dict(hit, cached=True)
        except (OSError, ValueError):
            pass
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    threads = thread_candidates if scatter == nsa.ATOMIC else (64,)
    trials = []
    for tb in tile_candidates:
        t0 = time.perf_counter()
        handles, b, vels, outs = build_batch(meshes, tb, scatter)
        plan_s = time.perf_counter() - t0
        for nt in threads:
            for g in grid_per_cu:
                grid = g * ncu * (4 if nt == 64 else 1)
                ms = _time(lambda: b.assemble(precision, grid_wgs=grid, block_threads=nt if nt != 64 else 0), reps)
                trials.append(dict(tile_blocks=tb, block_threads=nt, grid_wgs=grid, ms=ms))
                if log:
                    log(f"autotune tile={tb} threads={nt} grid={grid or 'one per tile'}: {ms:.4f} ms "
                        f"(plan {plan_s:.1f} s)")
        del handles, b, vels, outs
        torch.cuda.empty_cache()
    best = min(trials, key=lambda t: t["ms"])
    out = dict(best, key=key, trials=trials, cached=False)
    if cache:
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            data = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    data = json.load(f)
            data[key] = {k: v for k, v in out.items() if k != "cached"}
            with open(cache, "w") as f:
                json.dump(data, f, indent=1)
        except (OSError, ValueError):
            pass
    return out
