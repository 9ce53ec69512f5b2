"""Host autotuner of the launch shapes, through the C ABI only.

The knobs are the blocks per launch of the DG quadrilateral cell pass
(cvw_mesh_set_grid: each block walks a contiguous run of 16- or 64-cell tiles)
and of the batched work-list kernels (cvw_batch_set_grid).  Results do not
depend on them; the tuner checks that every candidate reproduces the first
candidate's output bit for bit before it keeps a timing.

The choice is cached in a JSON file keyed by (device architecture, degree,
space, nodes per cell, flux (which also fixes the number of variables), cell
count), so a later run with the same workload applies it without timing
(`params` is the struct from cvw.make_params):

    best = tune_mesh(mesh, params, u, cand, ws)        # times, caches, applies
    apply_cached(mesh, params)                          # applies a cached choice
    best = tune_batch(batch, ws)
"""
from __future__ import annotations

import json
import os

from . import cvw

MESH_CANDIDATES = (1024, 2048, 4096, 8192, 16384, 32768, 0)
BATCH_CANDIDATES = (256, 512, 1024, 2048, 4096, 0)


def cache_path() -> str:
    return os.environ.get("CVW_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "cvw", "tune.json"))


def arch() -> str:
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return str(getattr(props, "gcnArchName", props.name)).split(":")[0]


def mesh_key(mesh, params) -> str:
    info = mesh.info
    flux = int(params.flux)
    n_var = mesh.n_var(flux)
    return (f"{arch()}|mesh|deg{mesh.degree}|space{mesh.space}|nloc{info['n_loc']}|flux{flux}|nvar{n_var}"
            f"|cells{info['n_cells']}")


def batch_key(batch) -> str:
    return f"{arch()}|batch|{batch.signature()}"


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        try:
            data = json.load(f)
        except json.JSONDecodeError:
            return {}
    return data if isinstance(data, dict) else {}


def store(key: str, entry: dict, path: str | None = None) -> None:
    path = path or cache_path()
    data = load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time(torch, fn, reps: int) -> float:
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)                   # the events exist before the timing
    t1.record(stream)
    fn()
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(reps):
        fn()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / reps


def pick(timings: dict) -> int:
    """Fastest candidate; ties go to the earlier candidate in the list."""
    best, best_t = None, None
    for c, t in timings.items():
        if best_t is None or t < best_t:
            best, best_t = c, t
    return best


def tune_mesh(mesh, params, u, cand, ws, candidates=MESH_CANDIDATES, reps: int = 10,
              path: str | None = None) -> int:
    """Time one Runge-Kutta stage (cvw_rk_stage from u) for each candidate grid,
    check the outputs are bitwise equal, keep and apply the fastest."""
    import torch
    out = torch.empty_like(u)
    ref = None
    timings = {}
    for c in candidates:
        mesh.set_grid(c)
        cvw.rk_stage(mesh, params, u, cand, u, out, 1e-6, 0.75, 0.25, ws)
        torch.cuda.synchronize()
        if ref is None:
            ref = out.clone()
        elif not torch.equal(out, ref):
            raise RuntimeError(f"launch shape {c} changed the result")
        timings[c] = _time(torch, lambda: cvw.rk_stage(mesh, params, u, cand, u, out, 1e-6, 0.75, 0.25, ws), reps)
    best = pick(timings)
    mesh.set_grid(best)
    store(mesh_key(mesh, params), {"grid": best, "ms": timings[best], "timings_ms": {str(k): v for k, v in
                                                                                   timings.items()}}, path)
    return best


def apply_cached(mesh, params, path: str | None = None):
    """Apply a cached grid for this mesh and flux; returns it, or None if none is cached."""
    entry = load_cache(path).get(mesh_key(mesh, params))
    if entry is None:
        return None
    mesh.set_grid(int(entry["grid"]))
    return int(entry["grid"])


def tune_batch(batch, ws, candidates=BATCH_CANDIDATES, reps: int = 3, path: str | None = None) -> int:
    """Time one step of every instance for each candidate grid (eager launches,
    on copies of the states, restored afterwards), keep and apply the fastest."""
    import torch
    saved = [u.clone() for u in batch.states]
    timings = {}
    ref = None
    for c in candidates:
        batch.set_grid(c)
        for u, s in zip(batch.states, saved):
            u.copy_(s)
        batch.step(1, ws, use_graph=False)
        torch.cuda.synchronize()
        res = [u.clone() for u in batch.states]
        if ref is None:
            ref = res
        elif not all(torch.equal(x, y) for x, y in zip(res, ref)):
            raise RuntimeError(f"launch shape {c} changed the result")

        def one():
            batch.step(1, ws, use_graph=False)
        timings[c] = _time(torch, one, reps)
    for u, s in zip(batch.states, saved):
        u.copy_(s)
    best = pick(timings)
    batch.set_grid(best)
    store(batch_key(batch), {"grid": best, "ms": timings[best],
                             "timings_ms": {str(k): v for k, v in timings.items()}}, path)
    return best
