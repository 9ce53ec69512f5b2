"""Benchmark of the stabilised-residual hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (default): 2D Euler (gas gamma 1.4), DG Q3 on a periodic 1024 x 1024
grid of unit-square cells (1,048,576 cells, 16,777,216 nodes, 67,108,864
DOFs), float32 state, plain cell-vertex HWENO sensor with shock-capturing
quadrature.  Input: the seeded four-quadrant data (rho, p, velocities drawn
from the stated ranges) with its quadrant interfaces smoothed over about half
a cell, so that the sensor and the shock-capturing weights are active along
the interfaces.  Everything is resident in HBM before timing starts.

One step = one SSP-RK3 time step = three stages, each stage = the fused
sensor pass (vertex HWENO candidates and the cell sensor gamma_e in one
kernel) plus the cell pass (viscosity, shock-capturing weights, volume and
interface terms, mass inverse, stage update).  value = stabilised-residual DOF updates per second
= 3 * n_dof * n_var * K / (time of K steps).

The roofline object describes the dominant kernel (the cell pass,
dgq_eval_kernel, with gamma supplied by the sensor pass): its launches are
bracketed by HIP events on the stream they run on, inside the timed region.
It is bound by vector-ALU instruction issue ("alu": algorithmic flops per
launch against the fp32 vector peak; valu_issue relates the counted VALU wave
instructions per launch, profiles/valu_dgq_eval_config4.json, to the issue
roof; hbm_view gives its compulsory bytes against HBM).  sensor_pass gives the
fused sensor pass (one launch per stage) against HBM with its compulsory
bytes: read the sensor field once, write gamma.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SMOOTH_K = 400.0      # sharpness of the quadrant interfaces at n = 1024 (~0.4 cell wide)


def euler_config4_state(n: int, ref_nodes: np.ndarray, smooth_k: float):
    import synth
    h = 1.0 / n
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    xc = (ii.ravel() + 0.5) * h
    yc = (jj.ravel() + 0.5) * h
    X = xc[:, None] + 0.5 * h * ref_nodes[None, :, 0]
    Y = yc[:, None] + 0.5 * h * ref_nodes[None, :, 1]
    return np.asarray(synth.euler_state_config4(X, Y, smooth_k=smooth_k), np.float32)


def gauss_nodes_2d(p: int):
    """Reference node coordinates of the Gauss-point Lagrange basis (input sampling only)."""
    x, _ = np.polynomial.legendre.leggauss(p + 1)
    X, Y = np.meshgrid(x, x, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def kernel_source_hash() -> str:
    """Hash of the sources of the DG quadrilateral sensor and cell kernels;
    counter figures are valid only for the kernels they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("cvw_dgquad.hip", "cvw_dgsensor.hip", "cvw_device.h", "cvw_internal.h", "cvw_dgq_common.h"):
        with open(os.path.join(ROOT, "paper_2601_16911_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _measured(name: str, key: str):
    """A counter figure from profiles/<name>.json, or None when the kernels
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get(key)


def measured_traffic(key: str = "bytes_per_launch"):
    """HBM bytes per stage-mode launch of the cell pass (or, with
    key="sensor_pass_bytes_per_launch", of the fused sensor pass) from the
    calibrated FETCH_SIZE / WRITE_SIZE counter runs."""
    return _measured("traffic_dgq_eval_config4", key)


def measured_valu(key: str = "valu_instr_per_launch"):
    """VALU wave instructions per stage-mode launch of the cell pass (or of
    the sensor pass, key="sensor_pass_valu_instr_per_launch"), SQ counters."""
    return _measured("valu_dgq_eval_config4", key)


def host_cpu():
    """(logical CPUs visible, CPU model) of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 1, model


# VALU issue roof: 256 CUs x 4 SIMDs, one wave64 instruction per 4 cycles of
# a 16-lane SIMD, 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
# published fp32 vector peak (it counts packed fp32, which this build does not
# issue: ordinary fp32 code tops out at half of it)
FP32_VECTOR_PEAK_TFLOPS = 157.3


def cell_pass_flops(p: int, nv: int) -> float:
    """Algorithmic flops per cell of one DG quadrilateral cell pass (Euler,
    collocated Gauss rule, n = (p+1)^2 points, 4 (p+1) face points): the
    arithmetic the discretisation needs, counted once (an FMA is 2 flops)."""
    n1 = p + 1
    n = n1 * n1
    nf = 4 * n1
    grad = nv * n * 2 * n1 * 2                 # du/dxi, du/deta at every point (sum factorised)
    flux = 18 * n                              # Euler flux at the points
    speed = 6 * n + n                          # |v| + c and the cell maximum
    stab = nv * n * 2 * 3                      # W (nu (1 - gamma) alpha grad u - f)
    test = nv * n * 2 * n1 * 2                 # contraction with the test-function gradients
    traces = 2 * nv * nf * n1 * 2              # own and neighbour traces at the face points
    hll = 72 * nf + nv * nf                    # HLL flux with Davis speeds, face weight
    lift = nv * nf * n1 * 2                    # face flux back to the nodes of its normal line
    update = 5 * nv * n                        # mass inverse and the Shu-Osher update
    return float(grad + flux + speed + stab + test + traces + hll + lift + update)


def _oracle_residuals(args):
    """One worker of the CPU baseline: float64 oracle residuals of a periodic
    n x n DG Q3 Euler sub-problem for about `seconds`; returns (DOFs, calls, s)."""
    n, seconds = args
    import synth
    from oracle import build_space, nodal_interpolate, residual
    prm = synth.Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0))
    sp = build_space(synth.quad_mesh(n, n), 3, 1, 4)
    U = nodal_interpolate(sp, [(lambda c: (lambda x: synth.euler_state_config4(
        x[..., 0], x[..., 1], smooth_k=SMOOTH_K * n / 1024)[c]))(c) for c in range(4)])
    t0 = time.perf_counter()
    calls = 0
    while True:
        residual(sp, U, prm)
        calls += 1
        if time.perf_counter() - t0 > seconds:
            break
    return U.size, calls, time.perf_counter() - t0


def cpu_baseline(seconds: float = 8.0, max_workers: int = 16):
    """The float64 oracle timed on a bounded sample of the same workload (the
    stabilised residual on periodic 64 x 64 DG Q3 Euler sub-problems of the
    same recipe): one process on one core, then one process per core on all
    the host cores the GPU's share allows (at most max_workers), each with one
    BLAS thread; value = aggregate DOF-updates/s of the all-cores leg."""
    import multiprocessing as mp
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    ncpu, model = host_cpu()
    workers = max(1, min(ncpu, max_workers))
    ctx = mp.get_context("spawn")
    with ctx.Pool(1) as pool:
        d1, c1, t1 = pool.map(_oracle_residuals, [(64, seconds)])[0]
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_residuals, [(64, seconds)] * workers)
    agg = sum(d * c / t for d, c, t in res)
    return {"value": agg, "unit": "DOF-updates/s", "cores": workers, "kind": "oracle",
            "one_core": d1 * c1 / t1, "host_logical_cpus": ncpu, "cpu_model": model,
            "sample": f"float64 oracle residuals of periodic 64x64 DG Q3 Euler meshes ({d1} DOFs each) with the "
                      f"same state recipe, about {seconds:.0f} s per process: one process ({c1} calls), then "
                      f"{workers} processes with one BLAS thread each ({sum(c for _, c, _ in res)} calls)"}


class HipEvents:
    """Timing events of the HIP runtime in use (the one torch loaded: same
    soname), created with hipEventDisableSystemFence: a record then writes its
    timestamp without the system-scope cache write-back and invalidation that
    a default event performs, which would otherwise sit between the timed
    launches.  Elapsed times are read only after a device synchronisation."""
    DISABLE_SYSTEM_FENCE = 0x20000000

    def __init__(self):
        import ctypes
        self.C = ctypes
        self.lib = ctypes.CDLL("libamdhip64.so.7")
        self.lib.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        self.lib.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.lib.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self):
        ev = self.C.c_void_p()
        rc = self.lib.hipEventCreateWithFlags(self.C.byref(ev), self.DISABLE_SYSTEM_FENCE)
        if rc != 0:
            raise RuntimeError(f"hipEventCreateWithFlags failed ({rc})")
        return ev

    def record(self, ev, stream):
        rc = self.lib.hipEventRecord(ev, self.C.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"hipEventRecord failed ({rc})")

    def elapsed_ms(self, a, b) -> float:
        ms = self.C.c_float()
        rc = self.lib.hipEventElapsedTime(self.C.byref(ms), a, b)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return ms.value

    def destroy(self, *evs):
        for ev in evs:
            self.lib.hipEventDestroy(ev)


def _timed(torch, stream, fn, reps: int, trials: int = 3) -> float:
    """Seconds per call of fn() on `stream` (HIP events), after one warm-up
    call: the median over `trials` runs of `reps` calls, so that one host
    stall between launches (the GPU idles, the events still count it) does
    not set the figure."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)                   # created before the timing
    e1.record(stream)
    fn()
    torch.cuda.synchronize()
    per = []
    for _ in range(trials):
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        per.append(e0.elapsed_time(e1) / 1e3 / reps)
    return sorted(per)[len(per) // 2]


def bench_learned(torch, cvw, gm, prm, U, dt, steps: int):
    """The learned sensor on the benchmark workload: a network trained for a
    few seconds by the library's kernels on snapshots of a plain-sensor run
    of the same problem at 256 x 256, then the sensor alone (cells/s) and the
    full SSP-RK3 step (DOF-updates/s), plain vs learned."""
    import synth
    from paper_2601_16911_amd import learned
    stream = torch.cuda.current_stream()
    n_small = 256
    mesh_s = synth.quad_mesh(n_small, n_small)
    gs = cvw.Mesh(mesh_s, 3, cvw.DG)
    Us = torch.from_numpy(euler_config4_state(n_small, gauss_nodes_2d(3), SMOOTH_K * n_small / 1024).reshape(-1)).cuda()
    sref_s = learned.sigma_reference(gs, cvw.make_params(prm), Us)
    F, G = learned.collect(gs, prm, Us, dt * 1024 / n_small, 8, 4, sref_s)
    net = cvw.Mlp(learned.init_params(4))
    t0 = time.perf_counter()
    learned.train(net, F, G, epochs=20, batch=4096, lr=1e-3, seed=4)
    t_train = time.perf_counter() - t0
    E = gm.info["n_cells"]
    sref = learned.sigma_reference(gm, cvw.make_params(prm), U)
    prm_l = synth.Params(**{**prm.__dict__, "sensor": cvw.LEARNED})
    cpp = cvw.make_params(prm)
    cpl = cvw.make_params(prm_l, mlp=net, sigma_ref=sref)
    wsp = cvw.alloc_workspace(gm, cpp, 1)
    wsl = cvw.alloc_workspace(gm, cpl, 1)
    gam = torch.empty(E, dtype=torch.float32, device="cuda")
    t_sp = _timed(torch, stream, lambda: cvw.sensor(gm, cpp, U, gam, None, wsp), 10)
    t_sl = _timed(torch, stream, lambda: cvw.sensor(gm, cpl, U, gam, None, wsl), 10)
    ndof = U.numel()
    u1 = U.clone()
    t_step_p = _timed(torch, stream, lambda: cvw.step(gm, cpp, u1, dt, steps, wsp), 1) / steps
    u2 = U.clone()
    t_step_l = _timed(torch, stream, lambda: cvw.step(gm, cpl, u2, dt, steps, wsl), 1) / steps
    feat = torch.empty((E, 48), dtype=torch.int16, device="cuda")
    cand = torch.empty((gm.info["n_vertices"], gm.info["n_k"]), dtype=torch.float32, device="cuda")
    cvw.vertex_candidates(gm, cpl, U, cand, wsl)
    t_feat = _timed(torch, stream, lambda: cvw.mlp_features(gm, cpl, U, cand, feat), 10)
    t_inf = _timed(torch, stream, lambda: net.infer(feat, gam), 10)
    aud = cvw.learned_audit(gm, cvw.make_params(prm_l, mlp=net, sigma_ref=sref, audit_tol=1.0), U,
                            cvw.alloc_workspace(gm, cpl, 0))
    return {"training": {"snapshot_cells": int(F.shape[0]), "epochs": 20, "batch": 4096, "seconds": t_train},
            "audit_on_state": aud,
            "equal_l1": equal_l1(torch, cvw, prm, net),
            "sensor_plain": {"value": E / t_sp, "unit": "cells/s", "ms": t_sp * 1e3},
            "sensor_learned": {"value": E / t_sl, "unit": "cells/s", "ms": t_sl * 1e3},
            "step_plain": {"value": 3.0 * ndof / t_step_p, "unit": "DOF-updates/s", "ms_per_step": t_step_p * 1e3},
            "step_learned": {"value": 3.0 * ndof / t_step_l, "unit": "DOF-updates/s", "ms_per_step": t_step_l * 1e3},
            "features_ms": t_feat * 1e3, "network_ms": t_inf * 1e3,
            "network_tflops": 14464.0 * E / t_inf / 1e12,
            "status_flags": [cvw.poll_status(gm, wsp), cvw.poll_status(gm, wsl)]}


def cell_means(torch, U, n: int, p: int = 3):
    """Cell averages [4, n, n] of a DG Q_p state on n x n cells (collocated Gauss rule)."""
    _, w = np.polynomial.legendre.leggauss(p + 1)
    w2 = torch.from_numpy(np.outer(w, w).ravel() / 4.0).to(U.device, torch.float64)
    return (U.view(4, n * n, (p + 1) ** 2).double() @ w2).view(4, n, n)


def equal_l1(torch, cvw, prm, net, n: int = 128, steps: int = 40):
    """The learned sensor against the plain one at equal work on a reduced
    copy of the benchmark problem (n x n, DG Q3 Euler, the four-quadrant data
    with interfaces a fixed 0.02 wide): L1 errors of the cell averages after
    `steps` steps, against a plain-sensor run on the 2n x 2n mesh with half
    the step (its cell averages merged 2 x 2)."""
    import synth
    from paper_2601_16911_amd import learned
    k = 50.0
    res = {}
    U0 = euler_config4_state(n, gauss_nodes_2d(3), k).reshape(-1)
    rho, mx, my, En = (U0.reshape(4, -1)[c].astype(np.float64) for c in range(4))
    lam = float((np.hypot(mx, my) / rho + np.sqrt(1.4 * 0.4 * (En - 0.5 * (mx * mx + my * my) / rho) / rho)).max())
    dt = 0.1 * (1.0 / n) / (7 * lam)
    # reference: plain, 2n x 2n, dt / 2
    gf = cvw.Mesh(synth.quad_mesh(2 * n, 2 * n), 3, cvw.DG)
    Uf = torch.from_numpy(euler_config4_state(2 * n, gauss_nodes_2d(3), k).reshape(-1)).cuda()
    cpf = cvw.make_params(prm)
    cvw.step(gf, cpf, Uf, dt / 2, 2 * steps, cvw.alloc_workspace(gf, cpf, 1))
    ref = cell_means(torch, Uf, 2 * n).view(4, n, 2, n, 2).mean((2, 4))
    gm = cvw.Mesh(synth.quad_mesh(n, n), 3, cvw.DG)
    sref = learned.sigma_reference(gm, cvw.make_params(prm), torch.from_numpy(U0).cuda())
    prm_l = synth.Params(**{**prm.__dict__, "sensor": cvw.LEARNED})
    for name, cp in (("plain", cvw.make_params(prm)), ("learned", cvw.make_params(prm_l, mlp=net, sigma_ref=sref)),
                     ("gamma_0", cvw.make_params(synth.Params(**{**prm.__dict__, "sensor": 2, "fixed_gamma": 0.0})))):
        U = torch.from_numpy(U0.copy()).cuda()
        ws = cvw.alloc_workspace(gm, cp, 1)
        cvw.step(gm, cp, U, dt, steps, ws)
        err = (cell_means(torch, U, n) - ref).abs().sum((1, 2)) / (n * n)
        res[name] = {"l1_density": float(err[0].item()), "l1_all": float(err.sum().item()),
                     "flags": cvw.poll_status(gm, ws)}
    res["ratio_learned_to_plain"] = res["learned"]["l1_all"] / res["plain"]["l1_all"]
    res["workload"] = (f"2D Euler DG Q3, periodic {n}x{n}, {steps} steps of dt = 0.1 h / (7 lambda_max); reference: "
                       f"plain sensor on {2 * n}x{2 * n} with dt / 2, cell averages merged 2 x 2; L1 of the cell "
                       "averages per unit area, summed over the 4 variables")
    return res


def sensor_only(torch, cvw, n: int, part: str, calls: int, warmup: int):
    """Only the sensor pass (cvw_sensor, gamma of every cell) on the benchmark
    state, plain or learned (a network trained briefly as in bench_learned)."""
    import synth
    from paper_2601_16911_amd import learned
    mesh = synth.quad_mesh(n, n)
    gm = cvw.Mesh(mesh, 3, cvw.DG)
    prm = synth.Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0))
    U = torch.from_numpy(euler_config4_state(n, gauss_nodes_2d(3), SMOOTH_K * n / 1024).reshape(-1)).cuda()
    cp = cvw.make_params(prm)
    if part == "learned":
        ns = 256
        gs = cvw.Mesh(synth.quad_mesh(ns, ns), 3, cvw.DG)
        Us = torch.from_numpy(euler_config4_state(ns, gauss_nodes_2d(3), SMOOTH_K * ns / 1024).reshape(-1)).cuda()
        F, G = learned.collect(gs, prm, Us, 1e-5, 8, 4, learned.sigma_reference(gs, cp, Us))
        net = cvw.Mlp(learned.init_params(4))
        learned.train(net, F, G, epochs=5, batch=4096, lr=1e-3, seed=4)
        sref = learned.sigma_reference(gm, cp, U)
        cp = cvw.make_params(synth.Params(**{**prm.__dict__, "sensor": cvw.LEARNED}), mlp=net, sigma_ref=sref)
    ws = cvw.alloc_workspace(gm, cp, 1)
    E = mesh.n_cells
    gam = torch.empty(E, dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        cvw.sensor(gm, cp, U, gam, None, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(calls):
        cvw.sensor(gm, cp, U, gam, None, ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(calls, 1)
    return {"part": part, "cells": E, "calls": calls, "ms_per_call_wall": dt * 1e3,
            "status_flags": cvw.poll_status(gm, ws)}


def bench_ensemble(torch, cvw, steps: int, tune: bool = True):
    """The 64-instance DG ensemble (periodic unit squares, n in [64, 512], p in
    {1, 2, 3}, advection or Burgers, seeded), all instances stepped together by
    the batched stage, graph-captured and eager."""
    import synth
    stream = torch.cuda.current_stream()
    items, dofs, cells = [], 0, 0
    for inst in synth.config5_instances():
        mesh, p, prm, U, dt = synth.instance_case(inst)
        gm = cvw.Mesh(mesh, p, cvw.DG)
        u = torch.from_numpy(np.asarray(U, np.float32)).cuda()
        items.append((gm, cvw.make_params(prm), u, dt))
        dofs += U.size
        cells += mesh.n_cells
    b = cvw.Batch(items)
    ws = b.alloc_workspace()
    grid = 0
    if tune:
        from paper_2601_16911_amd import autotune
        entry = autotune.load_cache().get(autotune.batch_key(b))
        if entry is not None:
            grid = int(entry["grid"])
            b.set_grid(grid)
        else:
            grid = autotune.tune_batch(b, ws)
    out = {"workload": "64-instance DG ensemble, periodic n x n quads (n in [64, 512]), p in {1,2,3}, "
                       "advection / Burgers, SSP-RK3", "instances": len(items), "dofs": dofs, "steps": steps,
           "blocks": grid if grid else "one per item"}
    for name, graph in (("graph", True), ("eager", False)):
        t = _timed(torch, stream, lambda: b.step(steps, ws, use_graph=graph), 1) / steps
        out[name] = {"value": 3.0 * dofs / t, "unit": "DOF-updates/s", "ms_per_step": t * 1e3}
    out["status_flags"] = b.poll_status(ws)
    # compulsory bytes per step: per stage the sensor pass reads the stage
    # state and writes gamma, the cell pass reads the stage state and gamma and
    # writes the next state, and stages 2 and 3 read u_n: (3 + 2/3) x 4 B per
    # DOF and 8 B per cell, three stages
    alg = 3.0 * ((3.0 + 2.0 / 3.0) * 4.0 * dofs + 8.0 * cells)
    t = out["graph"]["ms_per_step"] * 1e-3
    out["roofline"] = {"bound": "alu", "hbm_bytes_per_step": alg, "hbm_achieved_GBs": alg / t / 1e9,
                       "hbm_peak_GBs": 8000.0, "hbm_frac": alg / t / 8e12,
                       "note": "the cell pass (82 % of the step) is bound by vector instruction issue per cell: "
                               "one variable per cell leaves the per-cell sensor, face and weight work "
                               "unshared, and degree-2 cells use 9 of the 16 lanes of a row"}
    return out


def bench_limiter(torch, cvw, gm, prm, U, dt):
    """The HWENO limiter (cvw_limit) on the benchmark state after the timed
    steps: every variable's vertex candidates, the sensor, and the
    componentwise reconstruction of the cells below the threshold, for
    threshold C_gamma = 0.9 (troubled cells) and 2 (every cell)."""
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, cvw.OP_LIMIT)
    out = torch.empty_like(U)
    gam = torch.empty(gm.info["n_cells"], dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    res = {"workload": "HWENO limiter on the 2D Euler DG Q3 1024x1024 state (67108864 DOFs), componentwise"}
    for name, thr in (("troubled", 0.9), ("all_cells", 2.0)):
        t = _timed(torch, stream, lambda: cvw.limit(gm, cp, U, out, thr, gam, ws), 5)
        res[name] = {"threshold": thr, "value": U.numel() / t, "unit": "DOF-updates/s", "ms": t * 1e3}
    res["limited_cells"] = int((gam < 0.9).sum().item())
    # in place, and the RKDG step: SSP-RK3 of the DG residual without
    # artificial viscosity (gamma = 1, SC off), the limiter after every stage
    Ui = U.clone()
    t = _timed(torch, stream, lambda: cvw.limit(gm, cp, Ui, Ui, 0.9, None, ws), 5)
    res["troubled_in_place"] = {"threshold": 0.9, "value": U.numel() / t, "unit": "DOF-updates/s", "ms": t * 1e3}
    import synth
    pr = cvw.make_params(synth.Params(**{**prm.__dict__, "sensor": 2, "fixed_gamma": 1.0, "sc_on": 0}))
    wr = cvw.alloc_workspace(gm, pr, 0)
    cand = torch.zeros((gm.info["n_vertices"], gm.info["n_k"]), dtype=torch.float32, device="cuda")
    Ur, S1, S2 = U.clone(), torch.empty_like(U), torch.empty_like(U)

    def rkdg_step():
        for us, un, uo, a0, b0 in ((Ur, None, S1, 0.0, 1.0), (S1, Ur, S2, 0.75, 0.25),
                                   (S2, Ur, Ur, 1.0 / 3.0, 2.0 / 3.0)):
            cvw.rk_stage(gm, pr, us, cand, un, uo, dt, a0, b0, wr)
            cvw.limit(gm, cp, uo, uo, 0.9, None, ws)

    t = _timed(torch, stream, rkdg_step, 3)
    res["rkdg_step"] = {"value": 3 * U.numel() / t, "unit": "DOF-updates/s", "ms_per_step": t * 1e3,
                        "finite": bool(torch.isfinite(Ur).all().item()),
                        "min_density": float(Ur[: U.numel() // 4].min().item())}
    return res


def bench_positivity(torch, cvw, gm, prm, U):
    """The Zhang-Shu positivity limiter (cvw_positivity) on the benchmark state
    after the timed steps (admissible: every cell is checked, none changes), in
    place, and out of place on a copy with negative density at one node of 1 %
    of the cells (seeded)."""
    cp = cvw.make_params(prm)
    stream = torch.cuda.current_stream()
    E = gm.info["n_cells"]
    nloc = U.numel() // (4 * E)
    ws = cvw.alloc_workspace(gm, cp, cvw.OP_POS)
    Ui = U.clone()
    t_ok = _timed(torch, stream, lambda: cvw.positivity(gm, cp, Ui, Ui, 1e-13, ws), 5)
    V = U.clone()
    g = torch.Generator(device="cpu").manual_seed(2024)
    cells = torch.randperm(E, generator=g)[: E // 100].cuda()
    V[cells * nloc] = -0.1
    out = torch.empty_like(V)
    t_bad = _timed(torch, stream, lambda: cvw.positivity(gm, cp, V, out, 1e-13, ws), 5)
    return {"workload": "Zhang-Shu positivity limiter on the 2D Euler DG Q3 1024x1024 state (67108864 DOFs)",
            "admissible_in_place": {"value": U.numel() / t_ok, "unit": "DOF-updates/s", "ms": t_ok * 1e3},
            "one_percent_cells_negative": {"value": U.numel() / t_bad, "unit": "DOF-updates/s", "ms": t_bad * 1e3,
                                           "min_density_after": float(out[: E * nloc].min().item())}}


def bench_triangles(torch, cvw, steps: int, n: int = 512, limiter: bool = True):
    """n x n squares split into 2 n^2 jittered triangles (512: 524,288; 2048:
    8,388,608, which no longer fits the 256 MB MALL), DG P3, KPP.  Roofline of
    the residual (vertex pass + cell pass) from its compulsory bytes per cell:
    read u and write R (2 x 40 B), the float64 geometry record (64 B), the
    neighbour and vertex tables (24 B), the vertex candidates written and read
    (9 floats per vertex, half a vertex per triangle: 36 B)."""
    import synth
    stream = torch.cuda.current_stream()
    p = 3
    mesh = synth.tri_mesh(n, n, -2.0, 2.0, -2.5, 1.5, jitter=0.1, seed=1003)
    X = mesh.cell_coords
    nodes = np.array([(i / p, j / p) for j in range(p + 1) for i in range(p + 1 - j)])
    px = X[:, 0, None, 0] + (X[:, 1, None, 0] - X[:, 0, None, 0]) * nodes[None, :, 0] \
        + (X[:, 2, None, 0] - X[:, 0, None, 0]) * nodes[None, :, 1]
    py = X[:, 0, None, 1] + (X[:, 1, None, 1] - X[:, 0, None, 1]) * nodes[None, :, 0] \
        + (X[:, 2, None, 1] - X[:, 0, None, 1]) * nodes[None, :, 1]
    U = torch.from_numpy(np.asarray(synth.u0_kpp(px, py), np.float32).ravel()).cuda()
    gm = cvw.Mesh(mesh, p, cvw.DG)
    prm = synth.Params(flux=synth.KPP, lambda_global=1.0)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 1)
    R = torch.empty_like(U)
    dofs = U.numel()
    h_min = 4.0 / n * 0.8
    dt = 0.1 * h_min / (2 * p + 1)
    t_res = _timed(torch, stream, lambda: cvw.residual(gm, cp, U, R, None, ws), 10)
    t_step = _timed(torch, stream, lambda: cvw.step(gm, cp, U, dt, steps, ws), 1) / steps
    alg = mesh.n_cells * (2 * 40 + 64 + 24 + 36)
    out = {"workload": f"KPP, DG P3 on {mesh.n_cells} jittered triangles ({n}x{n} squares)", "dofs": dofs,
           "residual": {"value": dofs / t_res, "unit": "DOF-updates/s", "ms": t_res * 1e3},
           "residual_roofline": {"bound": "hbm", "achieved": alg / t_res / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": alg / t_res / 1e9 / HBM_PEAK_GBS, "alg_bytes": alg},
           "step": {"value": 3.0 * dofs / t_step, "unit": "DOF-updates/s", "ms_per_step": t_step * 1e3},
           "status_flags": cvw.poll_status(gm, ws)}
    if limiter:
        # the HWENO limiter on the same state (threshold 0.9, out of place)
        wl = cvw.alloc_workspace(gm, cp, cvw.OP_LIMIT)
        Ul = torch.empty_like(U)
        t_lim = _timed(torch, stream, lambda: cvw.limit(gm, cp, U, Ul, 0.9, None, wl), 5)
        out["hweno_limiter"] = {"threshold": 0.9, "value": dofs / t_lim, "unit": "DOF-updates/s", "ms": t_lim * 1e3}
    return out


def bench_hex(torch, cvw, n: int = 128, p: int = 2, steps: int = 5, euler: bool = False):
    """3D: constant advection, DG Q_p on n^3 periodic cubes (128^3: 2,097,152
    cells, 56.6 M DOFs at p = 2), a smooth field plus a ball-shaped jump; or
    (euler) the Euler equations, gas gamma 1.4, a smooth flow with a ball of
    dense, high-pressure gas (five variables, the density the sensor field).
    Kernel times of the vertex pass (cvw_vertex_candidates) and of the cell
    pass in stage mode (cvw_rk_stage), the residual and the SSP-RK3 step.
    Roofline of the cell pass from its compulsory bytes per cell and stage:
    read u and write u_out (2 n_loc floats per variable), u_n in two of three
    stages, the candidates of one vertex per cell (n_k floats); the vertex
    pass: read the sensor field (n_loc floats per cell, one cell per vertex)
    and write the candidates."""
    import synth
    stream = torch.cuda.current_stream()
    mesh = synth.hex_mesh(n, n, n)
    n1 = p + 1
    x1 = np.polynomial.legendre.leggauss(n1)[0]
    Z, Y, X = np.meshgrid(x1, x1, x1, indexing="ij")
    nodes = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    h = 1.0 / n
    c0 = mesh.cell_coords[:, 0, :]
    pts = c0[:, None, :] + 0.5 * h * (nodes[None, :, :] + 1.0)
    x, y, z = pts[..., 0], pts[..., 1], pts[..., 2]
    ball = ((x - 0.45) ** 2 + (y - 0.4) ** 2 + (z - 0.5) ** 2) < 0.06
    if euler:
        g = 1.4
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 1.0 * ball
        vel = (0.4 * np.cos(2 * np.pi * z), -0.3 * np.sin(2 * np.pi * x), 0.2 * np.sin(2 * np.pi * y))
        pr = 1.0 + 0.2 * np.cos(2 * np.pi * (x + z)) + 1.5 * ball
        En = pr / (g - 1.0) + 0.5 * rho * sum(v * v for v in vel)
        U = torch.from_numpy(np.concatenate([np.asarray(a, np.float32).ravel()
                                             for a in (rho, rho * vel[0], rho * vel[1], rho * vel[2], En)])).cuda()
        lam = float(np.max(np.sqrt(sum(v * v for v in vel)) + np.sqrt(g * pr / rho)))
        del rho, vel, pr, En
        prm = synth.Params(flux=synth.EULER, flux_param=(g, 0, 0, 0))
        nv = 5
    else:
        u0 = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 0.5 * np.sin(2 * np.pi * z) + 1.5 * ball
        U = torch.from_numpy(np.asarray(u0, np.float32).ravel()).cuda()
        del u0
        prm = synth.Params(flux=synth.ADVECT_CONST, flux_param=(1.0, -0.6, 0.8, 0))
        lam = float(np.linalg.norm(prm.flux_param[:3]))
        nv = 1
    del pts, x, y, z, ball
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 1)
    R = torch.empty_like(U)
    V = torch.empty_like(U)
    nk = gm.info["n_k"]
    cand = torch.empty(mesh.n_vertices * nk, dtype=torch.float32, device="cuda")
    dofs = U.numel()
    dt = 0.1 * h / ((2 * p + 1) * lam)
    t_vtx = _timed(torch, stream, lambda: cvw.vertex_candidates(gm, cp, U, cand, ws), 10)
    t_cell = _timed(torch, stream, lambda: cvw.rk_stage(gm, cp, U, cand, U, V, dt, 0.75, 0.25, ws), 10)
    t_res = _timed(torch, stream, lambda: cvw.residual(gm, cp, U, R, None, ws), 10)
    t_step = _timed(torch, stream, lambda: cvw.step(gm, cp, U, dt, steps, ws), 1) / steps
    E = mesh.n_cells
    nl = n1 ** 3
    alg_cell = E * 4 * (nv * (2 * nl + 2.0 / 3.0 * nl) + nk)
    alg_vtx = E * 4 * (nl + nk)
    what = "Euler equations" if euler else "constant advection"
    return {"workload": f"3D {what}, DG Q{p} on {n}^3 periodic cubes ({E} cells)", "dofs": dofs,
            "vertex_pass": {"ms": t_vtx * 1e3, "achieved": alg_vtx / t_vtx / 1e9, "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": alg_vtx / t_vtx / 1e9 / HBM_PEAK_GBS},
            "cell_pass": {"ms": t_cell * 1e3, "achieved": alg_cell / t_cell / 1e9, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": alg_cell / t_cell / 1e9 / HBM_PEAK_GBS},
            "residual": {"value": dofs / t_res, "unit": "DOF-updates/s", "ms": t_res * 1e3},
            "step": {"value": 3.0 * dofs / t_step, "unit": "DOF-updates/s", "ms_per_step": t_step * 1e3},
            "status_flags": cvw.poll_status(gm, ws)}


def bench_tet(torch, cvw, n: int = 64, p: int = 2, steps: int = 5, euler: bool = False):
    """3D: constant advection, DG P_p on the six-tetrahedra split of n^3
    periodic cubes (64^3: 1,572,864 cells, 15.7 M DOFs at p = 2), a smooth
    field plus a ball-shaped jump; or (euler) the Euler equations, gas gamma
    1.4, a smooth flow with a ball of dense, high-pressure gas.  Kernel times
    of the vertex pass and of the cell pass in stage mode, the residual and
    the SSP-RK3 step.  Roofline of the cell pass from its compulsory bytes per
    cell and stage: read u and write u_out (2 n_loc floats per variable), u_n
    in two of three stages, the float64 geometry record (128 B), the
    neighbour codes (16 B) and the candidates of 1/6 vertex per cell (n_k
    floats)."""
    import synth
    stream = torch.cuda.current_stream()
    mesh = synth.tet_mesh(n, n, n)
    nodes = np.array([(i / p, j / p, k / p) for k in range(p + 1) for j in range(p + 1 - k)
                      for i in range(p + 1 - j - k)])
    X = mesh.cell_coords
    pts = X[:, None, 0, :] + np.einsum("edk,nk->end", np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0],
                                                               X[:, 3] - X[:, 0]], axis=-1), nodes)
    x, y, z = pts[..., 0], pts[..., 1], pts[..., 2]
    ball = ((x - 0.45) ** 2 + (y - 0.4) ** 2 + (z - 0.5) ** 2) < 0.06
    if euler:
        g = 1.4
        rho = 1.0 + 0.2 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 1.0 * ball
        vel = (0.4 * np.cos(2 * np.pi * z), -0.3 * np.sin(2 * np.pi * x), 0.2 * np.sin(2 * np.pi * y))
        pr = 1.0 + 0.2 * np.cos(2 * np.pi * (x + z)) + 1.5 * ball
        En = pr / (g - 1.0) + 0.5 * rho * sum(v * v for v in vel)
        U = torch.from_numpy(np.concatenate([np.asarray(a, np.float32).ravel()
                                             for a in (rho, rho * vel[0], rho * vel[1], rho * vel[2], En)])).cuda()
        lam = float(np.max(np.sqrt(sum(v * v for v in vel)) + np.sqrt(g * pr / rho)))
        del rho, vel, pr, En
        prm = synth.Params(flux=synth.EULER, flux_param=(g, 0, 0, 0))
        nv = 5
    else:
        u0 = np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 0.5 * np.sin(2 * np.pi * z) + 1.5 * ball
        U = torch.from_numpy(np.asarray(u0, np.float32).ravel()).cuda()
        del u0
        prm = synth.Params(flux=synth.ADVECT_CONST, flux_param=(1.0, -0.6, 0.8, 0))
        lam = float(np.linalg.norm(prm.flux_param[:3]))
        nv = 1
    del pts, x, y, z, ball
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 1)
    R = torch.empty_like(U)
    V = torch.empty_like(U)
    nk = gm.info["n_k"]
    cand = torch.empty(mesh.n_vertices * nk, dtype=torch.float32, device="cuda")
    dofs = U.numel()
    h = 1.0 / n
    dt = 0.05 * h / ((2 * p + 1) * lam)
    t_vtx = _timed(torch, stream, lambda: cvw.vertex_candidates(gm, cp, U, cand, ws), 10)
    t_cell = _timed(torch, stream, lambda: cvw.rk_stage(gm, cp, U, cand, U, V, dt, 0.75, 0.25, ws), 10)
    t_res = _timed(torch, stream, lambda: cvw.residual(gm, cp, U, R, None, ws), 10)
    t_step = _timed(torch, stream, lambda: cvw.step(gm, cp, U, dt, steps, ws), 1) / steps
    E = mesh.n_cells
    nl = gm.info["n_loc"]
    alg_cell = E * (4 * nv * (2 * nl + 2.0 / 3.0 * nl) + 128 + 16 + 4 * nk * mesh.n_vertices / E)
    what = "Euler equations" if euler else "constant advection"
    return {"workload": f"3D {what}, DG P{p} on {E} tetrahedra ({n}^3 periodic cubes split in six)",
            "dofs": dofs,
            "vertex_pass": {"ms": t_vtx * 1e3},
            "cell_pass": {"ms": t_cell * 1e3, "achieved": alg_cell / t_cell / 1e9, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": alg_cell / t_cell / 1e9 / HBM_PEAK_GBS},
            "residual": {"value": dofs / t_res, "unit": "DOF-updates/s", "ms": t_res * 1e3},
            "step": {"value": 3.0 * dofs / t_step, "unit": "DOF-updates/s", "ms_per_step": t_step * 1e3},
            "status_flags": cvw.poll_status(gm, ws)}


def bench_small_configs(torch, cvw):
    """The two small workloads, per stage: 1D advection (128 periodic cells,
    CG P2, float64, the pulse and hump data, CFL 0.3) and solid-body rotation
    (256 x 256 jittered bilinear Q2 cells, CG, float32, consistent mass by
    PCG).  Both are launch- and latency-bound (a few MB, resident in caches)."""
    import synth
    stream = torch.cuda.current_stream()
    out = {}
    # 1D advection: 128 cells, CG P2 (Gauss-Lobatto nodes -1, 0, 1), float64
    mesh = synth.segment_mesh(128)
    gm = cvw.Mesh(mesh, 2, cvw.CG)
    X = mesh.cell_coords[:, :, 0]
    xn = X[:, :1] + (X[:, 1:] - X[:, :1]) * (np.array([-1.0, 0.0, 1.0])[None, :] + 1.0) / 2.0
    u = torch.from_numpy(_cg_gather(gm, synth.u0_config1(xn))).cuda()
    prm = synth.Params(flux=synth.ADVECT_CONST, flux_param=(1.0, 0, 0, 0))
    cp = cvw.make_params(prm, cvw.F64)
    ws = cvw.alloc_workspace(gm, cp, 1)
    t = _timed(torch, stream, lambda: cvw.step(gm, cp, u, 0.3 * (1.0 / 128) / 2, 200, ws), 1) / 200
    out["config1_1d_advection"] = {"workload": "1D advection, 128 periodic cells, CG P2, float64, 200 steps",
                                   "dofs": u.numel(), "us_per_stage": t / 3 * 1e6, "ms_per_step": t * 1e3,
                                   "value": 3 * u.numel() / t, "unit": "DOF-updates/s",
                                   "status_flags": cvw.poll_status(gm, ws)}
    # solid-body rotation: 256 x 256 jittered bilinear Q2 cells, CG, float32
    n = 256
    mesh = synth.quad_mesh(n, n, jitter=0.1, seed=1002)
    gm = cvw.Mesh(mesh, 2, cvw.CG)
    g = np.array([-1.0, 0.0, 1.0])
    xi, eta = np.tile(g, 3), np.repeat(g, 3)                      # local nodes, x fastest
    N = np.stack([(1 - xi) * (1 - eta), (1 + xi) * (1 - eta), (1 + xi) * (1 + eta), (1 - xi) * (1 + eta)]) / 4
    P = np.einsum("vq,evd->eqd", N, mesh.cell_coords)
    u = torch.from_numpy(_cg_gather(gm, synth.u0_config2(P[..., 0], P[..., 1])).astype(np.float32)).cuda()
    prm = synth.Params(flux=synth.ADVECT_ROT, flux_param=(0.5, 0.5, 1.0, 0.0))
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 1)
    dt = 0.1 * (0.8 / n) / (5 * 0.5 * np.sqrt(2.0))
    t = _timed(torch, stream, lambda: cvw.step(gm, cp, u, dt, 10, ws), 1) / 10
    out["config2_rotation"] = {"workload": "solid-body rotation, 256x256 jittered bilinear Q2 cells, CG, float32, "
                                           "consistent mass by PCG", "dofs": u.numel(),
                               "us_per_stage": t / 3 * 1e6, "ms_per_step": t * 1e3, "value": 3 * u.numel() / t,
                               "unit": "DOF-updates/s", "status_flags": cvw.poll_status(gm, ws)}
    return out


def _line_nodes(p: int, space: int):
    """Reference nodes of the 1D elements: Gauss points (DG) or Gauss-Lobatto
    points (CG), ascending."""
    if space == 1:
        return np.polynomial.legendre.leggauss(p + 1)[0]
    inner = np.sort(np.polynomial.legendre.Legendre.basis(p).deriv().roots().real)
    return np.concatenate([[-1.0], inner, [1.0]])


def bench_line_euler(torch, cvw, steps: int = 20):
    """1D Euler on the modified shock tube (inflow at x = 0, reflecting wall at
    x = 1, float64): the paper's extreme degree, p = 32 on eight elements (CG
    and DG), and DG p = 8 on 4096 cells; SSP-RK3 steps of dt = 0.1 h / (2 p^2)."""
    import synth
    stream = torch.cuda.current_stream()
    prm = synth.modified_sod_params()
    out = {}
    for space, p, N in ((cvw.CG, 32, 8), (cvw.DG, 32, 8), (cvw.DG, 8, 4096), (cvw.CG, 8, 4096)):
        mesh = synth.segment_mesh(N, periodic=False)
        gm = cvw.Mesh(mesh, p, space)
        X = mesh.cell_coords[:, :, 0]
        xn = X[:, :1] + (X[:, 1:] - X[:, :1]) * (_line_nodes(p, space)[None, :] + 1.0) / 2.0
        left = xn < 0.25
        U = np.stack(synth.euler1d_conserved(np.where(left, 1.0, 0.125), np.where(left, 0.75, 0.0),
                                             np.where(left, 1.0, 0.1)))
        U = np.concatenate([_cg_gather(gm, U[c]) for c in range(3)]) if space == cvw.CG else U.reshape(-1)
        u = torch.from_numpy(np.ascontiguousarray(U)).cuda()
        cp = cvw.make_params(prm, cvw.F64)
        ws = cvw.alloc_workspace(gm, cp, 1)
        dt = 0.1 * (1.0 / N) / (2.0 * p * p)
        cvw.step(gm, cp, u, dt, 2, ws)                       # warm-up
        t = _timed(torch, stream, lambda: cvw.step(gm, cp, u, dt, steps, ws), 1) / steps
        name = f"line_euler_{'cg' if space == cvw.CG else 'dg'}_p{p}_{N}"
        out[name] = {"workload": f"1D Euler, modified shock tube (inflow / wall), {'CG' if space == cvw.CG else 'DG'} "
                                 f"P{p} on {N} cells, float64", "dofs": u.numel(), "us_per_stage": t / 3 * 1e6,
                     "ms_per_step": t * 1e3, "value": 3 * u.numel() / t, "unit": "DOF-updates/s",
                     "status_flags": cvw.poll_status(gm, ws)}
    return out


def bench_dmr(torch, cvw, ny: int = 96, t_end: float = 0.2, lam_bound: float = 20.0, max_wall: float = 60.0):
    """The double Mach reflection run of Sec. 5.4 on the paper's mesh (DG Q2,
    4 ny x ny cells on (0, 4) x (0, 1), 384 x 96 at ny = 96) to t = 0.2: per
    stage the vertex candidates, the stage (plain sensor, SC quadrature, HLL
    faces, boundary faces) and the Zhang-Shu limiter in place; the top
    boundary's states follow the moving shock (rewritten when a face's
    midpoint is passed).  dt = 0.1 h / ((2p + 1) lam_bound), lam_bound above
    the largest signal speed of the run.  Reports the step time and the
    density range at the end (the paper prints its range for the same run)."""
    import synth
    p = 2
    mesh = synth.quad_mesh(4 * ny, ny, x1=4.0, periodic=(False, False))
    gm = cvw.Mesh(mesh, p, cvw.DG)
    E = mesh.n_cells
    corners = mesh.cell_coords                                     # [E, 4, 2]
    nodes = gauss_nodes_2d(p)
    h = 1.0 / ny
    X = corners[:, :1, 0] + 0.5 * h * (nodes[None, :, 0] + 1.0)
    Y = corners[:, :1, 1] + 0.5 * h * (nodes[None, :, 1] + 1.0)
    U0 = np.asarray(synth.u0_dmr(X, Y), np.float32).reshape(-1)   # [4, E, 9]
    bf = gm.export(cvw.EXPORT_BFACE).reshape(-1, 2)
    c, f = bf[:, 0], bf[:, 1]
    mid = 0.5 * (corners[c, f] + corners[c, (f + 1) % 4])
    nrm = np.array([[0.0, -1.0], [1.0, 0.0], [0.0, 1.0], [-1.0, 0.0]])[f]
    kinds, states = synth.dmr_boundary(mid, nrm, 0.0)
    prm = synth.Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0), bc_face_kind=kinds, bc_face_state=states)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, cvw.OP_STEP)
    wp = cvw.alloc_workspace(gm, cp, cvw.OP_POS)
    cand = torch.zeros(gm.info["n_vertices"] * gm.info["n_k"], dtype=torch.float32, device="cuda")
    V = torch.from_numpy(U0).cuda()
    V1, V2 = torch.empty_like(V), torch.empty_like(V)
    eps0 = 1e-4
    cvw.positivity(gm, cp, V, V, eps0, wp)
    dt = 0.1 * h / ((2 * p + 1) * lam_bound)
    n_steps = int(np.ceil(t_end / dt))
    dt = t_end / n_steps
    top = nrm[:, 1] > 0.7
    cur = [int((top & (mid[:, 0] >= synth.dmr_shock_x(1.0, 0.0))).sum())]

    def stage(us, un, uo, a0, b0, ts):
        n_r = int((top & (mid[:, 0] >= synth.dmr_shock_x(1.0, ts))).sum())
        if n_r != cur[0]:                                          # a top face changed sides
            cvw.set_boundary_data(cp, states=synth.dmr_boundary(mid, nrm, ts)[1])
            cur[0] = n_r
        cvw.vertex_candidates(gm, cp, us, cand, ws)
        cvw.rk_stage(gm, cp, us, cand, un, uo, dt, a0, b0, ws)
        cvw.positivity(gm, cp, uo, uo, eps0, wp)

    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    t, done = 0.0, 0
    for _ in range(n_steps):
        stage(V, None, V1, 0.0, 1.0, t)
        stage(V1, V, V2, 0.75, 0.25, t + dt)
        stage(V2, V, V, 1.0 / 3.0, 2.0 / 3.0, t + 0.5 * dt)
        t += dt
        done += 1
        if done % 500 == 0:
            torch.cuda.synchronize()
            if time.perf_counter() - w0 > max_wall:
                break
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_s = e0.elapsed_time(e1) / 1e3
    flags = cvw.poll_status(gm, ws)
    rho = V[:E * 9]
    return {"workload": f"double Mach reflection, DG Q2 on {4 * ny} x {ny} quads (0,4)x(0,1), Euler, plain sensor + "
                        f"SC quadrature, Zhang-Shu limiter (eps0 {eps0}) after every stage, moving top boundary data",
            "cells": E, "dofs": 4 * E * 9, "steps": done, "t_reached": t, "dt": dt,
            "ms_per_step": gpu_s / done * 1e3, "wall_s": wall,
            "value": 3 * 4 * E * 9 * done / gpu_s, "unit": "DOF-updates/s",
            "rho_min": float(rho.min()), "rho_max": float(rho.max()),
            "paper_rho_range_sc": [1.274, 22.423], "status_flags": flags}


def _cg_gather(gm, vals):
    """Global CG vector from values at every cell's local nodes [E, n_loc]
    (the first occurrence of each DOF in (cell, local node) order)."""
    cd = gm.export(5).reshape(vals.shape)
    flat = cd.ravel()
    _, first = np.unique(flat, return_index=True)
    out = np.empty(int(flat.max()) + 1)
    out[flat[first]] = np.asarray(vals, np.float64).ravel()[first]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024, help="cells per direction")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the side measurements (ensemble batch, triangles)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one 256 MiB device copy (HBM counter calibration)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the built-in launch shapes (no autotuner launches before the timed region)")
    ap.add_argument("--part", choices=("step", "sensor", "learned", "small", "tri", "dmr", "hex", "hexeuler", "tet",
                                       "teteuler"),
                    default="step",
                    help="sensor / learned: only the plain or learned sensor pass, --steps calls after --warmup "
                         "(a short program for kernel traces and counters); small: only the 1D and CG "
                         "rotation workloads; tri: only the KPP triangle residual on 2048 x 2048 squares, --steps "
                         "calls; dmr: only the double Mach reflection run; hex / tet: only the 3D DG advection "
                         "on cubes / tetrahedra; hexeuler / teteuler: only the 3D Euler equations on cubes / "
                         "tetrahedra")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the hot path is benchmarked on one MI355X; "
              "multi-GPU sharding is a design note, not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2601_16911_amd import cvw

    torch.cuda.set_device(0)
    if args.part == "tri":
        print(json.dumps(bench_triangles(torch, cvw, args.steps, n=2048, limiter=False)))
        return
    if args.part == "dmr":
        print(json.dumps(bench_dmr(torch, cvw)))
        return
    if args.part == "hex":
        print(json.dumps(bench_hex(torch, cvw)))
        return
    if args.part == "hexeuler":
        print(json.dumps(bench_hex(torch, cvw, n=96, euler=True)))
        return
    if args.part == "tet":
        print(json.dumps(bench_tet(torch, cvw)))
        return
    if args.part == "teteuler":
        print(json.dumps(bench_tet(torch, cvw, euler=True)))
        return
    if args.part == "small":
        out = bench_small_configs(torch, cvw)
        out.update(bench_line_euler(torch, cvw))
        print(json.dumps(out))
        return
    if args.part != "step":
        print(json.dumps(sensor_only(torch, cvw, args.n, args.part, args.steps, args.warmup)))
        return
    n, p, nv = args.n, 3, 4
    mesh = synth.quad_mesh(n, n)
    gm = cvw.Mesh(mesh, p, cvw.DG)
    prm = synth.Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0))
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 1)
    U_h = euler_config4_state(n, gauss_nodes_2d(p), SMOOTH_K * n / 1024)
    U = torch.from_numpy(U_h.reshape(-1)).cuda()
    E = mesh.n_cells
    nloc = (p + 1) ** 2
    nk = (p + 1) * (p + 2) // 2 - 1
    ndof = E * nloc
    U1 = torch.empty_like(U)
    U2 = torch.empty_like(U)
    cand = torch.empty((mesh.n_vertices, nk), dtype=torch.float32, device="cuda")
    # fixed step inside the SSP-RK3 / DG stability region: CFL 0.1 / (2p + 1)
    rho, mx, my, En = (U_h[c].astype(np.float64) for c in range(4))
    pres = 0.4 * (En - 0.5 * (mx * mx + my * my) / rho)
    lam_max = float((np.hypot(mx, my) / rho + np.sqrt(1.4 * pres / rho)).max())
    dt = 0.1 * (1.0 / n) / ((2 * p + 1) * lam_max)
    stream = torch.cuda.current_stream()

    # launch shape of the cell pass: the autotuner's cached choice, else tuned
    # here (outside the timed region; results do not depend on it)
    grid = 0
    if not args.no_tune:
        from paper_2601_16911_amd import autotune
        grid = autotune.apply_cached(gm, cp)
        if grid is None:
            cvw.vertex_candidates(gm, cp, U, cand, ws)
            grid = autotune.tune_mesh(gm, cp, U, cand, ws)

    # every timing event is created and recorded once before the timed region
    # (the first event record of a process initialises the runtime's event
    # machinery, a host stall of tens of ms)
    hev = HipEvents()
    ev = [(hev.create(), hev.create(), hev.create()) for _ in range(3 * args.steps)]
    t_start, t_end = hev.create(), hev.create()
    for e in [t_start, t_end] + [x for tri in ev for x in tri]:
        hev.record(e, stream)
    torch.cuda.synchronize()
    n_rec = [0]
    gam = torch.empty(E, dtype=torch.float32, device="cuda")

    def rk_step(record: bool):
        # one stage: the sensor pass (gamma_e of u_stage), then the cell pass
        # with that gamma (viscosity, SC weights, volume and interface terms,
        # mass inverse, stage update); events before, between and after
        stages = ((U, None, U1, 0.0, 1.0), (U1, U, U2, 0.75, 0.25), (U2, U, U, 1.0 / 3.0, 2.0 / 3.0))
        for (us, un, uo, a0, b0) in stages:
            if record:
                e0, e1, e2 = ev[n_rec[0]]
                n_rec[0] += 1
                hev.record(e0, stream)
            cvw.sensor(gm, cp, us, gam, None, ws)
            if record:
                hev.record(e1, stream)
            cvw.rk_stage_gamma(gm, cp, us, gam, un, uo, dt, a0, b0, ws)
            if record:
                hev.record(e2, stream)

    for _ in range(args.warmup):
        rk_step(False)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    hev.record(t_start, stream)
    for _ in range(args.steps):
        rk_step(True)
    hev.record(t_end, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    t_total = hev.elapsed_ms(t_start, t_end) / 1e3
    sensor_ms = [hev.elapsed_ms(a, b) for a, b, _ in ev]
    eval_ms = [hev.elapsed_ms(b, c) for _, b, c in ev]
    hev.destroy(t_start, t_end, *[x for tri in ev for x in tri])
    flags = cvw.poll_status(gm, ws)

    # residual-only timing (vertex pass + fused cell pass writing R), same state
    R = torch.empty_like(U)
    wsr = cvw.alloc_workspace(gm, cp, 0)
    for _ in range(3):
        cvw.residual(gm, cp, U, R, None, wsr)
    torch.cuda.synchronize()
    r0 = torch.cuda.Event(enable_timing=True)
    r1 = torch.cuda.Event(enable_timing=True)
    r1.record(stream)
    torch.cuda.synchronize()
    r0.record(stream)
    nres = 10
    for _ in range(nres):
        cvw.residual(gm, cp, U, R, None, wsr)
    r1.record(stream)
    torch.cuda.synchronize()
    t_res = r0.elapsed_time(r1) / 1e3 / nres

    # the cell pass (dominant kernel): algorithmic flops per launch, and the
    # bytes it must move (read u_stage and gamma, write u_out, read u_n in
    # stages 2 and 3: averaged over the three stages)
    t_eval = float(np.mean(eval_ms)) / 1e3
    flops = cell_pass_flops(p, nv) * E
    state_bytes = nv * ndof * 4
    alg_bytes = state_bytes * (1 + 1 + 2.0 / 3.0) + 4 * E
    traffic = measured_traffic()
    valu = measured_valu()
    # the sensor pass (fused: read the sensor field once, write gamma)
    t_sens = float(np.mean(sensor_ms)) / 1e3
    sens_bytes = (4 * nloc + 4) * E

    value = 3.0 * ndof * nv * args.steps / t_total
    out = {
        "metric": "stabilized-residual DOF updates/s", "value": value, "unit": "DOF-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_total / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2D Euler DG Q3, periodic {n}x{n} quads ({E} cells, {ndof * nv} DOFs), "
                               "four-quadrant data with interfaces smoothed over ~2 cells, plain CV-WENO sensor + SC "
                               "quadrature, SSP-RK3", "cells": E, "degree": p, "n_var": nv,
                   "dofs": ndof * nv, "step": "one SSP-RK3 step = 3 x (fused sensor pass + cell pass)",
                   "cell_pass_blocks": grid if grid else "default"},
        "roofline": {"bound": "alu", "achieved": flops / t_eval / 1e12, "peak": FP32_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": flops / t_eval / 1e12 / FP32_VECTOR_PEAK_TFLOPS, "traffic": traffic,
                     "kernel": "dgq_eval_kernel<3, EULER> (cell pass, stage mode, gamma supplied)",
                     "avg_launch_ms": t_eval * 1e3, "alg_flops_per_launch": flops,
                     "flops_per_cell": cell_pass_flops(p, nv)},
        "hbm_view": {"achieved": alg_bytes / t_eval / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg_bytes / t_eval / 1e9 / HBM_PEAK_GBS, "alg_bytes_per_launch": alg_bytes},
        "valu_issue": {"instr_per_launch": valu, "achieved": (valu / t_eval) if valu else None,
                       "peak": VALU_ISSUE_PEAK, "unit": "wave-instr/s",
                       "frac": (valu / t_eval / VALU_ISSUE_PEAK) if valu else None,
                       "kernel": "dgq_eval_kernel<3, EULER>"},
        "sensor_pass": {"bound": "hbm", "kernel": "dgq_sensor_tile_kernel<3> (fused plain sensor pass)",
                        "avg_launch_ms": t_sens * 1e3, "value": E / t_sens, "unit_value": "cells/s",
                        "achieved": sens_bytes / t_sens / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": sens_bytes / t_sens / 1e9 / HBM_PEAK_GBS, "alg_bytes_per_launch": sens_bytes,
                        "traffic": measured_traffic("sensor_pass_bytes_per_launch"),
                        "valu_issue_frac": (measured_valu("sensor_pass_valu_instr_per_launch") / t_sens /
                                            VALU_ISSUE_PEAK) if measured_valu("sensor_pass_valu_instr_per_launch")
                        else None},
        "residual_only": {"value": ndof * nv / t_res, "unit": "DOF-updates/s", "ms": t_res * 1e3},
        "status_flags": flags,
        "wall_s_timed": wall,
    }
    if args.copy_calib:
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calib_bytes"] = a.numel() * 4
    if not args.no_extra:
        torch.cuda.empty_cache()
        out["learned_sensor"] = bench_learned(torch, cvw, gm, prm, U, dt, 5)
        torch.cuda.empty_cache()
        out["ensemble_batch"] = bench_ensemble(torch, cvw, 10, tune=not args.no_tune)
        torch.cuda.empty_cache()
        out["triangles_kpp"] = bench_triangles(torch, cvw, 5)
        torch.cuda.empty_cache()
        out["triangles_kpp_2048"] = bench_triangles(torch, cvw, 2, n=2048, limiter=False)
        torch.cuda.empty_cache()
        out.update(bench_small_configs(torch, cvw))
        out.update(bench_line_euler(torch, cvw))
        torch.cuda.empty_cache()
        out["hweno_limiter"] = bench_limiter(torch, cvw, gm, prm, U, dt)
        torch.cuda.empty_cache()
        out["positivity_limiter"] = bench_positivity(torch, cvw, gm, prm, U)
        torch.cuda.empty_cache()
        out["double_mach"] = bench_dmr(torch, cvw)
        torch.cuda.empty_cache()
        out["hexahedra_q2"] = bench_hex(torch, cvw)
        torch.cuda.empty_cache()
        out["hexahedra_q2_euler"] = bench_hex(torch, cvw, n=96, euler=True)
        torch.cuda.empty_cache()
        out["tetrahedra_p2"] = bench_tet(torch, cvw)
        torch.cuda.empty_cache()
        out["tetrahedra_p2_euler"] = bench_tet(torch, cvw, euler=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
