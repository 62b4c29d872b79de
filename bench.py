#!/usr/bin/env python3
"""Benchmark of the FP64 matrix-free action on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--all] [--no-batch] [--no-cpu-baseline]

A step is one full action y = A(u) (gather, geometry, evaluation, pointwise form,
quadrature, fixed-order scatter) over the whole mesh, inputs resident in HBM.  The
default workload is the 2D P4 compressible neo-Hookean residual on the 512x512 unit
square (524288 triangles, 8,396,802 DoFs, quadrature degree 8).  Prints ONE JSON line.

Besides the headline (warm: back-to-back steps) the default line carries its VJP, the
P2 mass action at 1024^2 and at 64^2, and the 3D P2 elasticity action at 64^3, each warm
and cold (every step after a read-only pass over 1.25 GiB that evicts L2 and the 256 MB
memory-side cache), the library's STREAM copy as the achievable bandwidth, the 64-mesh
batch, and the oracle on the host's CPUs.

Roofline: the kernel is bound by FP64 vector arithmetic (its arithmetic intensity is far
above the 9.8 flop/byte ridge), so `roofline` reports achieved FP64 flop/s of the
algorithmic flop count (the plain per-cell quadrature loop, counted per cell below)
against the 78.6 TFLOP/s FP64 vector peak.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6


# ----------------------------------------------------------------------- cost model
def cell_geometry_flops(dim: int, nq: int, ng: int) -> float:
    """J, det J, K = J^-1 and |det J|: once per affine cell, or at each of the nq points of
    a curved cell from its ng geometry nodes (J = sum_g x_g (x) grad phiG_g, 2 d^2 ng)."""
    d = dim
    inv = 3 + 1 + 4 + 1 if d == 2 else 17 + 1 + 45 + 1
    if ng:
        return nq * (2 * d * d * ng + inv)
    return (4 if d == 2 else 9) + inv


def flops_per_cell(form: int, dim: int, nloc: int, nq: int, ng: int = 0) -> float:
    """Algorithmic FP64 flops of one cell of the plain quadrature loop (FMA = 2); ng > 0
    for curved cells with ng geometry nodes."""
    d = dim
    geo = cell_geometry_flops(d, nq, ng)
    if form == 0:                        # mass: eval 2n, weight 2, contraction 2n
        per_q = 2 * nloc + 2 + 2 * nloc
        return geo + nq * per_q
    if form in (4, 5):                   # Laplace (+ mass term for Helmholtz)
        per_q = 2 * d * nloc + 2 * d * d + d + 1 + 2 * d * nloc
        if form == 5:
            per_q += 2 * nloc + 1 + 2 * nloc
        return geo + 2 * d ** 3 + nq * per_q
    ev = 2 * d * d * nloc                # reference gradients of the d components
    ct = 2 * d * d * nloc                # contraction against the test gradients
    geo_q = 2 * d ** 3 + (2 * d ** 3 + d * d) + 1   # G = gref K, T = W S K^T, W
    if form == 1:
        pw = d + 3 * d * d + d           # trace, mu (G + G^T), lam tr on diagonal
    elif form == 2:
        inv = 3 + 1 + 4 if d == 2 else 17 + 1 + 45
        pw = d + inv + 1 + 2 + 2 * d * d  # F = I + G, inverse, log, lam ln J - mu, P
    else:
        # SVK: F = I + G, F^T F (sym), tr E, S = lam trE I + 2 mu E, P = F S
        pw = d + d * (d + 1) * d + 2 * d + d * (d + 1) + 2 * d ** 3
    return geo + nq * (ev + ct + geo_q + pw)


def vjp_flops_per_cell(form: int, dim: int, nloc: int, nq: int, ng: int = 0) -> float:
    """The tangent contracted with grad v: neo-Hookean (2) or St Venant-Kirchhoff (3)."""
    d = dim
    geo = cell_geometry_flops(d, nq, ng)
    ev = 2 * (2 * d * d * nloc)          # gradients of u and v
    ct = 2 * d * d * nloc
    geo_q = 2 * (2 * d ** 3) + (2 * d ** 3 + d * d) + 1
    if form == 2:
        inv = 3 + 1 + 4 if d == 2 else 17 + 1 + 45
        pw = d + inv + 1 + 2 + 2 * d ** 3 + d + 2 * d ** 3 + 4 * d * d
    else:
        # F^T F, F^T H (sym), traces, S and dS, H S + F dS
        pw = d + 2 * d * (d + 1) * d + 4 * d + 2 * d * (d + 1) + 4 * d ** 3
    return geo + nq * (ev + ct + geo_q + pw)


def footprint_bytes(dim, n_vert, n_cell, nloc, n_dof, vectors=2, ng=None) -> float:
    """Each DoF, coordinate and map entry counted once (ng geometry nodes per cell: the
    d+1 vertices unless given)."""
    ng = dim + 1 if ng is None else ng
    return 8.0 * n_dof * vectors + 8.0 * dim * n_vert + 4.0 * nloc * n_cell + 4.0 * ng * n_cell


# ----------------------------------------------------------------------- timing
def time_steps(fn, steps: int, warmup: int):
    """Mean milliseconds per step over `steps` back-to-back steps: one pair of HIP events
    brackets the whole run on the current stream (per-step events would put their own
    packets and gaps between the steps).  Also returns the host wall time of the run."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(end) / steps, wall


def median_step_ms(fn, steps: int) -> float:
    """Median of per-step times, each step bracketed by its own pair of HIP events on the
    current stream (the per-step events add their packets; the mean comes from time_steps)."""
    import torch
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in evs]))


def time_kernel(plan, fn, steps: int):
    """Mean duration of the plan's main kernel (the patch kernel, without the shared-node
    fixup), from HIP events the library records around that launch on the same stream."""
    import torch
    torch.cuda.synchronize()
    plan.set_timing(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    ms, n = plan.timing()
    plan.set_timing(False)
    return ms / max(n, 1)


def kernel_source_hash() -> str:
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in ("paper_2506_17471_amd/csrc/forms.h", "paper_2506_17471_amd/csrc/kernel_templates.h",
              "paper_2506_17471_amd/csrc/mfma_patch.h", "paper_2506_17471_amd/csrc/kernels.hip"):
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(workload: str, kernel: str):
    """HBM bytes per launch measured by rocprofv3 counters (profiles/traffic.json), or None
    when the kernel sources changed since they were taken or another kernel ran."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != kernel_source_hash() or workload not in rec:
        return None
    r = rec[workload]
    if r.get("kernel") != kernel:
        return None
    return r["fetch_kib"] * 1024 * r["fetch_scale"] + r["write_kib"] * 1024 * r["write_scale"]


def fx_stream_sink() -> int:
    import paper_2506_17471_amd as fx
    return fx.STREAM_SINK


class ColdFlush:
    """Evict L2 and the 256 MB memory-side cache (MALL) before a cold step: the library's
    read-only pass over 1.25 GiB (five times the MALL).  Nothing is written but one partial
    sum per workgroup, so no dirty lines are left to be written back inside the timed step;
    the previous step's dirty output lines are written back during the pass, outside it."""

    def __init__(self, gib: float = 1.25):
        import torch
        self.buf = torch.ones(int(gib * (1 << 30)) // 8, dtype=torch.float64, device="cuda")
        self.sink = torch.empty(fx_stream_sink(), dtype=torch.float64, device="cuda")

    def __call__(self):
        import paper_2506_17471_amd as fx
        fx.stream_read(self.buf, self.sink)


def make_plan(w, tune: bool, vjp: bool = False, rule: str = "default", launch=None):
    import torch
    import paper_2506_17471_amd as fx
    plan = fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params)
    if rule != "default":
        plan.set_quadrature(fx.QUAD_CONICAL if rule == "conical" else fx.QUAD_SYMMETRIC)
    u = torch.as_tensor(w.u, device="cuda")
    y = torch.empty_like(u)
    v = None
    if vjp:
        v = torch.as_tensor(w.v if w.v is not None else
                            np.random.default_rng(9).uniform(-1, 1, w.n_dof), device="cuda")
    tuned = None
    if launch is not None:
        plan.set_strategy(*launch)
    elif tune:
        res = plan.tune(u, y=y, v=v)
        st = plan.strategy()          # what the tuner applied (the entry config wins ties)
        mine = [r for r in res if int(r[0]) == st[0] and (st[0] == 0 or (int(r[1]), int(r[2]),
                int(r[4])) == (st[1], st[2], st[3]))]
        tuned = {"strategy": "patch" if st[0] == 1 else "colour", "cells_per_patch": st[1],
                 "lanes_per_cell": st[2],
                 "sum_mode": SUM_NAMES.get(st[3], "-"),
                 "tuner_ms": float(min(r[5] for r in mine)) if mine else None,
                 "fastest_candidate_ms": float(min(r[5] for r in res)), "candidates": len(res)}
    return plan, u, v, y, tuned


def cold_steps(fn, steps: int, warmup: int, flush) -> np.ndarray:
    """Milliseconds of each of `steps` steps, each timed by its own pair of HIP events
    after a cache-evicting pass and a synchronisation (the pass is outside the events)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ms = []
    for _ in range(steps):
        flush()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn()
        b.record(st)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    return np.array(ms)


def run_workload(name: str, steps: int, warmup: int, cold: bool = False, vjp: bool = False,
                 tune: bool = True, rule: str = "default", flush=None, launch=None):
    """The workload's tuned plan timed warm (back-to-back steps, inputs resident in HBM and
    whatever of them the caches hold) and, with `cold`, cold (every step after a
    cache-evicting pass).  Returns (warm info, cold info or None, workload)."""
    import meshgen

    w = meshgen.workload(name, with_v=vjp)
    plan, u, v, y, tuned = make_plan(w, tune, vjp, rule, launch)
    if vjp:
        fn = lambda: plan.vjp(u, v, out=y)  # noqa: E731
    else:
        fn = lambda: plan.action(u, out=y)  # noqa: E731
    st = plan.strategy()
    curved = w.mesh.cell_gnodes is not None
    nv = w.mesh.gcoords.shape[0] if curved else w.mesh.n_vert
    ng = w.mesh.cell_gnodes.shape[1] if curved else 0
    if vjp and w.form in (2, 3):
        fl = vjp_flops_per_cell(w.form, w.mesh.dim, plan.n_loc, plan.n_quad, ng)
    else:
        fl = flops_per_cell(w.form, w.mesh.dim, plan.n_loc, plan.n_quad, ng)
    base = dict(workload=name, vjp=vjp, n_cell=w.mesh.n_cell, n_dof=w.n_dof,
                n_loc=plan.n_loc, n_quad=plan.n_quad, quad_family=plan.quad_family_name,
                tuned=tuned, flops_per_cell=fl, flops=fl * w.mesh.n_cell,
                bytes=footprint_bytes(w.mesh.dim, nv, w.mesh.n_cell, plan.n_loc, w.n_dof,
                                      3 if vjp and w.form in (2, 3) else 2, ng or None),
                geometry=2 if curved else 1, kernel_info=plan.kernel_info(vjp),
                launch={"strategy": "patch" if st[0] == 1 else "colour", "cells_per_patch": st[1],
                        "lanes_per_cell": st[2],
                        "sum_mode": SUM_NAMES.get(st[3], "-")})

    def finish(info, ms_mean, ms_median, kernel_ms):
        info.update(ms_mean=ms_mean, ms_median=ms_median, kernel_ms=kernel_ms)
        t = ms_mean / 1e3
        info["dof_per_s"] = w.n_dof / t
        info["tflops"] = info["flops"] / t / 1e12
        info["hbm_gbs_footprint"] = info["bytes"] / t / 1e9
        info["hbm_frac_footprint"] = info["hbm_gbs_footprint"] / HBM_PEAK_GBS
        info["fp64_frac"] = info["tflops"] / FP64_PEAK_TFLOPS
        if kernel_ms:
            info["kernel_tflops"] = info["flops"] / (kernel_ms / 1e3) / 1e12
            info["kernel_fp64_frac"] = info["kernel_tflops"] / FP64_PEAK_TFLOPS
            info["kernel_hbm_frac_footprint"] = info["bytes"] / (kernel_ms / 1e3) / 1e9 / HBM_PEAK_GBS
        return info

    ms, wall = time_steps(fn, steps, warmup)
    warm = finish(dict(base, cold=False, wall_s=wall), ms, median_step_ms(fn, steps),
                  time_kernel(plan, fn, steps))
    cold_info = None
    if cold:
        flush = flush or ColdFlush()
        cms = cold_steps(fn, steps, warmup, flush)
        # the kernel alone, cold: the library's events on the patch dispatch of each step
        plan.set_timing(True)
        for _ in range(steps):
            flush()
            fn()
        import torch
        torch.cuda.synchronize()
        kms, n = plan.timing()
        plan.set_timing(False)
        cold_info = finish(dict(base, cold=True, wall_s=float(cms.sum()) / 1e3), float(cms.mean()),
                           float(np.median(cms)), kms / max(n, 1))
    del plan
    return warm, cold_info, w


def run_autograd(name: str, steps: int, warmup: int) -> dict:
    """Forward plus backward through the torch.autograd.Function (y = A(u), then
    (dA/du)^T v as the backward of <y, v>) against the raw forward and VJP calls on the same
    plan (default launch configuration): the cost of the autograd path itself."""
    import torch
    import meshgen
    import paper_2506_17471_amd as fx
    w = meshgen.workload(name, with_v=True)
    plan = fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params)
    u = torch.as_tensor(w.u, device="cuda")
    v = torch.as_tensor(w.v, device="cuda")
    y, g = torch.empty_like(u), torch.empty_like(u)
    raw_ms, _ = time_steps(lambda: (plan.action(u, out=y), plan.vjp(u, v, out=g)), steps, warmup)
    ug = u.clone().requires_grad_(True)

    def step():
        ug.grad = None
        fx.FemAction.apply(ug, plan).backward(v)

    ag_ms, _ = time_steps(step, steps, warmup)
    torch.cuda.synchronize()
    ref = plan.vjp(u, v)
    same = bool(torch.equal(ug.grad, ref))
    del plan
    return {"workload": name, "raw_forward_plus_vjp_ms": raw_ms, "autograd_forward_backward_ms": ag_ms,
            "autograd_overhead": ag_ms / raw_ms, "autograd_grad_equals_raw_vjp": same}


def run_batch(steps: int, warmup: int, tune: bool = True, n_mesh: int = 64):
    """64 uneven meshes (2D P3 mass, 2D P6 neo-Hookean, 3D P4 elasticity): the sum of the
    per-mesh actions launched one by one against one replay of the batch graph."""
    import torch
    import meshgen
    import paper_2506_17471_amd as fx

    ws = meshgen.batch_workloads(n_mesh=n_mesh)
    plans, us, ys = [], [], []
    for w in ws:
        plan, u, _, y, _ = make_plan(w, False)
        plans.append(plan)
        us.append(u)
        ys.append(y)
    tuned = {}
    if tune:
        # tune the largest mesh of each kind and give its configuration to the others
        kinds = {}
        for i, w in enumerate(ws):
            k = w.name.split("_", 1)[1]
            if k not in kinds or w.mesh.n_cell > ws[kinds[k]].mesh.n_cell:
                kinds[k] = i
        for k, i in kinds.items():
            plans[i].tune(us[i], y=ys[i])
            st = plans[i].strategy()
            tuned[k] = list(st)
            for j, w in enumerate(ws):
                if w.name.split("_", 1)[1] == k and j != i:
                    if st[0] == 1:
                        plans[j].set_strategy(1, st[1], st[2], st[3])
                    else:
                        plans[j].set_strategy(0)
    per_mesh = lambda: [p.action(u, out=y) for p, u, y in zip(plans, us, ys)]  # noqa: E731
    ms_each, _ = time_steps(per_mesh, steps, warmup)
    # each mesh alone, to split out launch overhead
    alone = []
    for p, u, y in zip(plans, us, ys):
        m, _ = time_steps(lambda p=p, u=u, y=y: p.action(u, out=y), max(5, steps // 3), 2)
        alone.append(m)
    # the same per-mesh launches captured in one graph: isolates launch overhead from the
    # grouping of meshes into few launches; its replays must give the eager results bitwise
    y_eager = [y.clone() for y in ys]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        per_mesh()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        per_mesh()
    ms_pm_graph, _ = time_steps(g.replay, steps, warmup)
    torch.cuda.synchronize()
    pm_graph_ok = all(torch.equal(a, b) for a, b in zip(ys, y_eager))
    del g
    batch = fx.Batch(plans, us, ys)
    ms_graph, _ = time_steps(lambda: batch.run(graph=True), steps, warmup)
    ms_eager, _ = time_steps(lambda: batch.run(graph=False), steps, warmup)
    n_dof = sum(w.n_dof for w in ws)
    n_cell = sum(w.mesh.n_cell for w in ws)
    out = dict(n_mesh=len(ws), n_cell=n_cell, n_dof=n_dof, groups=batch.n_groups, tuned=tuned,
               patches=batch.n_patches,
               per_mesh_loop_ms=ms_each, sum_of_alone_ms=float(np.sum(alone)),
               per_mesh_graph_ms=ms_pm_graph, per_mesh_graph_matches_eager=pm_graph_ok,
               batch_graph_ms=ms_graph, batch_eager_ms=ms_eager,
               dof_per_s=n_dof / (ms_graph / 1e3))
    out["speedup_vs_per_mesh"] = out["per_mesh_loop_ms"] / out["batch_graph_ms"]
    out["speedup_vs_per_mesh_graph"] = out["per_mesh_graph_ms"] / out["batch_graph_ms"]
    batch.close()
    return out


def _sample_mesh(m, c0: int, c1: int, u: np.ndarray, ncomp: int):
    """Cells [c0, c1) of a mesh as a mesh of their own (nodes, vertices and geometry nodes
    renumbered compactly) and the matching slice of u."""
    import meshgen

    def compact(cells):
        ids, inv = np.unique(cells, return_inverse=True)
        return ids, inv.reshape(cells.shape).astype(np.int32)

    nodes, cn = compact(m.cell_nodes[c0:c1])
    verts, cv = compact(m.cell_verts[c0:c1])
    sub = meshgen.Mesh(m.dim, m.n, m.k, m.coords[verts], cv, cn, len(nodes), m.h)
    if m.cell_gnodes is not None:
        gn, cg = compact(m.cell_gnodes[c0:c1])
        sub.gcoords, sub.cell_gnodes = m.gcoords[gn], cg
    return sub, np.ascontiguousarray(u.reshape(-1, ncomp)[nodes].ravel())


def host_cpus() -> dict:
    """The host's processor as the process sees it: logical CPUs, the CPUs this process
    may run on, and the model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return {"cpu_count": os.cpu_count(), "affinity": allowed, "model": model}


# host threads the CPU baseline may use: the per-GPU CPU share of the MI355X boxes (16),
# or fewer where the process may run on fewer CPUs
CPU_SHARE = 16


def cpu_baseline(w, family: str, max_cells: int = 65536, seconds: float = 10.0):
    """The oracle on the first `max_cells` cells of the same mesh (a mesh of their own),
    with the quadrature rule the GPU plan used: on all the host threads the process may use
    (up to the per-GPU share), as independent contiguous chunks of the sample run
    concurrently (the C oracle releases the GIL), and on one thread."""
    import concurrent.futures
    import oracle
    m = w.mesh
    nc = min(max_cells, m.n_cell)
    sub, us = _sample_mesh(m, 0, nc, w.u, w.ncomp)
    oracle.action(w.form, sub, us, w.quad_degree, w.params, family=family)   # warm (tables, library)
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.action(w.form, sub, us, w.quad_degree, w.params, family=family)
        reps += 1
        if time.perf_counter() - t0 > seconds / 2:
            break
    dt = (time.perf_counter() - t0) / reps
    dofs_per_cell = w.n_dof / m.n_cell
    host = host_cpus()
    threads = max(1, min(CPU_SHARE, host["affinity"]))
    bounds = np.linspace(0, nc, threads + 1).astype(int)
    chunks = [_sample_mesh(m, int(a), int(b), w.u, w.ncomp) for a, b in zip(bounds[:-1], bounds[1:])]
    with concurrent.futures.ThreadPoolExecutor(threads) as ex:
        def once():
            list(ex.map(lambda c: oracle.action(w.form, c[0], c[1], w.quad_degree, w.params,
                                                family=family), chunks))
        once()
        t1 = time.perf_counter()
        preps = 0
        while True:
            once()
            preps += 1
            if time.perf_counter() - t1 > seconds / 2:
                break
        pdt = (time.perf_counter() - t1) / preps
    return {"value": nc * dofs_per_cell / pdt, "unit": "DoF/s", "cores": threads, "kind": "oracle",
            "sample": f"first {nc} of {m.n_cell} cells of the same mesh as a mesh of their own, "
                      f"in {threads} contiguous chunks run concurrently on {threads} threads, "
                      f"{preps} runs, {pdt * 1e3:.1f} ms each; DoF/s scaled by DoFs per cell of "
                      f"the full mesh",
            "host": host,
            "one_thread": {"value": nc * dofs_per_cell / dt, "cores": 1,
                           "sample": f"the same {nc} cells on one thread, {reps} runs, "
                                     f"{dt * 1e3:.1f} ms each"}}


def stream_copy_gbs(gib: float = 1.0, steps: int = 20) -> dict:
    """Achievable HBM bandwidth: the library's STREAM copy of `gib` GiB (read + write
    counted), mean over back-to-back copies, and the same pass read-only."""
    import torch
    import paper_2506_17471_amd as fx
    n = int(gib * (1 << 30)) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.empty(fx.STREAM_SINK, dtype=torch.float64, device="cuda")
    ms, _ = time_steps(lambda: fx.stream_copy(src, dst), steps, 3)
    rms, _ = time_steps(lambda: fx.stream_read(src, sink), steps, 3)
    torch.cuda.synchronize()
    assert torch.equal(dst[-5:], src[-5:])
    return {"bytes_each_way": n * 8, "copy_ms": ms, "copy_gbs": 2 * n * 8 / (ms / 1e3) / 1e9,
            "read_ms": rms, "read_gbs": n * 8 / (rms / 1e3) / 1e9}


SUM_NAMES = {1: "element", 2: "coloured"}
FORM_NAMES = {0: "mass", 1: "elasticity", 2: "neohookean", 3: "svk", 4: "laplace", 5: "helmholtz"}


def quad_degree_for(form: int, k: int) -> int:
    """Exact for the bilinear forms' polynomial integrands; 2k for the hyperelastic ones."""
    return 2 * (k - 1) if form in (1, 4) else 2 * k


def run_sweep(steps: int, warmup: int, tri_cells: float = 5e5, tet_cells: float = 2e5):
    """Every (form, dimension, degree) the library builds, at the paper's smaller mesh sizes
    (about 5e5 triangles / 2e5 tetrahedra), default launch configuration and rule: µs per
    action, DoF/s, algorithmic GFLOP/s and footprint GB/s, and the fraction of the binding
    roof (FP64 vector if the algorithmic intensity is above the 9.8 flop/byte ridge, else
    HBM)."""
    import torch
    import meshgen
    import paper_2506_17471_amd as fx

    out = []
    for dim, degrees in ((2, range(1, 9)), (3, range(1, 7))):
        for k in degrees:
            rng = np.random.default_rng(100 * dim + k)
            if dim == 2:
                mesh = meshgen.unit_square(max(1, round(math.sqrt(tri_cells / 2))), k, 0.1, rng)
            else:
                mesh = meshgen.unit_cube(max(1, round((tet_cells / 6) ** (1 / 3))), k, 0.05, rng)
            for form in range(6):
                ncomp = 1 if form in (0, 4, 5) else dim
                n_dof = mesh.n_node * ncomp
                params = () if ncomp == 1 else ((10.0, 1.0) if form in (2, 3)
                                                 else meshgen.lame_from_young(1.0, 0.3))
                if form in (2, 3):
                    u0 = meshgen.nh_displacement(rng, mesh)
                else:
                    u0 = rng.uniform(-1, 1, n_dof)
                plan = fx.Plan.from_mesh(form, mesh, quad_degree_for(form, k), params)
                u = torch.as_tensor(u0, device="cuda")
                y = torch.empty_like(u)
                ms, _ = time_steps(lambda: plan.action(u, out=y), steps, warmup)
                kms = time_kernel(plan, lambda: plan.action(u, out=y), steps)
                fl = flops_per_cell(form, dim, plan.n_loc, plan.n_quad) * mesh.n_cell
                by = footprint_bytes(dim, mesh.n_vert, mesh.n_cell, plan.n_loc, n_dof, 2)
                t = ms / 1e3
                ai = fl / by
                bound = "alu" if ai > FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9) else "hbm"
                frac = (fl / t / 1e12 / FP64_PEAK_TFLOPS) if bound == "alu" else (by / t / 1e9 / HBM_PEAK_GBS)
                st = plan.strategy()
                row = dict(form=FORM_NAMES[form], dim=dim, degree=k, n_cell=mesh.n_cell,
                           n_dof=n_dof, n_quad=plan.n_quad, rule=plan.quad_family_name,
                           launch=list(st), us=ms * 1e3, kernel_us=kms * 1e3,
                           dof_per_s=n_dof / t, gflops=fl / t / 1e9, gbs=by / t / 1e9,
                           intensity=ai, bound=bound, frac=frac)
                out.append(row)
                print(f"# sweep {row['form']:10s} {dim}D P{k}: {row['us']:9.1f} us "
                      f"{row['dof_per_s']:.3e} DoF/s {bound} {100 * frac:5.1f}%",
                      file=sys.stderr, flush=True)
                del plan, u, y
            del mesh
    return out


def spearman(a, b) -> float:
    """Rank correlation (average ranks for ties)."""
    from scipy.stats import rankdata
    ra, rb = rankdata(a), rankdata(b)
    ra, rb = ra - ra.mean(), rb - rb.mean()
    return float((ra @ rb) / math.sqrt((ra @ ra) * (rb @ rb)))


# cases the model's constants were set on, and held-out cases never looked at while setting them
MODEL_CASES = [(f, 2, k) for f in (0, 1, 2, 4) for k in (2, 4)] + [(f, 3, 2) for f in (0, 1, 2, 4)]
MODEL_HOLDOUT = [(0, 2, 3), (1, 2, 3), (3, 2, 3), (5, 2, 5), (2, 2, 5), (4, 3, 1), (1, 3, 1),
                 (5, 3, 2), (3, 3, 2), (1, 3, 3), (0, 3, 4)]


def run_model_eval(tri_cells: float = 5e5, tet_cells: float = 2e5, cases=None):
    """The tuner's cost model against the tuner's own measurements (the paper's evaluation
    of its heuristic model): per case the Spearman rank correlation between predicted and
    measured candidate times, and the top-k regret -- the throughput of the best measured
    candidate among the model's k best, as a fraction of the best measured overall."""
    import torch
    import meshgen
    import paper_2506_17471_amd as fx

    cases = MODEL_CASES if cases is None else cases
    out = []
    for form, dim, k in cases:
        rng = np.random.default_rng(7 * dim + k)
        if dim == 2:
            mesh = meshgen.unit_square(round(math.sqrt(tri_cells / 2)), k, 0.1, rng)
        else:
            mesh = meshgen.unit_cube(round((tet_cells / 6) ** (1 / 3)), k, 0.05, rng)
        ncomp = 1 if form in (0, 4, 5) else dim
        params = () if ncomp == 1 else ((10.0, 1.0) if form in (2, 3) else
                                        meshgen.lame_from_young(1.0, 0.3))
        u0 = meshgen.nh_displacement(rng, mesh) if form in (2, 3) else rng.uniform(-1, 1, mesh.n_node * ncomp)
        plan = fx.Plan.from_mesh(form, mesh, quad_degree_for(form, k), params)
        u = torch.as_tensor(u0, device="cuda")
        pred = {tuple(int(x) for x in r[:5]): r[5] for r in plan.tune_predict()}
        meas = {tuple(int(x) for x in r[:5]): r[5] for r in plan.tune(u)}
        keys = [key for key in meas if key in pred]
        pm, mm = np.array([pred[key] for key in keys]), np.array([meas[key] for key in keys])
        order = np.argsort(pm)
        best = mm.min()
        regret = {f"top{kk}": float(best / mm[order[:kk]].min()) for kk in (1, 3, 5)}
        row = dict(form=FORM_NAMES[form], dim=dim, degree=k, candidates=len(keys),
                   spearman=spearman(pm, mm), **regret,
                   best_measured_ms=float(best), model_pick_ms=float(mm[order[0]]))
        out.append(row)
        print(f"# model {row['form']:10s} {dim}D P{k}: rho {row['spearman']:.2f} "
              f"top1 {regret['top1']:.2f} top3 {regret['top3']:.2f} top5 {regret['top5']:.2f}",
              file=sys.stderr, flush=True)
        del plan, u
    summary = {k: float(np.mean([r[k] for r in out])) for k in ("spearman", "top1", "top3", "top5")}
    return {"cases": out, "mean": summary}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="nh_p4_2d")
    ap.add_argument("--all", action="store_true", help="also time the other workloads and the batch")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-mesh batch (timed by default: the batched speedup)")
    ap.add_argument("--batch", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-tune", action="store_true", help="use the plans' default launch configuration")
    ap.add_argument("--rule", choices=["default", "conical", "symmetric"], default="default",
                    help="quadrature rule family of the timed workload (default: the plan's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", default=None, metavar="S,P,L,M",
                    help="with --only: this launch configuration (strategy, cells per patch, "
                         "lanes per cell, sum mode, as fem_plan_set_strategy takes them) instead "
                         "of tuning")
    ap.add_argument("--only", action="store_true",
                    help="time the named workload alone (no VJP, other workloads, copy or batch); "
                         "for profiler runs")
    ap.add_argument("--sweep", action="store_true",
                    help="only run the degree sweep over every built (form, dim, degree)")
    ap.add_argument("--model-eval", action="store_true",
                    help="only evaluate the tuner's cost model against measured candidates")
    ap.add_argument("--holdout", action="store_true",
                    help="with --model-eval: the held-out cases instead of the calibration cases")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (5 times), to calibrate the "
                         "FETCH_SIZE / WRITE_SIZE counters against a known byte count")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the action "
              f"shards by cells across GPUs, which this library does not implement)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        import paper_2506_17471_amd as fx
        n = args.copy_calibration * 1024 * 1024 // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            fx.stream_copy(src, dst)
        torch.cuda.synchronize()
        ms, _ = time_steps(lambda: fx.stream_copy(src, dst), 20, 0)
        print(json.dumps({"copy_calibration_bytes_each_way": n * 8, "copies": 25,
                          "copy_gbs_read_plus_write": 2 * n * 8 / (ms / 1e3) / 1e9}))
        return
    tune = not args.no_tune
    if args.sweep:
        print(json.dumps({"sweep": run_sweep(args.steps, args.warmup)}))
        return
    if args.model_eval:
        print(json.dumps({"model_eval": run_model_eval(cases=MODEL_HOLDOUT if args.holdout else None)}))
        return

    def note(msg):
        print(f"# {msg}", file=sys.stderr, flush=True)

    if args.only:
        launch = tuple(int(x) for x in args.launch.split(",")) if args.launch else None
        info, _, _ = run_workload(args.workload, args.steps, args.warmup, tune=tune, rule=args.rule,
                                  launch=launch)
        print(json.dumps({"only": info}))
        return
    flush = ColdFlush()
    main_info, main_cold, w = run_workload(args.workload, args.steps, args.warmup, cold=True,
                                           tune=tune, rule=args.rule, flush=flush)
    note(f"{args.workload}: {main_info['ms_mean']:.4f} ms/step warm, {main_cold['ms_mean']:.4f} cold, "
         f"tuned {main_info['tuned']}")
    extras = {args.workload + "_cold": main_cold}
    if w.form == 2:
        vinfo, vcold, _ = run_workload(args.workload, args.steps, args.warmup, cold=True, vjp=True,
                                       tune=tune, rule=args.rule, flush=flush)
        extras["vjp"] = vinfo
        extras["vjp_cold"] = vcold
        extras["adjoint_forward_time_ratio"] = vinfo["ms_mean"] / main_info["ms_mean"]
        note(f"vjp: {vinfo['ms_mean']:.4f} ms/step warm, {vcold['ms_mean']:.4f} cold")
        extras["autograd"] = run_autograd(args.workload, args.steps, args.warmup)
        note(f"autograd: {extras['autograd']}")
    # the memory-bound form at a size where HBM, not launch latency, binds (P2 mass at
    # 1024^2), the 3D P2 elasticity action and the P2 mass action at its stated 64^2 size:
    # warm and cold
    for name in ("mass_p2_2d_1024", "elast_p2_3d", "mass_p2_2d"):
        info, cinfo, _ = run_workload(name, args.steps, args.warmup, cold=True, tune=tune, flush=flush)
        extras[name] = info
        extras[name + "_cold"] = cinfo
        note(f"{name}: {info['ms_mean']:.4f} ms/step warm, {cinfo['ms_mean']:.4f} cold")
    extras["stream"] = stream_copy_gbs()
    note(f"stream: {extras['stream']}")
    if args.all:
        # the paper's hyperelastic law (St Venant-Kirchhoff): residual and tangent action
        info, _, _ = run_workload("svk_p4_2d", args.steps, args.warmup, tune=tune)
        extras["svk_p4_2d"] = info
        note(f"svk_p4_2d: {info['ms_mean']:.4f} ms/step")
        info, _, _ = run_workload("svk_p4_2d", args.steps, args.warmup, vjp=True, tune=tune)
        extras["svk_p4_2d_tangent"] = info
        note(f"svk_p4_2d tangent: {info['ms_mean']:.4f} ms/step")
        if w.form == 2 and args.rule == "default":
            # the same operator family with the conical-product rule (more points)
            info, _, _ = run_workload(args.workload, args.steps, args.warmup, tune=tune, rule="conical")
            extras[args.workload + "_conical"] = info
            note(f"{args.workload} conical rule: {info['ms_mean']:.4f} ms/step")
        # curved (P2-geometry) cells: J, K and |det J| at every quadrature point
        for name in ("nh_p4_2d_curved", "mass_p2_2d_1024_curved"):
            info, _, _ = run_workload(name, args.steps, args.warmup, tune=tune)
            extras[name] = info
            note(f"{name}: {info['ms_mean']:.4f} ms/step")
    if not args.no_batch:
        extras["batch"] = run_batch(args.steps, args.warmup, tune=tune)
        note(f"batch: {extras['batch']}")
    del flush

    # the dominant kernel alone (its own HIP-event duration); the step adds the fixup
    achieved = main_info["kernel_tflops"]
    lanes, mode = main_info["launch"]["lanes_per_cell"], main_info["launch"]["sum_mode"]
    geo = main_info["geometry"]
    mode_id = {v: k for k, v in SUM_NAMES.items()}.get(mode, 0)
    prio = "true" if main_info["kernel_info"]["wave_priority"] else "false"
    if main_info["launch"]["strategy"] == "patch" and lanes == 4:
        kname = f"mfma_patch_kernel<{w.form}, {w.mesh.dim}, {w.mesh.k}, false>"
    elif main_info["launch"]["strategy"] == "patch":
        kname = (f"patch_kernel<{w.form}, {w.mesh.dim}, {w.mesh.k}, false, {lanes}, "
                 f"{mode_id}, {geo}, {prio}>")
    else:
        kname = f"colour_kernel<{w.form}, {w.mesh.dim}, {w.mesh.k}, false, {geo}>"
    stream_gbs = extras["stream"]["copy_gbs"]

    def hbm(info, kernel=False):
        return info["kernel_hbm_frac_footprint"] if kernel else info["hbm_frac_footprint"]

    mass, mass_c = extras["mass_p2_2d_1024"], extras["mass_p2_2d_1024_cold"]
    hbm_names = [args.workload, "mass_p2_2d_1024", "elast_p2_3d"]
    out = {
        "metric": "FP64 FE action DoF/s + % HBM roofline; adjoint/forward time ratio; batched speedup",
        "value": main_info["dof_per_s"],
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_info["ms_mean"],
        "ms_per_step_median": main_info["ms_median"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_cell": main_info["n_cell"],
                   "n_dof": main_info["n_dof"], "n_quad": main_info["n_quad"],
                   "quad_rule": main_info["quad_family"],
                   "launch": main_info["launch"], "tuner": main_info["tuned"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": recorded_traffic(args.workload, kname),
                     "kernel": kname,
                     "flops_per_launch": main_info["flops"],
                     "avg_kernel_ms": main_info["kernel_ms"],
                     "avg_step_ms": main_info["ms_mean"],
                     "step_tflops": main_info["tflops"],
                     "footprint_gbs": main_info["hbm_gbs_footprint"]},
        # the metric's other parts on this run.  HBM roofline fractions: footprint bytes per
        # step (each DoF, coordinate and map entry once) against 8 TB/s, cold (every step
        # after a read-only pass over 1.25 GiB that evicts L2 and the 256 MB MALL) and warm
        # (back-to-back steps); "kernel" is the main kernel's own time without the fixup.
        "summary": {
            "dof_per_s": main_info["dof_per_s"],
            "hbm_roofline_frac": {
                "cold": {n: hbm(extras[n + "_cold"]) for n in hbm_names},
                "cold_kernel": {n: hbm(extras[n + "_cold"], True) for n in hbm_names},
                "warm": {n: hbm(extras[n] if n != args.workload else main_info) for n in hbm_names},
                "warm_kernel": {n: hbm(extras[n] if n != args.workload else main_info, True)
                                for n in hbm_names},
            },
            "mass_p2_2d_1024_vs_stream_copy": {"cold": mass_c["hbm_gbs_footprint"] / stream_gbs,
                                               "warm": mass["hbm_gbs_footprint"] / stream_gbs},
            "stream_copy_gbs": stream_gbs,
            "fp64_roofline_frac": {
                args.workload: main_info["fp64_frac"],
                args.workload + "_kernel": main_info["kernel_fp64_frac"],
                "elast_p2_3d": extras["elast_p2_3d"]["fp64_frac"],
                "elast_p2_3d_kernel": extras["elast_p2_3d"]["kernel_fp64_frac"],
                **({"nh_vjp": extras["vjp"]["fp64_frac"],
                    "nh_vjp_kernel": extras["vjp"]["kernel_fp64_frac"]} if "vjp" in extras else {}),
            },
            "us_per_step": {n: 1e3 * extras[n]["ms_mean"] for n in ("mass_p2_2d", "elast_p2_3d",
                                                                   "mass_p2_2d_1024")},
            "adjoint_forward_time_ratio": extras.get("adjoint_forward_time_ratio"),
            "batched_speedup": extras["batch"]["speedup_vs_per_mesh"] if "batch" in extras else None,
        },
        "extras": extras,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, main_info["quad_family"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
