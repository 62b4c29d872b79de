"""The 64-mesh uneven batch at its full size (seed 4: 3.3 M cells, 88 M DoFs; 2D P3 mass,
2D P6 neo-Hookean, 3D P4 elasticity, mesh i of form i mod 3, cell counts log-uniform in
[1e3, 2e5]) through fem_batch_run, every mesh's output against the oracle element by
element (relative max and L2 error <= 1e-12), in the default launch configuration and in
the one the benchmark's tuner picked on MI355X.  The oracle runs one mesh per host thread.
"""
import concurrent.futures
import os
import sys

import numpy as np
import pytest

import meshgen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2506_17471_amd as fx  # noqa: E402

TOL = 1e-12
DEV = torch.device("cuda:0")

# (form, dim, degree) -> (patch cells, lanes per cell, sum mode) the benchmark's tuner kept
TUNED = {(fx.FORM_MASS, 2, 3): (256, 1, fx.SUM_COLOURED),
         (fx.FORM_NEOHOOKEAN, 2, 6): (128, 2, fx.SUM_COLOURED),
         (fx.FORM_ELASTICITY, 3, 4): (42, 3, fx.SUM_COLOURED)}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def family(w):
    return "symmetric" if oracle.quadrature.has_symmetric(w.mesh.dim, w.quad_degree) else "conical"


_state = {}


def batch_and_reference():
    if not _state:
        ws = meshgen.batch_workloads()
        say(f"[batch-full] {len(ws)} meshes, {sum(w.mesh.n_cell for w in ws)} cells, "
            f"{sum(w.n_dof for w in ws)} DoFs")
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        with concurrent.futures.ThreadPoolExecutor(threads) as ex:
            refs = list(ex.map(lambda w: oracle.action(w.form, w.mesh, w.u, w.quad_degree,
                                                       w.params, family=family(w)), ws))
        say(f"[batch-full] oracle done on {threads} threads")
        _state["ws"], _state["refs"] = ws, refs
    return _state["ws"], _state["refs"]


@pytest.mark.parametrize("config", ["default", "tuned"])
def test_full_batch_against_oracle(config):
    ws, refs = batch_and_reference()
    plans = [fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params) for w in ws]
    for w, p in zip(ws, plans):
        assert p.quad_family_name == family(w)
        if config == "tuned":
            pc, ln, sm = TUNED[(w.form, w.mesh.dim, w.mesh.k)]
            p.set_strategy(fx.SCATTER_PATCH, pc, ln, sm)
    us = [torch.as_tensor(w.u, device=DEV) for w in ws]
    ys = [torch.full_like(u, 7.0) for u in us]
    b = fx.Batch(plans, us, ys)
    say(f"[batch-full] {config}: {b.n_groups} groups, {b.n_patches} patches")
    for rep in range(2):
        for y in ys:
            y.fill_(7.0)
        b.run(graph=True)
        torch.cuda.synchronize()
        worst = 0.0
        for i, (w, y, ref) in enumerate(zip(ws, ys, refs)):
            out = y.cpu().numpy()
            scale = max(np.max(np.abs(ref)), 1e-300)
            emax = np.max(np.abs(out - ref)) / scale
            el2 = np.linalg.norm(out - ref) / max(np.linalg.norm(ref), 1e-300)
            worst = max(worst, emax, el2)
            assert emax < TOL and el2 < TOL, (i, w.name, emax, el2)
        say(f"[batch-full] {config} replay {rep}: worst relative error {worst:.2e}")
    b.close()
    for p in plans:
        p.close()
