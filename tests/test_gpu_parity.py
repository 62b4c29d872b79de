"""GPU parity: the HIP path through the C ABI against the CPU oracle (FP64).

Bar: relative max error and relative L2 error <= 1e-12 against the oracle on the same
seeded inputs (the forms are evaluated in FP64 on both sides, only the summation order
differs), bit-exact for the colouring, bitwise-identical repeated runs.
"""
import ctypes
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
NH = (10.0, 1.0)
LAME = meshgen.lame_from_young(1.0, 0.3)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_err(y, ref):
    y = np.asarray(y)
    ref = np.asarray(ref)
    scale = max(np.max(np.abs(ref)), 1e-300)
    return np.max(np.abs(y - ref)) / scale, np.linalg.norm(y - ref) / max(np.linalg.norm(ref), 1e-300)


def gpu(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def params_for(form):
    if form in fx.SCALAR_FORMS:
        return ()
    return LAME if form == fx.FORM_ELASTICITY else NH


HYPERELASTIC = (fx.FORM_NEOHOOKEAN, fx.FORM_SVK)



def rule_families(dim, quad_degree):
    """The rule families a plan can run at this degree: conical always, symmetric where
    one is built."""
    return ["conical"] + (["symmetric"] if oracle.quadrature.has_symmetric(dim, quad_degree) else [])



def vjp_or_skip(plan, u, v):
    """The VJP, or a skip where the configuration's tangent kernel spills to scratch or needs
    more LDS than a workgroup has (the library refuses to run those)."""
    try:
        return plan.vjp(u, v)
    except fx.FemError as e:
        if e.status == fx.E_UNSUPPORTED and "scratch" in str(e):
            pytest.skip(f"tangent kernel spills: {e}")
        if e.status == fx.E_UNSUPPORTED and "LDS" in str(e):
            pytest.skip(f"tangent kernel does not fit the workgroup's LDS: {e}")
        raise


def inputs(form, mesh, seed):
    rng = np.random.default_rng(seed)
    ncomp = 1 if form in fx.SCALAR_FORMS else mesh.dim
    if form == fx.FORM_NEOHOOKEAN:
        u = meshgen.nh_displacement(rng, mesh, 0.01)
        # an admissible state: det F > 0 at every quadrature point of every rule a test
        # may run at this degree (the plans default to the symmetric rule where one is
        # built; the conical rule is always available)
        for fam in rule_families(mesh.dim, 2 * mesh.k):
            assert oracle.min_det_f(mesh, u, 2 * mesh.k, family=fam) > 0.5
    elif form == fx.FORM_SVK:
        # SVK needs no det F > 0; a larger state exercises its cubic terms
        u = meshgen.nh_displacement(rng, mesh, 0.2)
    else:
        u = rng.uniform(-1, 1, mesh.n_node * ncomp)
    v = rng.uniform(-1, 1, mesh.n_node * ncomp)
    return u, v


def qdeg(form, k):
    return 2 * (k - 1) if form in (fx.FORM_ELASTICITY, fx.FORM_LAPLACE) else 2 * k


CASES = [(f, 2, k) for f in range(6) for k in range(1, 7)] + \
        [(f, 3, k) for f in range(6) for k in range(1, 5)]


def plan_family(w):
    """The rule family a plan picks for this workload: the symmetric rule where one is
    built for the degree (the library's documented default), else the conical rule."""
    return "symmetric" if oracle.quadrature.has_symmetric(w.mesh.dim, w.quad_degree) else "conical"


STRATS = [(fx.SCATTER_PATCH, 0, 0, 0), (fx.SCATTER_PATCH, 64, 1, fx.SUM_ELEMENT),
          (fx.SCATTER_PATCH, 128, 1, fx.SUM_COLOURED), (fx.SCATTER_COLOUR, 0, 0, 0),
          (fx.SCATTER_PATCH, 42, 3, fx.SUM_ELEMENT), (fx.SCATTER_PATCH, 63, 3, fx.SUM_COLOURED),
          (fx.SCATTER_PATCH, 64, 2, fx.SUM_ELEMENT), (fx.SCATTER_PATCH, 128, 2, fx.SUM_COLOURED),
          (fx.SCATTER_PATCH, 64, 4, fx.SUM_COLOURED)]
STRAT_IDS = ["patch", "patch64x1e", "patch128x1c", "colour", "patch42x3e", "patch63x3c",
             "patch64x2e", "patch128x2c", "mfma64"]


def apply_strategy(plan, strategy, form, dim):
    if strategy[2] == 4 and getattr(plan, "geometry", 1) == 2:
        pytest.skip("curved cells run one lane per cell")
    if strategy[2] == 3 and (dim != 3 or form in fx.SCALAR_FORMS):
        pytest.skip("three lanes per cell exist for the 3D vector forms only")
    if strategy[2] == 2 and (dim != 2 or form in fx.SCALAR_FORMS):
        pytest.skip("two lanes per cell exist for the 2D vector forms only")
    if strategy[2] > 1 and getattr(plan, "geometry", 1) == 2:
        pytest.skip("curved cells run one lane per cell")
    try:
        plan.set_strategy(*strategy)
    except fx.FemError as e:
        if e.status == fx.E_UNSUPPORTED and "LDS" in str(e):
            pytest.skip(f"configuration does not fit the workgroup's LDS: {e}")
        raise


@pytest.mark.parametrize("strategy", STRATS, ids=STRAT_IDS)
@pytest.mark.parametrize("form,dim,k", CASES)
def test_action_small_meshes(form, dim, k, strategy):
    # 2D n=9: 162 cells; 3D n=3: 162 cells -- several wavefronts / patches plus a ragged tail
    n = 9 if dim == 2 else 3
    mesh = meshgen.make_mesh(dim, n, k, None, np.random.default_rng(100 + k))
    u, _ = inputs(form, mesh, k)
    qd = qdeg(form, k)
    say(f"[action] form={form} dim={dim} k={k} n={n} cells={mesh.n_cell} qd={qd} strat={strategy}")
    plan = fx.Plan.from_mesh(form, mesh, qd, params_for(form))
    apply_strategy(plan, strategy, form, dim)
    y = plan.action(gpu(u)).cpu().numpy()
    ref = oracle.action(form, mesh, u, qd, params_for(form), family=plan.quad_family_name)
    emax, el2 = rel_err(y, ref)
    assert emax < TOL and el2 < TOL, (emax, el2)


@pytest.mark.parametrize("strategy", STRATS, ids=STRAT_IDS)
@pytest.mark.parametrize("form,dim,k", CASES)
def test_vjp_small_meshes(form, dim, k, strategy):
    n = 7 if dim == 2 else 2
    mesh = meshgen.make_mesh(dim, n, k, None, np.random.default_rng(200 + k))
    u, v = inputs(form, mesh, 50 + k)
    qd = qdeg(form, k)
    say(f"[vjp] form={form} dim={dim} k={k} n={n} cells={mesh.n_cell} qd={qd} strat={strategy}")
    plan = fx.Plan.from_mesh(form, mesh, qd, params_for(form))
    apply_strategy(plan, strategy, form, dim)
    g = vjp_or_skip(plan, gpu(u), gpu(v)).cpu().numpy()
    ref = oracle.vjp(form, mesh, u, v, qd, params_for(form), family=plan.quad_family_name)
    emax, el2 = rel_err(g, ref)
    assert emax < TOL and el2 < TOL, (emax, el2)


HIGH = [(f, 2, k) for f in range(6) for k in (7, 8)] + [(f, 3, k) for f in range(6) for k in (5, 6)]
HIGH_STRATS = [(fx.SCATTER_PATCH, 0, 0, 0), (fx.SCATTER_PATCH, 64, 1, fx.SUM_COLOURED),
               (fx.SCATTER_PATCH, 64, 0, fx.SUM_ELEMENT), (fx.SCATTER_COLOUR, 0, 0, 0),
               (fx.SCATTER_PATCH, 64, 4, fx.SUM_COLOURED)]


@pytest.mark.parametrize("strategy", HIGH_STRATS, ids=["patch", "patch64x1c", "patch64e", "colour",
                                                      "mfma64"])
@pytest.mark.parametrize("form,dim,k", HIGH)
def test_high_degrees(form, dim, k, strategy):
    # the rest of the degree sweep (2D P7, P8; 3D P5): action and VJP, several patches and a
    # ragged tail (2D n=6: 72 cells; 3D n=2: 48 cells)
    n = 6 if dim == 2 else 2
    mesh = meshgen.make_mesh(dim, n, k, None, np.random.default_rng(400 + k))
    u, v = inputs(form, mesh, 90 + k)
    qd = qdeg(form, k)
    say(f"[high] form={form} dim={dim} k={k} n={n} cells={mesh.n_cell} qd={qd} strat={strategy}")
    plan = fx.Plan.from_mesh(form, mesh, qd, params_for(form))
    apply_strategy(plan, strategy, form, dim)
    fam = plan.quad_family_name
    y = plan.action(gpu(u)).cpu().numpy()
    ref = oracle.action(form, mesh, u, qd, params_for(form), family=fam)
    emax, el2 = rel_err(y, ref)
    assert emax < TOL and el2 < TOL, ("action", emax, el2)
    g = vjp_or_skip(plan, gpu(u), gpu(v)).cpu().numpy()
    gref = oracle.vjp(form, mesh, u, v, qd, params_for(form), family=fam)
    emax, el2 = rel_err(g, gref)
    assert emax < TOL and el2 < TOL, ("vjp", emax, el2)


@pytest.mark.parametrize("name", ["mass_p2_2d", "nh_p4_2d", "elast_p2_3d"])
def test_action_once_matches_oracle(name):
    w = meshgen.workload(name, n=8 if name != "elast_p2_3d" else 3)
    say(f"[once] {name} cells={w.mesh.n_cell}")
    m = w.mesh
    y = fx.action_once(w.form, m.dim, m.k, w.quad_degree, m.coords, m.cell_verts, m.cell_nodes,
                       m.n_node, w.params, gpu(w.u)).cpu().numpy()
    ref = oracle.action(w.form, m, w.u, w.quad_degree, w.params, family=plan_family(w))
    emax, el2 = rel_err(y, ref)
    assert emax < TOL and el2 < TOL, (emax, el2)


@pytest.mark.parametrize("strategy", [fx.SCATTER_PATCH, fx.SCATTER_COLOUR])
def test_kernel_timing_counts_calls_and_leaves_results(strategy):
    w = meshgen.workload("nh_p4_2d", n=24)
    say(f"[timing] nh_p4_2d n=24 strategy={strategy}")
    plan = fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params)
    plan.set_strategy(strategy)
    u = gpu(w.u)
    y0 = plan.action(u)
    plan.set_timing(True)
    for _ in range(5):
        y1 = plan.action(u)
    ms, n = plan.timing()
    assert n == 5 and ms > 0.0
    assert torch.equal(y0, y1)
    plan.set_timing(False)
    plan.action(u)
    assert plan.timing() == (0.0, 0)


@pytest.mark.parametrize("form,dim,k", [c for c in CASES if c[0] in HYPERELASTIC])
def test_conical_rule_parity(form, dim, k):
    """The hyperelastic operators depend on the rule: both families against the oracle."""
    n = 7 if dim == 2 else 2
    mesh = meshgen.make_mesh(dim, n, k, None, np.random.default_rng(300 + k))
    u, v = inputs(form, mesh, 70 + k)
    qd = qdeg(form, k)
    plan = fx.Plan.from_mesh(form, mesh, qd, params_for(form))
    plan.set_quadrature(fx.QUAD_CONICAL)
    say(f"[conical] form={form} dim={dim} k={k} nq={plan.n_quad}")
    y = plan.action(gpu(u)).cpu().numpy()
    g = plan.vjp(gpu(u), gpu(v)).cpu().numpy()
    assert max(rel_err(y, oracle.action(form, mesh, u, qd, params_for(form), family="conical"))) < TOL
    assert max(rel_err(g, oracle.vjp(form, mesh, u, v, qd, params_for(form), family="conical"))) < TOL


@pytest.mark.parametrize("form", HYPERELASTIC)
@pytest.mark.parametrize("dim,k,n", [(2, 4, 6), (3, 2, 2)])
def test_jvp_is_tangent_action(form, dim, k, n):
    """(dA/du) w from fem_action_jvp: equal to the VJP (the hyperelastic tangents are
    symmetric), to the oracle's literal transpose, and to central differences of the
    residual along w (h = 1e-6)."""
    mesh = meshgen.make_mesh(dim, n, k, None, np.random.default_rng(400 + k))
    u, w = inputs(form, mesh, 90 + k)
    qd = qdeg(form, k)
    say(f"[jvp] form={form} dim={dim} k={k} n={n}")
    plan = fx.Plan.from_mesh(form, mesh, qd, params_for(form))
    ut, wt = gpu(u), gpu(w)
    jw = plan.jvp(ut, wt)
    assert torch.equal(jw, plan.vjp(ut, wt))
    ref = oracle.vjp(form, mesh, u, w, qd, params_for(form), family=plan.quad_family_name)
    assert max(rel_err(jw.cpu().numpy(), ref)) < TOL
    h = 1e-6
    fd = ((plan.action(ut + h * wt) - plan.action(ut - h * wt)) / (2 * h)).cpu().numpy()
    assert np.max(np.abs(fd - ref)) < 1e-6 * np.max(np.abs(ref))


@pytest.mark.parametrize("block", [64, 128, 256])
def test_block_sizes_bitwise_identical(block):
    w = meshgen.workload("nh_p4_2d", n=24)
    say(f"[block] nh_p4_2d n=24 block={block}")
    plan = fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params)
    plan.set_strategy(fx.SCATTER_COLOUR)
    u = gpu(w.u)
    y0 = plan.action(u).cpu().numpy()
    plan.set_block(block)
    y1 = plan.action(u).cpu().numpy()
    assert np.array_equal(y0, y1)


@pytest.mark.parametrize("strategy", STRATS, ids=STRAT_IDS)
def test_determinism_and_stream(strategy):
    w = meshgen.workload("elast_p2_3d", n=6)
    say(f"[determinism] elast_p2_3d n=6 {strategy}")
    plan = fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params)
    apply_strategy(plan, strategy, w.form, w.mesh.dim)
    u = gpu(w.u)
    y0 = plan.action(u)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        y1 = plan.action(u)
    s.synchronize()
    assert torch.equal(y0, y1)


def test_colouring_matches_host_and_oracle():
    w = meshgen.workload("nh_p4_2d", n=20)
    plan = fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params)
    col = plan.colouring()
    ocol, nc = oracle.colouring(w.mesh.cell_nodes, w.mesh.n_node)
    assert np.array_equal(col, ocol) and plan.n_colours == nc


def test_empty_mesh_and_unused_nodes():
    mesh = meshgen.unit_square(3, 2)
    say("[edge] empty mesh")
    empty = fx.Plan(fx.FORM_MASS, 2, 2, 4, mesh.coords, mesh.cell_verts[:0], mesh.cell_nodes[:0],
                    mesh.n_node)
    y = empty.action(gpu(np.ones(mesh.n_node)))
    assert torch.count_nonzero(y).item() == 0
    say("[edge] unused nodes")
    extra = 5
    plan = fx.Plan(fx.FORM_ELASTICITY, 2, 2, 2, mesh.coords, mesh.cell_verts, mesh.cell_nodes,
                   mesh.n_node + extra, LAME)
    u = np.random.default_rng(0).uniform(-1, 1, (mesh.n_node + extra) * 2)
    out = gpu(np.full(len(u), 7.0))
    plan.action(gpu(u), out=out)
    y = out.cpu().numpy()
    assert np.all(y[-2 * extra:] == 0)
    ref = oracle.action(1, mesh, u[:-2 * extra], 2, LAME, family=plan.quad_family_name)
    assert rel_err(y[:-2 * extra], ref)[0] < TOL


def test_single_cell_and_ragged_counts():
    for n in (1, 2, 5, 33):
        mesh = meshgen.unit_square(n, 3, 0.1, np.random.default_rng(n))
        if n == 1:
            mesh.cell_verts = mesh.cell_verts[:1]
            mesh.cell_nodes = mesh.cell_nodes[:1]
        u, _ = inputs(0, mesh, n)
        say(f"[ragged] mass P3 n={n} cells={mesh.n_cell}")
        plan = fx.Plan.from_mesh(0, mesh, 6)
        y = plan.action(gpu(u)).cpu().numpy()
        ref = oracle.action(0, mesh, u, 6, family=plan.quad_family_name)
        assert rel_err(y, ref)[0] < TOL


FULL = ["mass_p2_2d", "nh_p4_2d", "elast_p2_3d", "nh_vjp_p4_2d", "mass_p2_2d_1024", "svk_p4_2d",
        "nh_p4_2d_curved", "mass_p2_2d_1024_curved"]
_ref_cache = {}


@pytest.mark.parametrize("strategy", [(fx.SCATTER_PATCH, 0, 0), (fx.SCATTER_PATCH, 128, 1),
                                      (fx.SCATTER_COLOUR, 0, 0), (fx.SCATTER_PATCH, 84, 3),
                                      (fx.SCATTER_PATCH, 64, 2), (fx.SCATTER_PATCH, 64, 4)],
                         ids=["patch", "patch128x1", "colour", "patch84x3", "patch64x2", "mfma64"])
@pytest.mark.parametrize("name", FULL)
def test_full_size_against_oracle(name, strategy):
    """Every output of the full-size workloads against the oracle (seconds on the host)."""
    if name not in _ref_cache:
        _ref_cache.clear()
        w = meshgen.workload(name)
        fam = plan_family(w)
        if w.form == fx.FORM_NEOHOOKEAN:
            assert oracle.min_det_f(w.mesh, w.u, w.quad_degree, family=fam) > 0.5
        if w.v is not None:
            ref = oracle.vjp(w.form, w.mesh, w.u, w.v, w.quad_degree, w.params, family=fam)
        else:
            ref = oracle.action(w.form, w.mesh, w.u, w.quad_degree, w.params, family=fam)
        _ref_cache[name] = (w, ref)
    w, ref = _ref_cache[name]
    say(f"[full] {name} cells={w.mesh.n_cell} dofs={w.n_dof} {strategy}")
    plan = fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params)
    assert plan.quad_family_name == plan_family(w)
    apply_strategy(plan, strategy, w.form, w.mesh.dim)
    if w.v is not None:
        out = vjp_or_skip(plan, gpu(w.u), gpu(w.v)).cpu().numpy()
    else:
        out = plan.action(gpu(w.u)).cpu().numpy()
    emax, el2 = rel_err(out, ref)
    say(f"[full] {name} rel_max={emax:.3e} rel_l2={el2:.3e}")
    assert emax < TOL and el2 < TOL


def test_autograd_function_matches_oracle_vjp():
    w = meshgen.workload("nh_p4_2d", n=16)
    say("[autograd] nh_p4_2d n=16")
    plan = fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params)
    u = gpu(w.u).requires_grad_(True)
    rng = np.random.default_rng(3)
    v = rng.uniform(-1, 1, w.n_dof)
    y = fx.FemAction.apply(u, plan)
    (y * gpu(v)).sum().backward()
    fam = plan.quad_family_name
    ref = oracle.vjp(w.form, w.mesh, w.u, v, w.quad_degree, w.params, family=fam)
    assert rel_err(u.grad.cpu().numpy(), ref)[0] < TOL
    assert rel_err(y.detach().cpu().numpy(),
                   oracle.action(w.form, w.mesh, w.u, w.quad_degree, w.params, family=fam))[0] < TOL


def test_autograd_gradcheck_tiny():
    mesh = meshgen.unit_square(2, 2, 0.1, np.random.default_rng(4))
    u, _ = inputs(2, mesh, 4)
    plan = fx.Plan.from_mesh(2, mesh, 4, NH)
    say("[gradcheck] nh P2 2x2")
    ut = gpu(u).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: fx.FemAction.apply(x, plan), (ut,), eps=1e-6,
                                    atol=1e-7, rtol=1e-6)


@pytest.mark.parametrize("n,ncols", [(4, None), (16, 64)])
def test_vjp_against_assembled_jacobian_transpose(n, ncols):
    """J by central differences (h = 1e-6) of the GPU residual, column by column (all
    columns at 4x4, a seeded sample of 64 at 16x16); (J^T v)_i = v . J[:, i] against the
    VJP kernel."""
    w = meshgen.workload("nh_p4_2d", n=n)
    say(f"[jacobian] nh_p4_2d n={n}")
    plan = fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params)
    rng = np.random.default_rng(5)
    v = rng.uniform(-1, 1, w.n_dof)
    cols = np.arange(w.n_dof) if ncols is None else rng.choice(w.n_dof, ncols, replace=False)
    h = 1e-6
    ut, vt = gpu(w.u), gpu(v)
    jtv = np.zeros(len(cols))
    for j, i in enumerate(cols):
        e = torch.zeros(w.n_dof, dtype=torch.float64, device=DEV)
        e[i] = h
        jtv[j] = torch.dot(vt, (plan.action(ut + e) - plan.action(ut - e)) / (2 * h)).item()
    g = plan.vjp(ut, vt).cpu().numpy()[cols]
    assert np.max(np.abs(jtv - g)) < 1e-6 * np.max(np.abs(g))


def test_tuner_picks_a_candidate_and_keeps_parity(tmp_path):
    w = meshgen.workload("nh_p4_2d", n=32)
    say("[tune] nh_p4_2d n=32")
    plan = fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params)
    u = gpu(w.u)
    cache = tmp_path / "tune.json"
    res = plan.tune(u, cache_path=str(cache))
    assert len(res) >= 6
    best = min(res, key=lambda r: r[5])
    st, pc, ln, sm = plan.strategy()
    assert st == int(best[0])
    if st == fx.SCATTER_PATCH:
        assert (pc, ln, sm) == (int(best[1]), int(best[2]), int(best[4]))
    y = plan.action(u).cpu().numpy()
    ref = oracle.action(w.form, w.mesh, w.u, w.quad_degree, w.params, family=plan.quad_family_name)
    assert rel_err(y, ref)[0] < TOL
    assert cache.exists() and "f2/d2/k4/q8" in cache.read_text()


def test_cost_model_prunes_and_keeps_parity():
    w = meshgen.workload("nh_p4_2d", n=32)
    say("[tune-pruned] nh_p4_2d n=32")
    plan = fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params)
    pred = plan.tune_predict()
    assert len(pred) >= 6 and all(np.isfinite(r[5]) and r[5] > 0 for r in pred)
    # colour launches (one per colour, scattered read-add-writes) never beat patches here
    best_colour = min(r[5] for r in pred if r[0] == fx.SCATTER_COLOUR)
    best_patch = min(r[5] for r in pred if r[0] == fx.SCATTER_PATCH)
    assert best_patch < best_colour
    u = gpu(w.u)
    res = plan.tune(u, max_timed=3)
    assert 1 <= len(res) <= 4          # the model's three, plus the entry configuration
    y = plan.action(u).cpu().numpy()
    ref = oracle.action(w.form, w.mesh, w.u, w.quad_degree, w.params, family=plan.quad_family_name)
    assert rel_err(y, ref)[0] < TOL


def _batch_meshes(n_mesh=9, seed=11):
    """An uneven mix of the three batch forms at sizes the oracle handles quickly."""
    return meshgen.batch_workloads(n_mesh=n_mesh, seed=seed, lo=20, hi=600)


def test_batch_matches_oracle_and_per_mesh():
    ws = _batch_meshes()
    say("[batch] " + ", ".join(f"{w.name}:{w.mesh.n_cell}" for w in ws))
    plans = [fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params) for w in ws]
    us = [gpu(w.u) for w in ws]
    ys = [torch.full_like(u, 3.0) for u in us]
    b = fx.Batch(plans, us, ys)
    assert b.n_groups == 3
    for graph in (False, True, True, True):
        for y in ys:
            y.fill_(3.0)
        b.run(graph=graph)
        torch.cuda.synchronize()
        for w, p, u, y in zip(ws, plans, us, ys):
            ref = oracle.action(w.form, w.mesh, w.u, w.quad_degree, w.params,
                                family=p.quad_family_name)
            assert rel_err(y.cpu().numpy(), ref)[0] < TOL, w.name
            assert torch.equal(y, p.action(u)), w.name        # bitwise the per-mesh result
    b.close()


def test_batch_matrix_core_scalar_forms():
    """The batch's matrix-core variant for the scalar forms (mass P3 triangles, Helmholtz P2
    and Laplace P1 tetrahedra, all set to the matrix-core kernel): each mesh against the
    oracle and bitwise against its own fem_action."""
    rng = np.random.default_rng(21)
    meshes = [(fx.FORM_MASS, meshgen.unit_square(7, 3, 0.1, rng)),
              (fx.FORM_MASS, meshgen.unit_square(4, 3, 0.1, rng)),
              (fx.FORM_HELMHOLTZ, meshgen.unit_cube(3, 2, 0.05, rng)),
              (fx.FORM_LAPLACE, meshgen.unit_cube(4, 1, 0.05, rng))]
    plans, us, ys, refs = [], [], [], []
    for form, mesh in meshes:
        qd = qdeg(form, mesh.k)
        plan = fx.Plan.from_mesh(form, mesh, qd)
        plan.set_strategy(fx.SCATTER_PATCH, 64, 4, fx.SUM_COLOURED)
        u = rng.uniform(-1, 1, mesh.n_node)
        plans.append(plan)
        us.append(gpu(u))
        ys.append(torch.full_like(us[-1], 3.0))
        refs.append(oracle.action(form, mesh, u, qd, family=plan.quad_family_name))
    say("[batch mfma scalar] " + ", ".join(f"{f}:{m.n_cell}" for f, m in meshes))
    b = fx.Batch(plans, us, ys)
    assert b.n_groups == 3
    for graph in (False, True, True):
        for y in ys:
            y.fill_(3.0)
        b.run(graph=graph)
        torch.cuda.synchronize()
        for p, u, y, ref in zip(plans, us, ys, refs):
            assert rel_err(y.cpu().numpy(), ref)[0] < TOL
            assert torch.equal(y, p.action(u))
    b.close()


def test_batch_rebind_vectors():
    ws = _batch_meshes(n_mesh=4, seed=12)
    plans = [fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params) for w in ws]
    us = [gpu(w.u) for w in ws]
    ys = [torch.empty_like(u) for u in us]
    b = fx.Batch(plans, us, ys)
    b.run()
    us2 = [2.0 * u for u in us]
    ys2 = [torch.empty_like(u) for u in us]
    fx.lib().fem_batch_set_vectors(b._h,
                                   (ctypes.c_void_p * 4)(*[u.data_ptr() for u in us2]),
                                   (ctypes.c_void_p * 4)(*[y.data_ptr() for y in ys2]))
    b.run()
    torch.cuda.synchronize()
    for p, u, y in zip(plans, us2, ys2):
        assert torch.equal(y, p.action(u))


def test_batch_holds_its_plans():
    """While a batch holds a plan, the calls that would free or replace the arrays its
    descriptors and graph point at are refused (host-side checks) and leave the plan as it
    was; after the batch is destroyed they work again."""
    ws = _batch_meshes(n_mesh=3, seed=13)
    plans = [fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params) for w in ws]
    us = [gpu(w.u) for w in ws]
    ys = [torch.empty_like(u) for u in us]
    b = fx.Batch(plans, us, ys)
    b.run()
    torch.cuda.synchronize()
    before = [y.clone() for y in ys]
    p = plans[0]
    st = p.strategy()
    L = fx.lib()
    assert L.fem_plan_set_quadrature(p.handle, fx.QUAD_CONICAL) == fx.E_ARG
    assert L.fem_plan_set_strategy(p.handle, fx.SCATTER_COLOUR, 0, 0, 0) == fx.E_ARG
    assert L.fem_plan_destroy(p.handle) == fx.E_ARG
    assert b"held by a batch" in L.fem_last_error()
    with pytest.raises(fx.FemError):
        p.tune(us[0])
    assert p.strategy() == st
    b.run()
    torch.cuda.synchronize()
    assert all(torch.equal(a, y) for a, y in zip(before, ys))
    b.close()
    p.set_strategy(fx.SCATTER_COLOUR)
    p.close()


@pytest.mark.parametrize("form,dim,k", CASES)
def test_wave_priority_only_on_spill_free_kernels(form, dim, k):
    """The hinted variant of a coloured-sum patch kernel runs only where the compiled kernel
    has no scratch memory; curved cells and the element-buffer sums never take it."""
    mesh = meshgen.make_mesh(dim, 2, k, None, np.random.default_rng(7))
    plan = fx.Plan.from_mesh(form, mesh, qdeg(form, k), params_for(form))
    lanes = [1] + ([2] if dim == 2 and form not in fx.SCALAR_FORMS else []) + \
        ([3] if dim == 3 and form not in fx.SCALAR_FORMS else []) + [4]
    for ln in lanes:
        for mode in ((fx.SUM_COLOURED,) if ln == 4 else (fx.SUM_ELEMENT, fx.SUM_COLOURED)):
            plan.set_strategy(fx.SCATTER_PATCH, 63 if ln == 3 else 64, ln, mode)
            for vjp in (False, True):
                info = plan.kernel_info(vjp)
                say(f"[prio] form={form} dim={dim} k={k} lanes={ln} mode={mode} vjp={vjp} {info}")
                assert info["registers"] > 0
                if info["wave_priority"]:
                    assert info["scratch_bytes"] == 0 and mode == fx.SUM_COLOURED


def test_spilling_tangent_kernels_are_refused():
    """A hyperelastic tangent (VJP) kernel that spills to scratch is not run: the VJP on
    such a configuration fails with FEM_E_UNSUPPORTED (the action still runs), the default
    configuration's tangent kernel uses no scratch, and the tuner never keeps a refused one."""
    mesh = meshgen.make_mesh(3, 2, 4, None, np.random.default_rng(17))
    u, v = inputs(fx.FORM_NEOHOOKEAN, mesh, 18)
    plan = fx.Plan.from_mesh(fx.FORM_NEOHOOKEAN, mesh, 8, NH)
    assert plan.kernel_info(vjp=True)["scratch_bytes"] == 0
    g_default = plan.vjp(gpu(u), gpu(v))
    plan.set_strategy(fx.SCATTER_PATCH, 64, 1, fx.SUM_ELEMENT)
    assert plan.kernel_info(vjp=True)["scratch_bytes"] > 0
    y = plan.action(gpu(u)).cpu().numpy()
    assert rel_err(y, oracle.action(fx.FORM_NEOHOOKEAN, mesh, u, 8, NH,
                                    family=plan.quad_family_name))[0] < TOL
    with pytest.raises(fx.FemError) as e:
        plan.vjp(gpu(u), gpu(v))
    assert e.value.status == fx.E_UNSUPPORTED and "scratch" in str(e.value)
    plan.tune(gpu(u), v=gpu(v))
    assert plan.kernel_info(vjp=True)["scratch_bytes"] == 0
    g = plan.vjp(gpu(u), gpu(v)).cpu().numpy()
    ref = oracle.vjp(fx.FORM_NEOHOOKEAN, mesh, u, v, 8, NH, family=plan.quad_family_name)
    assert rel_err(g, ref)[0] < TOL and rel_err(g_default.cpu().numpy(), ref)[0] < TOL


def test_tangent_needing_more_lds_than_a_workgroup_is_refused():
    """3D P6 neo-Hookean on 64-cell patches of a 3^3-cube mesh: the largest patch holds
    3231 nodes, so the matrix-core tangent kernel, which stages u and v, would need 168,016
    bytes of LDS (> 160 KB) while the action (one vector) fits.  The plan is created and its
    action runs against the oracle; the VJP fails with FEM_E_UNSUPPORTED naming the LDS; a
    VJP tuning run, in which no configuration runs, fails the same way and leaves the plan's
    configuration as it was."""
    mesh = meshgen.unit_cube(3, 6, 0.05, np.random.default_rng(1))
    st = fx.check_patch_layout(fx.FORM_NEOHOOKEAN, mesh, 64)
    assert st["lds_bytes"] > 160 * 1024
    u, v = inputs(fx.FORM_NEOHOOKEAN, mesh, 19)
    say(f"[lds] nh 3D P6 cells={mesh.n_cell} max_patch_nodes={st['max_patch_nodes']}")
    plan = fx.Plan.from_mesh(fx.FORM_NEOHOOKEAN, mesh, 12, NH)
    plan.set_strategy(fx.SCATTER_PATCH, 64, 4, fx.SUM_COLOURED)
    before = plan.strategy()
    y = plan.action(gpu(u)).cpu().numpy()
    assert rel_err(y, oracle.action(fx.FORM_NEOHOOKEAN, mesh, u, 12, NH,
                                    family=plan.quad_family_name))[0] < TOL
    with pytest.raises(fx.FemError) as e:
        plan.vjp(gpu(u), gpu(v))
    assert e.value.status == fx.E_UNSUPPORTED and "LDS" in str(e.value)
    with pytest.raises(fx.FemError) as e:
        plan.tune(gpu(u), v=gpu(v))
    assert e.value.status == fx.E_UNSUPPORTED
    assert plan.strategy() == before
