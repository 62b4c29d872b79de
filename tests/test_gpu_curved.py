"""GPU parity on curved (non-affine, P2-geometry) cells: the HIP path through the C ABI
(fem_plan_create_curved) against the CPU oracle, FP64, same bar as the affine cells
(relative max and L2 error <= 1e-12)."""
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
    scale = max(np.max(np.abs(ref)), 1e-300)
    return np.max(np.abs(y - ref)) / scale, np.linalg.norm(y - ref) / max(np.linalg.norm(ref), 1e-300)


def gpu(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def params_for(form):
    if form in fx.SCALAR_FORMS:
        return ()
    return LAME if form == fx.FORM_ELASTICITY else NH



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
    if form in (fx.FORM_NEOHOOKEAN, fx.FORM_SVK):
        u = meshgen.nh_displacement(rng, mesh, 0.01 if form == fx.FORM_NEOHOOKEAN else 0.2)
        if form == fx.FORM_NEOHOOKEAN:
            # admissible under every rule a test may run at this degree
            for fam in rule_families(mesh.dim, 2 * mesh.k):
                assert oracle.min_det_f(mesh, u, 2 * mesh.k, family=fam) > 0.5
    else:
        u = rng.uniform(-1, 1, mesh.n_node * ncomp)
    return u, rng.uniform(-1, 1, mesh.n_node * ncomp)


CASES = [(f, 2, k) for f in range(6) for k in range(1, 7)] + \
        [(f, 3, k) for f in range(6) for k in range(1, 5)]
STRATS = [(fx.SCATTER_PATCH, 0, 0, 0), (fx.SCATTER_PATCH, 64, 1, fx.SUM_ELEMENT),
          (fx.SCATTER_PATCH, 128, 1, fx.SUM_COLOURED), (fx.SCATTER_COLOUR, 0, 0, 0),
          (fx.SCATTER_PATCH, 42, 3, fx.SUM_COLOURED), (fx.SCATTER_PATCH, 63, 3, fx.SUM_ELEMENT)]
STRAT_IDS = ["patch", "patch64e", "patch128c", "colour", "triple42c", "triple63e"]


@pytest.mark.parametrize("strategy", STRATS, ids=STRAT_IDS)
@pytest.mark.parametrize("form,dim,k", CASES)
def test_curved_action_and_vjp(form, dim, k, strategy):
    # 2D n=9: 162 cells; 3D n=3: 162 cells -- several patches plus a ragged tail
    n = 9 if dim == 2 else 3
    mesh = meshgen.curved(meshgen.make_mesh(dim, n, k, None, np.random.default_rng(300 + k)), 0.08)
    u, v = inputs(form, mesh, 70 + k)
    qd = 2 * k
    say(f"[curved] form={form} dim={dim} k={k} n={n} cells={mesh.n_cell} qd={qd} strat={strategy}")
    if strategy[2] == 3 and (dim != 3 or form in fx.SCALAR_FORMS):
        pytest.skip("lane triples exist for the 3D vector forms only")
    plan = fx.Plan.from_mesh(form, mesh, qd, params_for(form))
    assert plan.geometry == 2
    plan.set_strategy(*strategy)
    fam = plan.quad_family_name
    y = plan.action(gpu(u)).cpu().numpy()
    ref = oracle.action(form, mesh, u, qd, params_for(form), family=fam)
    emax, el2 = rel_err(y, ref)
    assert emax < TOL and el2 < TOL, ("action", emax, el2)
    g = vjp_or_skip(plan, gpu(u), gpu(v)).cpu().numpy()
    gref = oracle.vjp(form, mesh, u, v, qd, params_for(form), family=fam)
    emax, el2 = rel_err(g, gref)
    assert emax < TOL and el2 < TOL, ("vjp", emax, el2)


def test_curved_plan_lane_splits_and_batches():
    """Curved cells run one lane per cell or (3D vector forms) lane triples; lane pairs, the
    matrix-core kernel and batches are refused."""
    mesh = meshgen.curved(meshgen.make_mesh(3, 2, 3, None, np.random.default_rng(1)), 0.05)
    plan = fx.Plan.from_mesh(fx.FORM_ELASTICITY, mesh, 4, LAME)
    plan.set_strategy(fx.SCATTER_PATCH, 42, 3, fx.SUM_ELEMENT)
    assert plan.strategy()[2] == 3
    with pytest.raises(fx.FemError):
        plan.set_strategy(fx.SCATTER_PATCH, 64, 4, fx.SUM_COLOURED)
    u = gpu(np.zeros(mesh.n_node * 3))
    with pytest.raises(fx.FemError):
        fx.Batch([plan], [u], [torch.empty_like(u)])
    m2 = meshgen.curved(meshgen.make_mesh(2, 3, 3, None, np.random.default_rng(2)), 0.05)
    p2 = fx.Plan.from_mesh(fx.FORM_ELASTICITY, m2, 4, LAME)
    with pytest.raises(fx.FemError):
        p2.set_strategy(fx.SCATTER_PATCH, 64, 2, fx.SUM_ELEMENT)
    mass = fx.Plan.from_mesh(fx.FORM_MASS, mesh, 6)
    with pytest.raises(fx.FemError):
        mass.set_strategy(fx.SCATTER_PATCH, 42, 3, fx.SUM_COLOURED)


def test_curved_set_quadrature_and_straight_geometry():
    # straight P2 geometry through the curved path equals the affine plan (rounding only)
    m = meshgen.make_mesh(2, 6, 3, None, np.random.default_rng(5))
    ms = meshgen.curved(m, 0.0)
    u, _ = inputs(fx.FORM_NEOHOOKEAN, m, 9)
    pa = fx.Plan.from_mesh(fx.FORM_NEOHOOKEAN, m, 6, NH)
    pc = fx.Plan.from_mesh(fx.FORM_NEOHOOKEAN, ms, 6, NH)
    ya, yc = pa.action(gpu(u)).cpu().numpy(), pc.action(gpu(u)).cpu().numpy()
    assert rel_err(yc, ya)[0] < TOL
    # switching the rule family rebuilds the geometry part of the tables
    mc = meshgen.curved(m, 0.08)
    pc2 = fx.Plan.from_mesh(fx.FORM_NEOHOOKEAN, mc, 6, NH)
    pc2.set_quadrature(fx.QUAD_CONICAL)
    y = pc2.action(gpu(u)).cpu().numpy()
    ref = oracle.action(fx.FORM_NEOHOOKEAN, mc, u, 6, NH, family="conical")
    assert rel_err(y, ref)[0] < TOL


def test_curved_autograd_function_and_tuner():
    # the autograd Function's backward is the VJP on curved cells too; a tuned plan keeps
    # parity and its timing reports one call per action
    m = meshgen.curved(meshgen.make_mesh(2, 16, 4, None, np.random.default_rng(8)), 0.08)
    u0, v = inputs(fx.FORM_NEOHOOKEAN, m, 12)
    plan = fx.Plan.from_mesh(fx.FORM_NEOHOOKEAN, m, 8, NH)
    u = gpu(u0).requires_grad_(True)
    y = fx.FemAction.apply(u, plan)
    (y * gpu(v)).sum().backward()
    fam = plan.quad_family_name
    ref = oracle.vjp(fx.FORM_NEOHOOKEAN, m, u0, v, 8, NH, family=fam)
    assert rel_err(u.grad.cpu().numpy(), ref)[0] < TOL
    yref = oracle.action(fx.FORM_NEOHOOKEAN, m, u0, 8, NH, family=fam)
    assert rel_err(y.detach().cpu().numpy(), yref)[0] < TOL
    ud = gpu(u0)
    out = torch.empty_like(ud)
    plan.tune(ud, y=out)
    assert plan.strategy()[2] == 1
    plan.set_timing(True)
    for _ in range(3):
        plan.action(ud, out=out)
    ms, n = plan.timing()
    plan.set_timing(False)
    assert n == 3 and ms > 0
    assert rel_err(out.cpu().numpy(), yref)[0] < TOL


@pytest.mark.parametrize("form,k", [(fx.FORM_NEOHOOKEAN, 3), (fx.FORM_SVK, 4), (fx.FORM_ELASTICITY, 4)])
def test_curved_3d_default_takes_its_vjp(form, k):
    """Curved 3D P3/P4 vector forms default to lane triples where one lane's tangent spills
    (hyperelastic) or one lane spills (elasticity P4): the default configuration's tangent
    runs (no scratch) and its action and VJP match the oracle; a tuned plan keeps a runnable
    tangent."""
    mesh = meshgen.curved(meshgen.make_mesh(3, 2, k, None, np.random.default_rng(60 + k)), 0.06)
    u, v = inputs(form, mesh, 80 + k)
    qd = 2 * k
    plan = fx.Plan.from_mesh(form, mesh, qd, params_for(form))
    assert plan.strategy()[2] == 3
    assert plan.kernel_info(vjp=True)["scratch_bytes"] == 0
    fam = plan.quad_family_name
    y = plan.action(gpu(u)).cpu().numpy()
    assert rel_err(y, oracle.action(form, mesh, u, qd, params_for(form), family=fam))[0] < TOL
    g = plan.vjp(gpu(u), gpu(v)).cpu().numpy()
    assert rel_err(g, oracle.vjp(form, mesh, u, v, qd, params_for(form), family=fam))[0] < TOL
    if form != fx.FORM_ELASTICITY:
        plan.tune(gpu(u))
        assert plan.kernel_info(vjp=True)["scratch_bytes"] == 0
        g2 = plan.vjp(gpu(u), gpu(v)).cpu().numpy()
        assert rel_err(g2, oracle.vjp(form, mesh, u, v, qd, params_for(form), family=fam))[0] < TOL
