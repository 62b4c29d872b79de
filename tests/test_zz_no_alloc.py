"""fem_action_noalloc (the allocation-free action: shared-node partial sums in the library's
static device buffer) through the C ABI against fem_action on the same plan, which runs the
same kernels with the plan's own buffer: bitwise equal, on two calls in a row, the second
with a smaller input; and the refusal of a plan whose partial sums exceed the buffer.
Also checked against the oracle (1e-12), so the pair cannot agree on a wrong answer."""
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

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def noalloc(plan, u):
    y = torch.full_like(u, 5.0)
    st = fx.lib().fem_action_noalloc(plan.handle, ctypes.c_void_p(u.data_ptr()),
                                     ctypes.c_void_p(y.data_ptr()),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == fx.OK, fx.lib().fem_last_error()
    return y


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("first,second", [("nh_p4_2d", "mass_p2_2d"),
                                          ("mass_p2_2d_1024", "nh_p4_2d")])
def test_noalloc_matches_action_twice(first, second):
    big = meshgen.workload(first)
    small = meshgen.workload(second, n=48 if second == "nh_p4_2d" else None)
    assert small.mesh.n_cell < big.mesh.n_cell
    for w in (big, small):
        plan = fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params)
        assert plan.strategy()[0] == fx.SCATTER_PATCH
        u = torch.as_tensor(w.u, device=DEV)
        lay = fx.check_patch_layout(w.form, w.mesh, plan.strategy()[1])
        say(f"[noalloc] {w.name} cells={w.mesh.n_cell} partial slots={lay['partial_slots']}")
        assert 0 < lay["partial_slots"] * w.ncomp <= fx.NOALLOC_SCRATCH_DOUBLES
        ref = plan.action(u)
        y = noalloc(plan, u)
        torch.cuda.synchronize()
        assert torch.equal(y, ref)
        y2 = noalloc(plan, u)                   # the buffer keeps the last call's contents
        torch.cuda.synchronize()
        assert torch.equal(y2, ref)
        if w.mesh.n_cell <= 65536:
            fam = plan.quad_family_name
            want = oracle.action(w.form, w.mesh, w.u, w.quad_degree, w.params, family=fam)
            assert rel(y.cpu().numpy(), want) < 1e-12
        plan.close()


def test_noalloc_refuses_plans_beyond_the_buffer():
    w = meshgen.workload("elast_p2_3d", n=40)
    plan = fx.Plan.from_mesh(w.form, w.mesh, w.quad_degree, w.params)
    lay = fx.check_patch_layout(w.form, w.mesh, plan.strategy()[1])
    assert lay["partial_slots"] * 3 > fx.NOALLOC_SCRATCH_DOUBLES
    u = torch.as_tensor(w.u, device=DEV)
    y = torch.zeros_like(u)
    st = fx.lib().fem_action_noalloc(plan.handle, ctypes.c_void_p(u.data_ptr()),
                                     ctypes.c_void_p(y.data_ptr()), None)
    assert st == fx.E_UNSUPPORTED
    assert b"static scratch buffer" in fx.lib().fem_last_error()
    # the colour strategy needs no scratch and runs
    plan.set_strategy(fx.SCATTER_COLOUR)
    yc = noalloc(plan, u)
    torch.cuda.synchronize()
    assert torch.equal(yc, plan.action(u))
