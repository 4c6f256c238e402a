"""hps_leaf_interior_solve_noalloc (the entry point for callers that cannot allocate)
against hps_leaf_interior_solve, through the C ABI.

The two run the same kernels, the first on the library's fixed device scratch, the
second on a caller workspace, so u_i and the backward errors must agree bitwise.
Two calls in a row, the second with fewer boxes (the scratch keeps the first call's
contents), in both precisions; plus the size limit, checked on the host.
"""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def _factored(plan, prob, ids, dev):
    from oracle import leaf as ol  # node coordinates only (the same in both runs)
    i = plan.info
    org = prob.box_origins()
    xi = np.stack([ol.box_node_coords(org[t], prob.h, prob.p)[0] for t in ids])
    bv = torch.tensor(prob.b(xi), device=dev).contiguous()
    fv = torch.tensor(prob.f(xi), device=dev).contiguous()
    nb = len(ids)
    bufs = plan.alloc(nb, dev)
    plan.hps_leaf_operators(nb, bv, bufs["A"], bufs["anorm"])
    plan.hps_leaf_factor(nb, bufs["A"], bufs["perm"], bufs["dinv"], bufs["info"])
    return bv, fv, bufs


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_noalloc_interior_solve_matches_workspace_form(gpu, precision):
    from paper_2503_04033_amd.leaf import LeafPlan
    prob = W.multi_bump((3, 2, 2), 9, 7.0, 61, gaussian_source=True, name="noalloc_p9")
    dev = torch.device("cuda")
    plan = LeafPlan(prob.p, prob.h, prob.kappa, precision)
    i = plan.info
    rng = np.random.default_rng(62)
    for nb in (prob.nbox, 5):  # the second call has fewer boxes
        say(f"noalloc {prob.name} {precision} nbox={nb}")
        ids = list(range(nb))
        bv, fv, bufs = _factored(plan, prob, ids, dev)
        ub = torch.tensor(rng.standard_normal((nb, i.n_b)), device=dev).contiguous()
        u_ws = torch.empty(nb, i.n_i, dtype=torch.float64, device=dev)
        e_ws = torch.empty(nb, dtype=torch.float64, device=dev)
        plan.hps_leaf_interior_solve(nb, bufs["A"], bufs["perm"], bufs["dinv"], bv, bufs["anorm"], fv, ub, u_ws,
                                     2, e_ws, bufs["ws"])
        u_na = torch.full((nb, i.n_i), float("nan"), dtype=torch.float64, device=dev)
        e_na = torch.full((nb,), float("nan"), dtype=torch.float64, device=dev)
        plan.hps_leaf_interior_solve_noalloc(nb, bufs["A"], bufs["perm"], bufs["dinv"], bv, bufs["anorm"], fv, ub,
                                             u_na, 2, e_na)
        torch.cuda.synchronize()
        say(f"  backward errors {e_na.cpu().numpy().tolist()}")
        assert torch.equal(u_na, u_ws)
        assert torch.equal(e_na, e_ws)
        assert float(e_na.max()) < 1e-14


def test_noalloc_rejects_more_boxes_than_the_scratch_holds(gpu):
    # the size check runs on the host before any launch; the pointers are valid buffers
    from paper_2503_04033_amd import _lib
    from paper_2503_04033_amd.leaf import LeafPlan
    plan = LeafPlan(16, (1 / 16,) * 3, 40.0, "fp32_ir")
    i = plan.info
    limit = _lib.NOALLOC_SCRATCH_BYTES // (8 * (i.n_i + 3))
    assert limit == 1526
    lib = _lib.load()
    dev = torch.device("cuda")
    buf = torch.zeros(16, dtype=torch.float64, device=dev)
    ptr = buf.data_ptr()
    st = lib.hps_leaf_interior_solve_noalloc(plan.handle, limit + 1, ptr, ptr, ptr, ptr, ptr, ptr, ptr, ptr, 0,
                                             None, None)
    assert st == _lib.HPS_EINVAL
