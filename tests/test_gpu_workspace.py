"""Caller-owned solver state (dm_workspace_query / dm_set_workspace): with a
torch-owned buffer attached, the Jacobi solve, the bound, rounding and the
quasi-Newton solve give bit-identical results to the library's own
allocation; a buffer that is too small or misaligned is refused, and a
larger problem is refused until a larger buffer is attached."""
import pytest
import torch

from gpu_common import both, dm, np_, say
from synth import make_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg,prec", [(2, "fp32"), (1, "fp64")])
def test_torch_owned_solver_state_gives_identical_results(cfg, prec):
    p = make_pair(cfg, 0)
    S, ctx = both(p, p.spec.k, "fp64" if prec == "fp64" else "fp32")
    lam_a, tr_a = ctx.dual_solve(ctx.init_lambda(prec), 60, 0.5)
    lb_a = ctx.lower_bound(lam_a)
    x_a, p_a, f_a, _ = ctx.round_primal(lam_a, seed=1)
    q_a, qtr_a = ctx.lbfgs_solve(ctx.init_lambda(prec), 5)[:2]
    n = ctx.workspace_bytes(prec)
    ws = torch.zeros(n, dtype=torch.uint8, device="cuda")
    ctx.set_workspace(prec, ws)
    lam_b, tr_b = ctx.dual_solve(ctx.init_lambda(prec), 60, 0.5)
    torch.cuda.synchronize()
    say(f"  {prec}: workspace {n} bytes, nonzero bytes after the solve {int((ws != 0).sum())}")
    assert int((ws != 0).sum()) > 0   # the records live in the caller's buffer
    assert torch.equal(lam_a, lam_b) and torch.equal(tr_a, tr_b)
    assert ctx.lower_bound(lam_b) == lb_a
    x_b, p_b, f_b, _ = ctx.round_primal(lam_b, seed=1)
    assert torch.equal(x_a, x_b) and p_a == p_b and f_a == f_b
    q_b, qtr_b = ctx.lbfgs_solve(ctx.init_lambda(prec), 5)[:2]
    assert torch.equal(q_a, q_b) and torch.equal(qtr_a, qtr_b)
    ctx.set_workspace(prec, None)   # detached: the library allocates again
    lam_c, tr_c = ctx.dual_solve(ctx.init_lambda(prec), 60, 0.5)
    assert torch.equal(lam_a, lam_c) and torch.equal(tr_a, tr_c)


def test_workspace_refusals():
    DMError = dm().DMError
    p = make_pair(1, 0)
    S, ctx = both(p, p.spec.k, "fp32")
    n = ctx.workspace_bytes("fp32")
    assert ctx.workspace_bytes("fp64") > n
    with pytest.raises(DMError, match="needed"):
        ctx.set_workspace("fp32", torch.empty(n - 256, dtype=torch.uint8, device="cuda"))
    big = torch.empty(n + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(DMError, match="aligned"):
        ctx.set_workspace("fp32", big[1:])
    ctx.set_workspace("fp32", big)
    lam, tr = ctx.dual_solve(ctx.init_lambda("fp32"), 20, 0.5)
    # a larger problem: the attached buffer no longer suffices
    q = make_pair(2, 0)
    from oracle import oracle as O
    ctx.build_product_space(q.VX, q.FX, q.VY, q.FY, *O.knn(q.DX, q.DY, 16))
    ctx.build_costs(torch.from_numpy(q.DX), torch.from_numpy(q.DY), "fp32")
    assert ctx.workspace_bytes("fp32") > big.numel()
    with pytest.raises(DMError, match="workspace"):
        ctx.dual_solve(ctx.init_lambda("fp32"), 5, 0.5)
    ctx.set_workspace("fp32", torch.empty(ctx.workspace_bytes("fp32"), dtype=torch.uint8, device="cuda"))
    lam2, tr2 = ctx.dual_solve(ctx.init_lambda("fp32"), 5, 0.5)
    assert torch.isfinite(tr2).all()
