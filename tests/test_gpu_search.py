"""GPU exact search (branch and bound on the residual of confident fixing;
Appendix "Coarse-to-fine solving strategy") against exact optima: the
depth-first enumeration of every feasible 0/1 solution on the platonic pairs,
and HiGHS's MILP on an 80-face pair with an integrality gap and on residuals
of confident fixing.  The optimum is unique as a value while several x may
attain it, so x is checked for exact feasibility and for its objective.
"""
import numpy as np
import pytest
import torch

from gpu_common import both, np_, say
from helpers import enumerate_ilp, milp_optimum, reduced_rows
from synth import make_pair, tiny_pair

pytestmark = pytest.mark.gpu


def _check_x(S, ctx, x, pobj):
    xs = np_(x)
    assert ctx.check_primal(x) == 0 and S.check_primal(xs) == 0
    assert np.isclose(pobj, float(S.get("cost") @ xs.astype(np.float64)), rtol=1e-12)


@pytest.mark.parametrize("kind,K,dn", [("tetra", 2, 0.3), ("icosa", 3, 0.5), ("octa", 3, 0.3)])
def test_search_matches_enumeration(kind, K, dn):
    p = tiny_pair(kind, kind, desc_noise=dn)
    S, ctx = both(p, K, "fp64")
    c = S.get("cost")
    opt, _, nfeas, _ = enumerate_ilp(reduced_rows(S), S.info["n_free"], c[S.get("free_var")])
    opt += S.offset
    x, pobj, bound, nodes, status = ctx.exact_search(max_nodes=500, dual_iters=50)
    say(f"  {kind}: optimum {opt:.10f} ({nfeas} feasible), search {pobj:.10f} in {nodes} nodes, {status}")
    assert status == "optimal" and abs(pobj - opt) <= 1e-9 * max(1.0, abs(opt)) and bound == pobj
    _check_x(S, ctx, x, pobj)


def test_search_closes_an_integrality_gap():
    """80-face pair with noisy descriptors (noise 1.0, K = 16): the LP bound
    is below the ILP optimum, so the search has to branch."""
    p = make_pair(1, 0, desc_noise=1.0)
    S, ctx = both(p, 16, "fp64")
    opt = milp_optimum(S)
    root = ctx.lower_bound(ctx.dual_solve(ctx.init_lambda("fp64"), 60, 0.5)[0])
    x, pobj, bound, nodes, status = ctx.exact_search(max_nodes=3000, dual_iters=60)
    say(f"  free {S.info['n_free']}: HiGHS {opt:.10f}, root bound {root:.6f}, search {pobj:.10f} "
        f"in {nodes} nodes, {status}")
    assert root < opt - 1e-3 * abs(opt)   # a real gap
    assert status == "optimal" and nodes > 1
    assert abs(pobj - opt) <= 1e-9 * abs(opt)
    _check_x(S, ctx, x, pobj)
    # a node limit returns the best primal found and a valid bound
    x2, p2, b2, n2, st2 = ctx.exact_search(max_nodes=3, dual_iters=60)
    assert st2 == "limit" and n2 == 3 and b2 <= opt + 1e-9 * abs(opt) and p2 >= opt - 1e-9 * abs(opt)
    if np.isfinite(p2):
        _check_x(S, ctx, x2, p2)


@pytest.mark.parametrize("seed,frac", [(1, 0.5), (2, 0.9)])
def test_search_on_confident_fixing_residual(seed, frac):
    p = make_pair(1, seed, desc_noise=0.7)
    S, ctx = both(p, 16, "fp64")
    lam, _, _, _ = S.lbfgs_solve(30)
    fix, na, nf = ctx.confident_fixing(torch.from_numpy(lam).cuda(), frac)
    S.fix_variables(np_(fix))
    opt = milp_optimum(S)
    x, pobj, bound, nodes, status = ctx.exact_search(base_fix=fix, max_nodes=500, dual_iters=60)
    say(f"  fixed {nf} of {na}; residual free {S.info['n_free']}: HiGHS {opt:.10f}, search {pobj:.10f} "
        f"in {nodes} nodes, {status}")
    assert status == "optimal" and abs(pobj - opt) <= 1e-9 * abs(opt)
    assert ctx.info["n_free"] == S.info["n_free"] and ctx.info["nnz"] == S.info["nnz"]   # residual in place
    _check_x(S, ctx, x, pobj)


def test_search_with_infeasible_fixings():
    """Confident fixing is a heuristic: on the gap instance, fixing 90 % of
    the agreeing variables leaves no feasible completion."""
    p = make_pair(1, 0, desc_noise=1.0)
    S, ctx = both(p, 16, "fp64")
    free = ctx.info["n_free"]
    lam, _, _, _ = S.lbfgs_solve(30)
    fix, _, _ = ctx.confident_fixing(torch.from_numpy(lam).cuda(), 0.9)
    assert milp_optimum(S) is not None
    x, pobj, bound, nodes, status = ctx.exact_search(base_fix=fix, max_nodes=50, dual_iters=20)
    assert status == "infeasible" and pobj == np.inf and not np_(x).any()
    assert ctx.info["n_free"] == free   # the problem without fixings is back


def test_search_rejects_bad_parameters():
    DMError = __import__("paper_2310_08230_amd").DMError
    p = tiny_pair("tetra", "tetra", desc_noise=0.3)
    S, ctx = both(p, 2, "fp64")
    for kw in (dict(max_nodes=0), dict(dual_iters=0), dict(omega=0.0), dict(rel_tol=-1.0), dict(msg_prec="bf16")):
        with pytest.raises((DMError, KeyError)):
            ctx.exact_search(**kw)
    x, pobj, _, _, status = ctx.exact_search(max_nodes=10, dual_iters=20)   # still usable
    assert status == "optimal" and ctx.check_primal(x) == 0
