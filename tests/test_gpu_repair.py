"""Local exact repair of a primal (dm_repair_primal; Appendix "Coarse-to-fine
solving strategy": the confident part of an assignment stays fixed and the
rest is solved exactly).  The repaired x is checked for exact feasibility
(the library's check, the oracle's and a from-scratch check of the matching
constraints) and for its objective, and the objective is compared with
HiGHS's MILP optimum of the same neighbourhood problem, rebuilt here from
the full constraint rows and the definition of the neighbourhood."""
import numpy as np
import pytest
import torch

from gpu_common import both, dm, np_, say
from helpers import matching_violations
from oracle import oracle as O
from synth import make_pair

pytestmark = pytest.mark.gpu


def neighbourhood(rp, ev, nc, viol_rows, hops):
    """Elements freed after `hops` steps: step 1 takes the elements of the
    violated rows, each further step the elements of the closedness rows
    (rows below nc) that touch the elements taken so far."""
    nrows = len(rp) - 1
    rows = np.zeros(nrows, bool)
    rows[viol_rows] = True
    row_of = np.repeat(np.arange(nrows), np.diff(rp))
    elems = np.zeros(int(ev.max()) + 1, bool)
    for h in range(hops):
        if h > 0:
            touch = np.zeros(nrows, bool)
            np.logical_or.at(touch, row_of, elems[ev])
            rows |= touch & (np.arange(nrows) < nc)
        elems[ev[rows[row_of]]] = True
    return elems


def highs_neighbourhood_optimum(rp, ev, ec, rb, cost, fixed_val, free):
    """min cost.x over the free elements with every other element held at
    fixed_val, subject to all rows (HiGHS MILP); None if infeasible."""
    from scipy.optimize import Bounds, LinearConstraint, milp
    from scipy.sparse import csr_matrix
    row_of = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    fe = free[ev]
    fixed_sum = np.bincount(row_of, weights=np.where(fe, 0, ec * fixed_val[ev]), minlength=len(rb))
    rhs = rb - fixed_sum
    rows_f = np.unique(row_of[fe])
    untouched = np.setdiff1d(np.arange(len(rb)), rows_f)
    if np.any(rhs[untouched] != 0):
        return None
    idx = np.nonzero(free)[0]
    col = -np.ones(len(free), np.int64)
    col[idx] = np.arange(len(idx))
    rmap = -np.ones(len(rb), np.int64)
    rmap[rows_f] = np.arange(len(rows_f))
    A = csr_matrix((ec[fe].astype(float), (rmap[row_of[fe]], col[ev[fe]])), shape=(len(rows_f), len(idx)))
    res = milp(cost[idx], constraints=LinearConstraint(A, rhs[rows_f], rhs[rows_f]),
               integrality=np.ones(len(idx)), bounds=Bounds(0, 1), options={"time_limit": 120})
    if res.status != 0:
        return None
    return float(res.fun + cost[~free] @ fixed_val[~free])


def _rows(ctx):
    g = lambda n: np_(ctx.get_space(n)).astype(np.int64)
    return g("row_ptr"), g("ent_var"), g("ent_coef"), g("row_b")


def _violated(rp, ev, ec, rb, x):
    row_of = np.repeat(np.arange(len(rb)), np.diff(rp))
    return np.nonzero(np.bincount(row_of, weights=ec * x[ev], minlength=len(rb)) != rb)[0]


def test_repair_of_a_damaged_matching_equals_highs():
    p = make_pair(2, 0)
    S, ctx = both(p, 16, "fp64")
    lam, _ = ctx.dual_solve(ctx.init_lambda("fp64"), 200, 0.5)
    x, pobj, feas, _ = ctx.round_primal(lam, seed=0)
    assert feas
    # a feasible x comes back unchanged
    xa, pa, fa, ha, _ = ctx.repair_primal(x.clone(), msg_prec="fp64")
    assert fa and ha == 0 and torch.equal(xa, x) and abs(pa - pobj) <= 1e-12 * abs(pobj)
    lb_before, info_before = ctx.lower_bound(lam), dict(ctx.info)
    # damage it: drop three selected elements
    xs = np_(x).astype(np.int64)
    sel = np.nonzero(xs)[0]
    drop = np.random.default_rng(7).choice(sel, 3, replace=False)
    xd = xs.copy()
    xd[drop] = 0
    rp, ev, ec, rb = _rows(ctx)
    viol = _violated(rp, ev, ec, rb, xd)
    say(f"  damaged matching: {len(viol)} violated rows")
    assert len(viol) > 0
    xr, pr, fr, hops, nfree = ctx.repair_primal(torch.from_numpy(xd.astype(np.uint8)), max_hops=8, max_nodes=2000,
                                                msg_prec="fp64")
    say(f"  repaired in {hops} steps ({nfree} free elements): objective {pr:.10f} (rounded {pobj:.10f})")
    assert fr
    xrs = np_(xr)
    cost = S.get("cost")
    assert ctx.check_primal(xr) == 0 and S.check_primal(xrs) == 0
    assert matching_violations(S.get("pv"), S.get("code"), len(p.FX), len(p.FY), xrs) == 0
    assert abs(pr - float(cost @ xrs.astype(np.float64))) <= 1e-12 * abs(pr)
    # the same neighbourhood problem by HiGHS
    state = np_(ctx.get_space("state")).astype(np.int64)
    free = neighbourhood(rp, ev, ctx.info["n_closed_full"], viol, hops) & (state < 0)
    fixed_val = np.where(state >= 0, state, xd)
    ref = highs_neighbourhood_optimum(rp, ev, ec, rb, cost, fixed_val, free)
    say(f"  HiGHS on the neighbourhood ({int(free.sum())} free): {ref}")
    assert ref is not None and abs(pr - ref) <= 1e-9 * abs(ref)
    # the problem the context held is back
    assert dict(ctx.info) == info_before and ctx.lower_bound(lam) == lb_before


def test_repair_at_the_largest_pair():
    """2000/3000-face pair after 1000 Jacobi iterations: the rounding leaves
    a few rows violated; the repair returns a feasible matching within 1 % of
    the certified bound."""
    p = make_pair(5, 0)
    dev = torch.device("cuda", 0)
    D = lambda a: torch.from_numpy(a).to(dev)
    ctx = dm().Context(0)
    cxy, cyx = ctx.knn_candidates(D(p.DX), D(p.DY), p.spec.k, "bf16")
    ctx.build_product_space(D(p.VX), D(p.FX), D(p.VY), D(p.FY), cxy, cyx)
    cost = np_(ctx.build_costs(D(p.DX), D(p.DY), "bf16")).astype(np.float64)
    lam, _ = ctx.dual_solve(ctx.init_lambda("fp32"), 1000, 0.5)
    lb = ctx.lower_bound(lam.double())
    x, pobj, feas, _ = ctx.round_primal(lam, rounds=10, seed=0)
    rp, ev, ec, rb = _rows(ctx)
    xd = np_(x).astype(np.int64)
    viol = _violated(rp, ev, ec, rb, xd)
    say(f"  rounding: feasible {feas}, {len(viol)} violated rows")
    xr, pr, fr, hops, nfree = ctx.repair_primal(x.clone(), max_hops=8)
    say(f"  repair: feasible {fr} in {hops} steps ({nfree} free), objective {pr:.6f}, bound {lb:.6f}, "
        f"gap {(pr - lb) / pr:.5f}")
    assert fr and (pr - lb) / pr <= 1e-2 and pr >= lb
    xrs = np_(xr)
    assert ctx.check_primal(xr) == 0
    assert len(_violated(rp, ev, ec, rb, xrs.astype(np.int64))) == 0
    assert matching_violations(np_(ctx.get_space("pv")), np_(ctx.get_space("code")), len(p.FX), len(p.FY), xrs) == 0
    assert abs(pr - float(cost @ xrs.astype(np.float64))) <= 1e-6 * abs(pr)
    if len(viol):
        state = np_(ctx.get_space("state")).astype(np.int64)
        free = neighbourhood(rp, ev, ctx.info["n_closed_full"], viol, hops) & (state < 0)
        ref = highs_neighbourhood_optimum(rp, ev, ec, rb, cost, np.where(state >= 0, state, xd), free)
        say(f"  HiGHS on the neighbourhood ({int(free.sum())} free): {ref}")
        if ref is not None:
            assert pr >= ref - 1e-6 * abs(ref)


def test_quasi_newton_resumes_across_a_repair():
    """The repair rebuilds the problem it found, so a quasi-Newton session
    resumes after it exactly as without it."""
    p = make_pair(1, 0, desc_noise=1.0)
    S, ctx = both(p, 16, "fp32")
    ref = dm().Context(0)
    ref.build_product_space(p.VX, p.FX, p.VY, p.FY, *O.knn(p.DX, p.DY, 16))
    ref.build_costs(torch.from_numpy(p.DX), torch.from_numpy(p.DY), "fp32")
    a = ctx.lbfgs_solve(ctx.init_lambda("fp32"), 10)[0]
    b = ref.lbfgs_solve(ref.init_lambda("fp32"), 10)[0]
    assert torch.equal(a, b)
    x, _, feas, _ = ctx.round_primal(a, seed=0)
    xd = np_(x).copy()
    xd[np.nonzero(xd)[0][:2]] = 0   # a damaged primal to repair
    _, pr, fr, hops, _ = ctx.repair_primal(torch.from_numpy(xd), max_hops=4)
    say(f"  repair between the solves: feasible {fr}, {hops} steps")
    a2, tra = ctx.lbfgs_solve(a, 10, resume=True)[:2]
    b2, trb = ref.lbfgs_solve(b, 10, resume=True)[:2]
    assert torch.equal(a2, b2) and torch.equal(tra, trb)
