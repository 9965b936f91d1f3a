"""GPU generic 0-1 ILP path (Appendix "Other ILPs") against the oracle: the
full problem (one subproblem per input row, Eq. (D)) and the presolved
reduced problem are integer results and must agree exactly; FP64 bounds agree
to rounding; rounding and the exact search are checked against HiGHS."""
import numpy as np
import pytest
import torch

from gpu_common import dm, np_, rel_err, say
from helpers import milp_optimum
from synth import generic_ilp
from oracle import oracle as O

pytestmark = pytest.mark.gpu

REDUCED = ["state", "free_var", "rrow_orig", "rrow_ptr", "rent_var", "rent_coef", "rrow_b"]
FULL = ["row_ptr", "ent_var", "ent_coef", "row_b"]


def _both(n, n_side, seed):
    nv, rp, cols, coefs, b, c = generic_ilp(n, n_side, seed)
    S = O.Space.from_ilp(nv, rp, cols, coefs, b)
    S.set_costs(c)
    ctx = dm().Context(0)
    ctx.build_ilp(nv, rp, cols, coefs, b)
    ctx.set_costs(torch.from_numpy(c))
    return S, ctx, c


@pytest.mark.parametrize("n,n_side,seed", [(8, 10, 0), (20, 60, 1), (40, 200, 2)])
def test_ilp_build_matches_the_oracle(n, n_side, seed):
    S, ctx, _ = _both(n, n_side, seed)
    for k in ("n_rows_full", "nnz_full", "n_closed_full", "n_free", "n_rows", "nnz"):
        assert ctx.info[k] == S.info[k], k
    for name in FULL + REDUCED:
        assert np.array_equal(np_(ctx.get_space(name)).astype(np.int64), np.asarray(S.get(name)).astype(np.int64)), name
    assert abs(ctx.lower_bound(ctx.init_lambda("fp64")) - S.lower_bound(S.init_lambda())) <= 1e-12 * max(1, abs(S.offset))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_ilp_dual_parity(prec, tol):
    S, ctx, _ = _both(20, 60, 1)
    lam, tr = ctx.dual_solve(ctx.init_lambda(prec), 50, 0.5)
    rlam, rtr = S.dual_solve(50)
    say(f"  {prec}: bound rel err {rel_err(np_(tr), rtr):.2e}")
    assert rel_err(np_(tr), rtr) <= tol


def test_ilp_rounding_and_exact_search_reach_highs():
    S, ctx, c = _both(20, 60, 1)
    opt = milp_optimum(S)
    lam, tr = ctx.lbfgs_solve(ctx.init_lambda("fp64"), 40)[:2]
    assert float(tr.max()) <= opt + 1e-9 * abs(opt)
    x, pobj, bound, nodes, status = ctx.exact_search(max_nodes=2000, dual_iters=60)
    say(f"  HiGHS {opt:.10f}, bound {float(tr.max()):.10f}, search {pobj:.10f} in {nodes} nodes, {status}")
    assert status == "optimal" and abs(pobj - opt) <= 1e-9 * abs(opt)
    assert ctx.check_primal(x) == 0 and S.check_primal(np_(x)) == 0
    assert np.isclose(pobj, float(c @ np_(x).astype(np.float64)), rtol=1e-12)


def test_ilp_errors_and_refused_calls():
    DMError = __import__("paper_2310_08230_amd").DMError
    ctx = dm().Context(0)
    rp = np.array([0, 2], np.int32)
    with pytest.raises(DMError):   # coefficient 2
        ctx.build_ilp(2, rp, np.array([0, 1]), np.array([2, 1]), np.array([1]))
    with pytest.raises(DMError):   # a variable twice with one sign
        ctx.build_ilp(2, rp, np.array([0, 0]), np.array([1, 1]), np.array([1]))
    with pytest.raises(DMError):   # variable 1 in no row
        ctx.build_ilp(2, np.array([0, 1], np.int32), np.array([0]), np.array([1]), np.array([1]))
    # malformed row pointers (chosen so that every entry a row names is
    # still inside the arrays passed): not starting at 0, decreasing, and a
    # row ending past the entry count row_ptr[n_rows]
    for bad_rp, n_ent in (([1, 2], 2), ([0, 2, 1], 2), ([0, 3, 2], 3)):
        with pytest.raises(DMError, match="row pointers"):
            ctx.build_ilp(2, np.array(bad_rp, np.int32), np.arange(n_ent) % 2, np.ones(n_ent),
                          np.ones(len(bad_rp) - 1))
    ctx.build_ilp(2, rp, np.array([0, 1]), np.array([1, 1]), np.array([1]))   # usable afterwards
    assert ctx.info["n_prod_tri"] == 2
    S, ctx, _ = _both(8, 10, 0)
    x = torch.zeros(ctx.info["n_prod_tri"], dtype=torch.uint8, device="cuda")
    for call in (lambda: ctx.matched_pairs(x), lambda: ctx.get_space("pv"),
                 lambda: ctx.smoothed_backward(ctx.init_lambda("fp32"), 0.1, torch.zeros(4, 2), torch.zeros(4, 2))):
        with pytest.raises(DMError):
            call()
    assert ctx.check_primal(x) > 0   # still usable afterwards


def test_ilp_smoothed_dual_parity():
    """The smoothed dual on a generic ILP (side rows in the 8- and 16-lane
    soft segments, assignment rows on the exactly-one path)."""
    S, ctx, _ = _both(20, 60, 1)
    T = 0.1
    r0 = S.lower_bound(S.init_lambda(), T)
    assert abs(ctx.lower_bound(ctx.init_lambda("fp64"), T) - r0) <= 1e-13 * max(1.0, abs(r0))
    lam, tr = ctx.dual_solve(ctx.init_lambda("fp64"), 20, 0.5, T)
    rlam, rtr = S.dual_solve(20, T=T)
    say(f"  smoothed: bound rel err {rel_err(np_(tr), rtr):.2e}")
    assert rel_err(np_(tr), rtr) <= 1e-10


@pytest.mark.parametrize("seed", [4, 0])
def test_ilp_without_exactly_one_rows(seed):
    """A generic ILP whose rows are all short +-1 rows (half +1, half -1, so
    none is an exactly-one row), costs of both signs: the problem has no
    projection rows, and the sweeps, rounding, the primal check and the
    exact search run without them.  Seed 4 keeps 10 free variables and an
    integrality gap; seed 0 is decided entirely by presolve.  Bounds against
    the oracle, the optimum against HiGHS."""
    rng = np.random.default_rng(seed)
    n = 16
    planted = rng.integers(0, 2, n)
    rows, deg = [], np.zeros(n, int)
    while len(rows) < 12:
        k = int(rng.choice([2, 4, 6]))
        vs = rng.choice(n, k, replace=False)
        if np.any(deg[vs] >= 5):
            continue
        a = np.array([1] * (k // 2) + [-1] * (k // 2))
        rng.shuffle(a)
        rows.append((vs, a))
        deg[vs] += 1
    for v in range(n):   # every variable in some row
        if deg[v] == 0:
            u = next(u for u in range(n) if u != v and deg[u] < 5)
            rows.append((np.array([v, u]), np.array([1, -1])))
            deg[[v, u]] += 1
    rp = np.cumsum([0] + [len(vs) for vs, _ in rows]).astype(np.int32)
    cols = np.concatenate([vs for vs, _ in rows]).astype(np.int32)
    coefs = np.concatenate([a for _, a in rows]).astype(np.int8)
    b = np.array([int(a @ planted[vs]) for vs, a in rows], np.int32)
    c = rng.uniform(0.5, 2.0, n) * rng.choice([-1, 1], n)
    S = O.Space.from_ilp(n, rp, cols, coefs, b)
    S.set_costs(c)
    ctx = dm().Context(0)
    ctx.build_ilp(n, rp, cols, coefs, b)
    ctx.set_costs(torch.from_numpy(c))
    assert (ctx.info["n_rows"], ctx.info["nnz"], ctx.info["n_free"]) == (S.info["n_rows"], S.info["nnz"],
                                                                         S.info["n_free"])
    for name in REDUCED:
        assert np.array_equal(np_(ctx.get_space(name)).astype(np.int64),
                              np.asarray(S.get(name)).astype(np.int64)), name
    lam, tr = ctx.dual_solve(ctx.init_lambda("fp64"), 30, 0.5)
    _, rtr = S.dual_solve(30)
    assert rel_err(np_(tr), rtr) <= 1e-10
    opt = milp_optimum(S)
    assert float(np_(tr).max()) <= opt + 1e-9 * max(1.0, abs(opt))
    x, pobj, feas, _ = ctx.round_primal(lam, seed=0)
    if feas:
        assert ctx.check_primal(x) == 0 and pobj >= opt - 1e-9 * max(1.0, abs(opt))
    xs, p2, bound, nodes, status = ctx.exact_search()
    say(f"  seed {seed}: free {ctx.info['n_free']}, rows {ctx.info['n_rows']}: HiGHS {opt:.10f}, "
        f"rounding feasible {feas}, search {p2:.10f} in {nodes} nodes, {status}")
    assert status == "optimal" and abs(p2 - opt) <= 1e-9 * max(1.0, abs(opt))
    assert ctx.check_primal(xs) == 0 and S.check_primal(np_(xs)) == 0
