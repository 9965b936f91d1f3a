"""Oracle of the generic 0-1 ILP path (Appendix "Other ILPs"): the plain
decomposition of Eq. (D), one subproblem per input row, pinned by a
per-row brute-force evaluation of the dual written from the input CSR,
weak duality and exactness against brute-force enumeration, HiGHS and an
independent assignment solver."""
import itertools

import numpy as np
import pytest

from helpers import enumerate_ilp, milp_optimum, reduced_rows
from synth import generic_ilp
from oracle import oracle as O


def test_assignment_bound_reaches_the_optimum():
    from scipy.optimize import linear_sum_assignment
    n = 6
    nv, rp, cols, coefs, b, c = generic_ilp(n, 0, 1)
    S = O.Space.from_ilp(nv, rp, cols, coefs, b)
    # one subproblem per input row, nothing added: 2n exactly-one rows of n entries
    assert S.info["n_rows_full"] == 2 * n and S.info["nnz_full"] == 2 * n * n
    assert S.info["n_closed_full"] == 0
    S.set_costs(c)
    r, k = linear_sum_assignment(c.reshape(n, n))
    opt = c.reshape(n, n)[r, k].sum()
    lam, tr = S.dual_solve(200)
    assert np.all(tr <= opt + 1e-12) and opt - tr.max() < 1e-9   # the assignment polytope is integral
    x, pobj, feas, _ = S.round(lam)
    assert feas and abs(pobj - opt) < 1e-9


def _dual_by_rows(rp, cols, coefs, b, lam_of):
    """sum over input rows of min over the row's feasible 0/1 assignments of
    sum_i lam^j_i s_i, by enumeration (Eq. (D) read directly off the CSR)."""
    tot = 0.0
    for j in range(len(rp) - 1):
        vs, cs = cols[rp[j]:rp[j + 1]], coefs[rp[j]:rp[j + 1]]
        lj = np.array([lam_of(j, int(v)) for v in vs])
        best = np.inf
        for s in itertools.product((0, 1), repeat=len(vs)):
            s = np.array(s)
            if int(cs @ s) == int(b[j]):
                best = min(best, float(lj @ s))
        tot += best
    return tot


def _hand_ilp():
    """Seven variables in one, two or three rows: x0 + x1 + x2 = 1,
    x0 - x3 = 0, x1 + x3 - x4 = 0, x2 + x4 = 1, x5 + x6 - x2 = 0; three
    feasible points, and every row alone allows both values of each of its
    variables, so presolve fixes nothing."""
    rows = [([0, 1, 2], [1, 1, 1], 1), ([0, 3], [1, -1], 0), ([1, 3, 4], [1, 1, -1], 0), ([2, 4], [1, 1], 1),
            ([5, 6, 2], [1, 1, -1], 0)]
    rp = np.cumsum([0] + [len(r[0]) for r in rows]).astype(np.int32)
    cols = np.concatenate([r[0] for r in rows]).astype(np.int32)
    coefs = np.concatenate([r[1] for r in rows]).astype(np.int8)
    b = np.array([r[2] for r in rows], np.int32)
    return 7, rp, cols, coefs, b, np.linspace(0.3, 1.5, 7)


@pytest.mark.parametrize("case", ["hand", (4, 4, (2, 4), 0), (3, 3, (3, 4), 1)])
def test_dual_is_one_subproblem_per_input_row(case):
    """L(lambda) of the oracle equals the sum of per-row minima enumerated
    from the input rows for multipliers that split each cost over the
    variable's rows (here unevenly, at random), and the degrees are the
    input degrees: variables in one, two or three rows get no extra rows."""
    if case == "hand":
        nv, rp, cols, coefs, b, c = _hand_ilp()
        seed = 5
    else:
        n, ns, sl, seed = case
        nv, rp, cols, coefs, b, c = generic_ilp(n, ns, seed, side_len=sl)
    S = O.Space.from_ilp(nv, rp, cols, coefs, b)
    assert S.info["n_rows_full"] == len(b) and S.info["nnz_full"] == len(cols)
    deg_in = np.bincount(cols, minlength=nv)
    assert deg_in.min() >= 1
    if case == "hand":
        assert sorted(set(deg_in.tolist())) == [1, 2, 3]
    S.set_costs(c)
    assert S.info["n_free"] == nv   # presolve fixes nothing on these instances
    # the reduced problem keeps every input row, in the order
    # [other rows | exactly-one rows]
    eo = [j for j in range(len(b)) if np.all(coefs[rp[j]:rp[j + 1]] == 1) and b[j] == 1]
    other = [j for j in range(len(b)) if j not in eo]
    order = other + eo
    assert S.get("row_key").tolist() == order and S.get("rrow_orig").tolist() == list(range(len(b)))
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.2, 1.0, len(cols))
    share = {}
    for v in range(nv):
        ents = np.nonzero(cols == v)[0]
        for e in ents:
            share[(int(np.searchsorted(rp, e, side="right") - 1), v)] = c[v] * w[e] / w[ents].sum()
    # multipliers in the oracle's (reordered) entry order
    lam = np.array([share[(j, int(v))] for j in order for v in cols[rp[j]:rp[j + 1]]])
    assert np.allclose(np.bincount(S.get("rent_var"), weights=lam, minlength=nv), c, rtol=1e-14)
    want = _dual_by_rows(rp, cols, coefs, b, lambda j, v: share[(j, v)])
    assert abs(S.lower_bound(lam) - want) <= 1e-12 * max(1.0, abs(want))
    # the first multipliers split each cost evenly over its input rows
    lam0 = S.init_lambda()
    assert np.allclose(lam0, c[S.get("rent_var")] / deg_in[S.get("rent_var")], rtol=1e-15)
    # and the Jacobi iteration keeps every cost split (Eq. (D)'s constraint)
    lam1, _ = S.dual_solve(30)
    assert np.allclose(np.bincount(S.get("rent_var"), weights=lam1, minlength=nv), c, rtol=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_side_constrained_ilp_against_enumeration(seed):
    nv, rp, cols, coefs, b, c = generic_ilp(4, 5, seed)
    S = O.Space.from_ilp(nv, rp, cols, coefs, b)
    S.set_costs(c)
    fv = S.get("free_var")
    opt, _, nfeas, _ = enumerate_ilp(reduced_rows(S), S.info["n_free"], c[fv])
    opt += S.offset
    assert nfeas >= 1 and np.isclose(opt, milp_optimum(S), rtol=1e-9)
    lam, tr = S.dual_solve(100)
    assert np.all(tr <= opt + 1e-9)   # weak duality
    if S.info["n_free"] == 0:
        return
    # the dual optimum is the LP optimum (every single +-1 row with 0/1
    # bounds is integral), so no bound may exceed HiGHS's LP value
    from scipy.optimize import linprog
    rows = reduced_rows(S)
    A = np.zeros((len(rows), S.info["n_free"]))
    for j, (vs, cs, _) in enumerate(rows):
        A[j, vs] = cs
    lp = linprog(c[fv], A_eq=A, b_eq=[bb for _, _, bb in rows], bounds=(0, 1), method="highs")
    assert lp.status == 0 and np.all(tr <= lp.fun + S.offset + 1e-9)
    x, pobj, feas, _ = S.round(lam, seed=1)
    if feas:
        assert S.check_primal(x) == 0 and pobj >= opt - 1e-9


def test_invalid_ilps_are_rejected():
    rp = np.array([0, 2], np.int32)
    with pytest.raises(O.OracleError):   # coefficient 2
        O.Space.from_ilp(2, rp, np.array([0, 1]), np.array([2, 1]), np.array([1]))
    with pytest.raises(O.OracleError):   # a variable twice with one sign
        O.Space.from_ilp(2, rp, np.array([0, 0]), np.array([1, 1]), np.array([1]))
    with pytest.raises(O.OracleError):   # a variable twice with opposite signs
        O.Space.from_ilp(2, rp, np.array([0, 0]), np.array([1, -1]), np.array([0]))
    with pytest.raises(O.OracleError):   # variable 1 in no row
        O.Space.from_ilp(2, np.array([0, 1], np.int32), np.array([0]), np.array([1]), np.array([1]))
    six = np.array([0, 1] * 6).reshape(6, 2)
    with pytest.raises(O.OracleError):   # variable 0 in six rows
        O.Space.from_ilp(2, np.arange(0, 13, 2, dtype=np.int32), six.ravel(), np.ones(12, int),
                         np.ones(6, int))
