"""Oracle of the generic 0-1 ILP path (Appendix "Other ILPs"): padding rows,
weak duality and exactness pinned by brute-force enumeration, HiGHS and an
independent assignment solver."""
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
    # every variable is in two exactly-one rows: one padding row each
    assert S.info["n_rows_full"] == 2 * n + nv and S.info["nnz_full"] == 2 * n * n + 2 * nv
    S.set_costs(c)
    r, k = linear_sum_assignment(c.reshape(n, n))
    opt = c.reshape(n, n)[r, k].sum()
    lam, tr = S.dual_solve(200)
    assert np.all(tr <= opt + 1e-12) and opt - tr.max() < 1e-9   # the assignment polytope is integral
    x, pobj, feas, _ = S.round(lam)
    assert feas and abs(pobj - opt) < 1e-9


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
    # every full row is satisfied by the optimum's assignment; padding rows by construction
    x, pobj, feas, _ = S.round(lam, seed=1)
    if feas:
        assert S.check_primal(x) == 0 and pobj >= opt - 1e-9


def test_invalid_ilps_are_rejected():
    rp = np.array([0, 2], np.int32)
    with pytest.raises(O.OracleError):   # coefficient 2
        O.Space.from_ilp(2, rp, np.array([0, 1]), np.array([2, 1]), np.array([1]))
    with pytest.raises(O.OracleError):   # a variable twice with one sign
        O.Space.from_ilp(2, rp, np.array([0, 0]), np.array([1, 1]), np.array([1]))
    with pytest.raises(O.OracleError):   # variable 1 in no row
        O.Space.from_ilp(2, np.array([0, 1], np.int32), np.array([0]), np.array([1]), np.array([1]))
    six = np.array([0, 1] * 6).reshape(6, 2)
    with pytest.raises(O.OracleError):   # variable 0 in six rows
        O.Space.from_ilp(2, np.arange(0, 13, 2, dtype=np.int32), six.ravel(), np.ones(12, int),
                         np.ones(6, int))
