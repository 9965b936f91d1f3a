"""Pins of the oracle's subproblem minima, min-marginals, Jacobi dual ascent,
rounding and smoothed dual: exhaustive enumeration, exact LP/ILP optima
(HiGHS), invariants and finite differences."""
import itertools

import numpy as np
import pytest

from helpers import enumerate_ilp, matching_violations, reduced_rows
from oracle import oracle as O
from synth import make_pair, tiny_pair


def _enum_row(coef, b, lam, T=0.0):
    """Minimum / soft-minimum and min-marginals of one row by listing all
    2^n assignments (the definition of the subproblem S_j and of M_i)."""
    n = len(lam)
    sols = [np.array(s) for s in itertools.product((0, 1), repeat=n) if np.dot(s, coef) == b]
    vals = np.array([np.dot(s, lam) for s in sols])
    S = np.array(sols)

    def smin(v):
        if len(v) == 0:
            return np.inf
        if T == 0:
            return v.min()
        m = v.min()
        return m - T * np.log(np.exp(-(v - m) / T).sum())

    tot = smin(vals)
    M = np.array([smin(vals[S[:, i] == 1]) - smin(vals[S[:, i] == 0]) for i in range(n)])
    mu = (np.array([np.exp(-(smin(vals[S[:, i] == 1]) - tot) / T) for i in range(n)])
          if T > 0 else None)
    return tot, M, mu


@pytest.mark.parametrize("seed", range(12))
def test_row_dp_matches_enumeration(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 13))
    coef = rng.choice([-1, 1], size=n)
    P, N = int((coef > 0).sum()), int((coef < 0).sum())
    b = int(rng.integers(-N, P + 1))
    lam = rng.normal(size=n) * rng.choice([0.1, 1.0, 10.0])
    if seed % 3 == 0:
        lam[rng.integers(n)] = lam[0]    # ties
    for T in (0.0, 0.3):
        tot, M, mu = O.row_dp(coef, b, lam, T)
        rtot, rM, rmu = _enum_row(coef, b, lam, T)
        finite = np.isfinite(rM)
        assert np.isclose(tot, rtot, rtol=1e-12, atol=1e-12)
        assert np.allclose(M[finite], rM[finite], rtol=1e-10, atol=1e-10)
        if T > 0:
            assert np.allclose(mu[finite], rmu[finite], rtol=1e-10, atol=1e-12)


def test_exactly_one_row_closed_form():
    rng = np.random.default_rng(5)
    for n in (2, 3, 17, 300):
        lam = rng.normal(size=n)
        tot, M, _ = O.row_dp(np.ones(n, int), 1, lam)
        assert tot == lam.min()
        others = np.array([np.min(np.delete(lam, i)) for i in range(n)])
        assert np.array_equal(M, lam - others)
        # soft version: softmax marginals
        T = 0.2
        tot, M, mu = O.row_dp(np.ones(n, int), 1, lam, T)
        w = np.exp(-(lam - lam.min()) / T)
        assert np.allclose(mu, w / w.sum(), rtol=1e-10)
        assert np.isclose(tot, lam.min() - T * np.log(w.sum()), rtol=1e-12)


def test_damped_update_never_lowers_exactly_one_row():
    rng = np.random.default_rng(7)
    for _ in range(50):
        lam = rng.normal(size=int(rng.integers(2, 20)))
        _, M, _ = O.row_dp(np.ones(len(lam), int), 1, lam)
        for w in (0.25, 0.5, 1.0):
            new, _, _ = O.row_dp(np.ones(len(lam), int), 1, lam - w * M)
            assert new >= lam.min() - 1e-15


def _space(p, K):
    cxy, cyx = O.knn(p.DX, p.DY, K)
    S = O.Space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    S.costs(p.DX, p.DY)
    return S


def _lp_ilp(S, integral):
    from scipy.optimize import Bounds, LinearConstraint, linprog, milp
    from scipy.sparse import csr_matrix
    rows = reduced_rows(S)
    n = S.info["n_free"]
    c = S.get("cost")[S.get("free_var")]
    r = np.concatenate([[j] * len(vs) for j, (vs, _, _) in enumerate(rows)])
    A = csr_matrix((np.concatenate([cs for _, cs, _ in rows]).astype(float),
                    (r, np.concatenate([vs for vs, _, _ in rows]))), shape=(len(rows), n))
    b = np.array([b for _, _, b in rows], float)
    if integral:
        res = milp(c, constraints=LinearConstraint(A, b, b), integrality=np.ones(n),
                   bounds=Bounds(0, 1))
    else:
        res = linprog(c, A_eq=A, b_eq=b, bounds=(0, 1), method="highs")
    assert res.status == 0
    return res.fun + S.offset


def test_dual_feasibility_and_weak_duality_hard_instance():
    p = make_pair(1, 0, desc_noise=1.0)
    S = _space(p, 16)
    lam, tr = S.dual_solve(60)
    # sum_j lambda^j_i = c_i (constraint of Eq. (D))
    rp, rv = S.get("rrow_ptr"), S.get("rent_var")
    sums = np.bincount(rv, weights=lam, minlength=S.info["n_free"])
    c = S.get("cost")[S.get("free_var")]
    assert np.all(np.abs(sums - c) <= 1e-12 * (1 + c))
    lp = _lp_ilp(S, integral=False)
    # the dual optimum of (D) equals the LP relaxation: every row polytope is
    # integral, so no bound may exceed it
    assert np.all(tr <= lp + 1e-9 * abs(lp))
    assert S.lower_bound(lam) <= lp + 1e-9 * abs(lp)
    assert tr[-1] > tr[0]
    # trace entry t is the bound at the t-th iterate
    lam5, tr5 = S.dual_solve(5)
    assert np.isclose(S.lower_bound(lam5), S.dual_solve(6)[1][5], rtol=0, atol=1e-12)
    assert np.array_equal(tr5, tr[:5])


def test_bound_reaches_lp_on_small_config():
    p = make_pair(1, 0)
    S = _space(p, 6)
    lam, tr = S.dual_solve(200)
    lp = _lp_ilp(S, integral=False)
    ilp = _lp_ilp(S, integral=True)
    assert tr.max() <= lp + 1e-9 * abs(lp) and lp <= ilp + 1e-9
    assert (lp - tr.max()) / lp < 1e-6


@pytest.mark.parametrize("kind,K,dn", [("tetra", 2, 0.3), ("icosa", 3, 0.5), ("octa", 3, 0.3)])
def test_bruteforce_optimum_vs_dual_and_rounding(kind, K, dn):
    p = tiny_pair(kind, kind, desc_noise=dn)
    S = _space(p, K)
    c = S.get("cost")
    fv = S.get("free_var")
    opt, nopt, nfeas, _ = enumerate_ilp(reduced_rows(S), S.info["n_free"], c[fv])
    opt += S.offset
    assert nfeas >= 1
    milp_opt = _lp_ilp(S, integral=True)
    assert np.isclose(opt, milp_opt, rtol=1e-9)
    lam, tr = S.dual_solve(100)
    assert np.all(tr <= opt + 1e-9)          # weak duality
    x, pobj, feas, _ = S.round(lam, seed=3)
    if feas:
        assert S.check_primal(x) == 0
        assert matching_violations(S.get("pv"), S.get("code"), len(p.FX), len(p.FY), x) == 0
        assert pobj >= opt - 1e-9
        assert np.isclose(pobj, float(c @ x), rtol=1e-12)


@pytest.mark.parametrize("cfg,seed", [(1, 0), (1, 1), (1, 2), (1, 3), (1, 4)])
def test_rounding_small_config(cfg, seed):
    p = make_pair(cfg, seed)
    S = _space(p, p.spec.k)
    lam, tr = S.dual_solve(p.spec.iters)
    x, pobj, feas, rounds = S.round(lam, seed=seed)
    assert feas
    assert S.check_primal(x) == 0
    assert matching_violations(S.get("pv"), S.get("code"), len(p.FX), len(p.FY), x) == 0
    ilp = _lp_ilp(S, integral=True)
    assert pobj >= ilp - 1e-9
    gap = (pobj - tr.max()) / pobj
    assert gap <= 1e-2


def test_rounding_perturbs_hard_instance():
    # a harder instance: rounding needs perturbation rounds, and whatever it
    # returns as feasible is exactly feasible
    p = make_pair(1, 0, desc_noise=0.3)
    S = _space(p, 6)
    lam, _ = S.dual_solve(3)
    x, pobj, feas, rounds = S.round(lam, R=30, T_iters=25, seed=11)
    assert feas and S.check_primal(x) == 0


def test_splitmix64_reference_value():
    # splitmix64 of state 0 (one step of the published generator): 0xE220A8397B1DCDAF
    # uniform_pm1 maps (splitmix64(splitmix64(seed) ^ (r<<32 | i)) >> 11) to [-1, 1)
    u = O.uniform_pm1(0, 0, 0)
    z = 0xE220A8397B1DCDAF  # splitmix64(0)
    # second step applied to z ^ 0
    def mix(z):
        m = (1 << 64) - 1
        z = (z + 0x9E3779B97F4A7C15) & m
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
        return z ^ (z >> 31)
    assert mix(0) == z
    assert u == (mix(z) >> 11) * 2.0 ** -53 * 2 - 1
    vals = np.array([O.uniform_pm1(9, r, i) for r in range(3) for i in range(2000)])
    assert vals.min() >= -1 and vals.max() < 1 and abs(vals.mean()) < 0.05


# ---------------------------------------------------------------- smoothed dual
def test_smoothed_bound_brackets_hard_bound():
    p = make_pair(1, 0, desc_noise=0.3)
    S = _space(p, 6)
    lam, _ = S.dual_solve(20)
    T = 0.1
    hard = S.lower_bound(lam)
    soft = S.lower_bound(lam, T)
    rows = reduced_rows(S)
    logS = 0.0
    for vs, cs, b in rows:
        # |S_j| by counting assignments with the row's +1/-1 split
        P, N = int((cs > 0).sum()), int((cs < 0).sum())
        from math import comb
        logS += np.log(sum(comb(P, k) * comb(N, k - b) for k in range(max(0, b), P + 1)
                           if 0 <= k - b <= N))
    assert hard - T * logS - 1e-9 <= soft <= hard + 1e-12


@pytest.mark.parametrize("T", [0.1, 0.5])
def test_smoothed_gradient_finite_differences(T):
    p = make_pair(1, 1, desc_noise=0.3)
    S = _space(p, 6)
    c0 = S.get("cost")
    lam, _ = S.dual_solve(30, T=T)
    lam0 = S.init_lambda()
    phi = lam - lam0
    v, gc, gX, gY = S.smoothed_grad(lam, T, p.DX, p.DY)
    assert np.isclose(v, S.smoothed_value_phi(c0, phi, T), rtol=1e-12)
    rng = np.random.default_rng(0)
    h = 1e-3
    errs = []
    for _ in range(20):
        side = rng.integers(2)
        D = (p.DX if side == 0 else p.DY).astype(np.float64)
        i, k = rng.integers(D.shape[0]), rng.integers(D.shape[1])
        g = (gX if side == 0 else gY)[i, k]
        vals = []
        for s in (+1, -1):
            DX = p.DX.astype(np.float64).copy()
            DY = p.DY.astype(np.float64).copy()
            (DX if side == 0 else DY)[i, k] += s * h
            # float32 descriptors would round h away: evaluate costs from the
            # FP64 perturbed descriptors through the oracle's cost routine
            c = _costs64(S, p, DX, DY)
            vals.append(S.smoothed_value_phi(c, phi, T))
        fd = (vals[0] - vals[1]) / (2 * h)
        errs.append(abs(fd - g) / max(1e-3, abs(g)))
    assert max(errs) <= 1e-4


def _costs64(S, p, DX, DY):
    """Eq. (cost) on FP64 descriptors, using the oracle's mixed areas and the
    element list (the oracle's cost routine takes float32 descriptors)."""
    AX = O.mixed_areas(p.VX, p.FX)
    AY = O.mixed_areas(p.VY, p.FY)
    pv = S.get("pv")
    nvy = len(p.VY)
    m, n = pv // nvy, pv % nvy
    d = np.sqrt(((DX[m] - DY[n]) ** 2).sum(-1))
    return ((AX[m] + AY[n]) * d).sum(1)


def test_smoothed_gradient_single_row_is_softmax():
    # dL_T / dlambda for one exactly-one row is softmax(-lambda / T)
    lam = np.array([0.3, -0.2, 0.5, 0.1])
    T = 0.25
    tot, _, mu = O.row_dp(np.ones(4, int), 1, lam, T)
    h = 1e-6
    fd = np.array([(O.row_dp(np.ones(4, int), 1, lam + h * e, T)[0]
                    - O.row_dp(np.ones(4, int), 1, lam - h * e, T)[0]) / (2 * h) for e in np.eye(4)])
    w = np.exp(-lam / T)
    assert np.allclose(mu, w / w.sum(), rtol=1e-12) and np.allclose(fd, mu, rtol=1e-7)


# ---------------------------------------------------------------------------
# Quasi-Newton layer (Sec. 4.1, Alg. 1; Appendix "Quasi-Newton Updates")
# ---------------------------------------------------------------------------
def _dense_bfgs_inverse(S, Y):
    """Inverse-Hessian estimate built by the textbook BFGS update
    H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T, applied to the pairs
    oldest first from H0 = (s^T y / y^T y) I of the newest pair (Nocedal &
    Wright, Eqs. 6.17 and 7.20).  The two-loop recursion must equal H g."""
    n = S.shape[1]
    H = (S[-1] @ Y[-1]) / (Y[-1] @ Y[-1]) * np.eye(n)
    for s, y in zip(S, Y):
        rho = 1.0 / (s @ y)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    return H


@pytest.mark.parametrize("m", [1, 2, 5])
def test_lbfgs_direction_equals_dense_bfgs(m):
    rng = np.random.default_rng(m)
    n = 9
    B = rng.normal(size=(n, n))
    A = B @ B.T + n * np.eye(n)                 # SPD: y = A s gives s^T y > 0
    S = rng.normal(size=(m, n))
    Y = S @ A.T + 0.01 * rng.normal(size=(m, n))
    g = rng.normal(size=n)
    d = O.lbfgs_direction(S, Y, g)
    assert np.allclose(d, _dense_bfgs_inverse(S, Y) @ g, rtol=1e-10, atol=1e-12)
    # secant condition of the newest pair: H y_k = s_k
    assert np.allclose(O.lbfgs_direction(S, Y, Y[-1]), S[-1], rtol=1e-10, atol=1e-12)


def test_lbfgs_direction_without_history_is_identity():
    g = np.arange(7.0) - 3.0
    assert np.array_equal(O.lbfgs_direction(np.zeros((0, 7)), np.zeros((0, 7)), g), g)


def test_find_step_worked_examples():
    """FindStepSize on E(gamma) = -(gamma - c)^2 with E_init = E(0), factors
    1.1 up and 0.8 down and K = 5; the expected step sizes are worked out by
    hand from the procedure:
      c = 1,   gamma = 0.5: every trial improves and beats the best so far, so
               gamma grows five times: 0.5 * 1.1^5;
      same with Delta_min = 0.5: E(0.55) - E(0) = 0.7975 stops the search;
      c = 0.1, gamma = 1: no trial beats E(0) = -0.01, so gamma shrinks five
               times; the best trial is the last one, 0.8^5, still worse than
               E(0) (no step is taken);
      c = 1,   gamma = 1.9: trials 2.09 (worse than E_init -> shrink), 1.672
               (best), 1.8392, 2.02312 (worse than E_init -> shrink), 1.618496
               (best)."""
    gm, e = O.find_step_parabola(1.0, 0.5)
    assert np.isclose(gm, 0.5 * 1.1 ** 5, rtol=1e-14) and np.isclose(e, -(gm - 1) ** 2)
    gm, _ = O.find_step_parabola(1.0, 0.5, dmin=0.5)
    assert np.isclose(gm, 0.55, rtol=1e-14)
    gm, e = O.find_step_parabola(0.1, 1.0)
    assert np.isclose(gm, 0.8 ** 5, rtol=1e-14) and e < -0.01
    gm, _ = O.find_step_parabola(1.0, 1.9)
    assert np.isclose(gm, 1.618496, rtol=1e-12)
    # a single search step (K = 1) from the worked case above keeps 1.9
    gm, _ = O.find_step_parabola(1.0, 1.9, K=1)
    assert np.isclose(gm, 1.9, rtol=1e-14)


def _perturbed_lambda(S, seed, scale=0.05):
    """A dual-feasible lambda away from the initial point: c/deg plus a
    zero-mean (per variable) random perturbation."""
    lam = S.init_lambda()
    rng = np.random.default_rng(seed)
    z = rng.normal(size=len(lam)) * scale
    rv = S.get("rent_var")
    mean = np.bincount(rv, weights=z, minlength=S.info["n_free"]) / np.bincount(rv)
    return lam + z - mean[rv]


def test_subgradient_is_a_row_minimiser():
    p = make_pair(1, 0, desc_noise=1.0)
    S = _space(p, 16)
    lam = _perturbed_lambda(S, 3)
    g = S.subgradient(lam)
    _, rowmin, _ = S.min_marginals(lam)
    rp, coef, b = S.get("rrow_ptr"), S.get("rent_coef"), S.get("rrow_b")
    assert set(np.unique(g)) <= {0.0, 1.0}
    for j in range(S.info["n_rows"]):
        sl = slice(rp[j], rp[j + 1])
        assert int(np.dot(coef[sl], g[sl])) == b[j]
        assert abs(np.dot(g[sl], lam[sl]) - rowmin[j]) <= 1e-12 * (1 + abs(rowmin[j]))
    # short rows: the minimiser is the unique one found by enumeration
    for j in range(0, S.info["n_rows"], 7):
        n = rp[j + 1] - rp[j]
        if n > 12:
            continue
        sl = slice(rp[j], rp[j + 1])
        sols = [np.array(s) for s in itertools.product((0, 1), repeat=n)
                if np.dot(s, coef[sl]) == b[j]]
        vals = np.array([np.dot(s, lam[sl]) for s in sols])
        assert np.array_equal(g[sl], sols[int(np.argmin(vals))])


def test_subgradient_is_a_supergradient_of_the_dual():
    """E is concave: E(l') <= E(l) + g^T (l' - l) for every l', with equality
    for small steps while every row keeps its (unique) minimiser."""
    p = make_pair(1, 1, desc_noise=1.0)
    S = _space(p, 16)
    lam = _perturbed_lambda(S, 4)
    g = S.subgradient(lam)
    E = S.lower_bound(lam)
    rng = np.random.default_rng(9)
    for scale in (1e-9, 1e-3, 1e-1, 1.0):
        u = rng.normal(size=len(lam)) * scale
        assert S.lower_bound(lam + u) <= E + g @ u + 1e-10 * (1 + abs(E))
    u = rng.normal(size=len(lam)) * 1e-9
    assert np.isclose(S.lower_bound(lam + u) - E, g @ u, rtol=1e-4, atol=1e-14)


def test_lbfgs_with_zero_step_is_plain_mma():
    """With step size 0 no trial improves, so no quasi-Newton step is taken and
    the iteration reduces to the Jacobi MMA update."""
    p = make_pair(1, 0, desc_noise=1.0)
    S = _space(p, 16)
    lam, tE, tg, tk = S.lbfgs_solve(12, gamma0=0.0)
    lam_j, tr = S.dual_solve(12)
    assert not tk.any() and np.all(tg == 0.0)
    assert np.array_equal(lam, lam_j)
    assert np.array_equal(tE[:12], tr)


def test_lbfgs_feasible_bounded_and_faster_than_mma():
    p = make_pair(1, 0, desc_noise=1.0)
    S = _space(p, 16)
    lam, tE, tg, tk = S.lbfgs_solve(60, gamma0=0.1)
    rv = S.get("rent_var")
    c = S.get("cost")[S.get("free_var")]
    sums = np.bincount(rv, weights=lam, minlength=S.info["n_free"])
    assert np.all(np.abs(sums - c) <= 1e-10 * (1 + c))
    lp = _lp_ilp(S, integral=False)
    assert np.all(tE <= lp + 1e-9 * abs(lp))
    assert np.isclose(tE[-1], S.lower_bound(lam), rtol=0, atol=1e-12)
    _, tr = S.dual_solve(60)
    # the quasi-Newton steps raise the bound well beyond the same number of
    # Jacobi iterations on this instance (Sec. 4.1: faster than MMA alone)
    assert (lp - tE.max()) < 0.5 * (lp - tr.max())
    assert tk.sum() > 30


def test_feasibility_projection_is_orthogonal():
    """Alg. 1's projection removes each variable's mean: the result sums to 0
    over every variable's entries, is idempotent, and d - Pd is orthogonal to
    every feasible direction."""
    S = _space(make_pair(1, 0), 6)
    rng = np.random.default_rng(1)
    d = rng.normal(size=S.info["nnz"])
    e = S.project_feasible(d)
    rv = S.get("rent_var")
    assert np.abs(np.bincount(rv, weights=e)).max() < 1e-12
    assert np.allclose(S.project_feasible(e), e, atol=1e-15)
    f = S.project_feasible(rng.normal(size=S.info["nnz"]))
    assert abs((d - e) @ f) < 1e-10


# ---------------------------------------------------------------------------
# Confident-variable fixing (Appendix "Coarse-to-fine solving strategy")
# ---------------------------------------------------------------------------
def test_confident_selection_from_min_marginals():
    """The oracle's fixings equal a selection recomputed with numpy from its
    min-marginals: agreeing variables (all M < 0 or all M > 0), ranked by
    |sum_j M| with ties to the lower variable, the top floor(0.9 n) fixed."""
    S = _space(make_pair(1, 0, desc_noise=0.5), 16)
    lam, _, _, _ = S.lbfgs_solve(20)
    M, _, _ = S.min_marginals(lam)
    rv = S.get("rent_var")
    n = S.info["n_free"]
    neg = np.bincount(rv, weights=(M < 0), minlength=n) == np.bincount(rv, minlength=n)
    pos = np.bincount(rv, weights=(M > 0), minlength=n) == np.bincount(rv, minlength=n)
    score = np.abs(np.bincount(rv, weights=M, minlength=n))
    agree = np.nonzero(neg | pos)[0]
    order = agree[np.lexsort((agree, -score[agree]))]
    take = int(np.floor(0.9 * len(agree)))
    ref = S.get("state").astype(np.int8).copy()
    fv = S.get("free_var")
    ref[fv[order[:take]]] = np.where(neg[order[:take]], 1, 0)
    fix, na, nf = S.confident_fix(lam, 0.9)
    assert na == len(agree) and nf == take
    assert np.array_equal(fix, ref)


@pytest.mark.parametrize("kind,K,dn", [("tetra", 2, 0.3), ("octa", 3, 0.3)])
def test_fixed_residual_keeps_exactly_the_matching_solutions(kind, K, dn):
    """After fixing some variables to the values of one feasible solution, the
    residual problem's solutions are exactly the original solutions that agree
    with the fixings (exhaustive enumeration on both)."""
    p = tiny_pair(kind, kind, 8, 3, 0.01, dn)
    cxy, cyx = O.knn(p.DX, p.DY, K)
    S = O.Space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    S.costs(p.DX, p.DY)

    def solutions():
        rows = reduced_rows(S)
        sols = enumerate_ilp(rows, S.info["n_free"], np.zeros(S.info["n_free"]), limit=200000)[3]
        fv, state = S.get("free_var"), S.get("state")
        full = []
        for x in sols:
            y = (state == 1).astype(np.int8)
            y[fv] = x
            full.append(y)
        return full
    all_sols = solutions()
    assert len(all_sols) >= 1
    rng = np.random.default_rng(0)
    ref = all_sols[rng.integers(len(all_sols))]
    fv = S.get("free_var")
    pick = rng.choice(fv, size=max(1, len(fv) // 3), replace=False)
    fix = S.get("state").astype(np.int8).copy()
    fix[pick] = ref[pick]
    S.fix_variables(fix)
    got = {tuple(x) for x in solutions()}
    want = {tuple(x) for x in all_sols if np.array_equal(x[pick], ref[pick])}
    assert got == want
    S.fix_variables(None)
    assert {tuple(x) for x in solutions()} == {tuple(x) for x in all_sols}


def test_fix_and_solve_residual_reaches_the_optimum():
    """On an LP-tight pair, fixing 90 % of the agreeing variables and solving
    the residual with the same dual + rounding gives the ILP optimum (HiGHS)."""
    S = _space(make_pair(1, 0, desc_noise=0.5), 16)
    ilp = _lp_ilp(S, integral=True)
    lam, tE, _, _ = S.lbfgs_solve(60)
    fix, na, nf = S.confident_fix(lam, 0.9)
    S.fix_variables(fix)
    assert S.info["n_free"] < 0.2 * na
    lam2, _ = S.dual_solve(100)
    x, p, feas, _ = S.round(lam2)
    assert feas and S.check_primal(x) == 0
    assert abs(p - ilp) <= 1e-9 * abs(ilp)
    S.fix_variables(None)


def test_infeasible_fixings_are_reported():
    S = _space(make_pair(1, 0, desc_noise=1.0), 16)
    lam, _, _, _ = S.lbfgs_solve(60)
    fix, _, _ = S.confident_fix(lam, 0.9)
    with pytest.raises(O.OracleError):
        S.fix_variables(fix)


def test_costs_equal_eq_cost_restated():
    """The oracle's element costs equal Eq. (cost) written out here from the
    element list: c_p = sum over its three product vertices (m, n) of
    (A_X(m) + A_Y(n)) ||F_X(m) - F_Y(n)||, with the oracle's mixed areas
    (pinned above) and FP64 descriptors."""
    for cfg, seed in ((1, 0), (1, 2)):
        p = make_pair(cfg, seed)
        S = _space(p, 6)
        want = _costs64(S, p, p.DX.astype(np.float64), p.DY.astype(np.float64))
        got = S.get("cost")
        assert got.shape == want.shape and np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-300)) <= 1e-12


def test_identity_elements_cost_nothing():
    """Matching a shape onto itself with identical descriptors: every
    triangle-triangle element (f, f) with the faces aligned (rotation 0) has
    cost 0, and only those (and degenerate elements of zero-distance pairs)
    do."""
    p = make_pair(1, 0)
    cxy, cyx = O.knn(p.DX, p.DX, 6)
    S = O.Space(p.VX, p.FX, p.VX, p.FX, cxy, cyx)
    S.costs(p.DX, p.DX)
    code, cost = S.get("code"), S.get("cost")
    tt0 = (code[:, 0] == 0) & (code[:, 2] == 0) & (code[:, 1] == code[:, 3])
    assert tt0.sum() == len(p.FX) and np.all(cost[tt0] == 0.0)
    pv = S.get("pv")
    nv = len(p.VX)
    diag = np.all(pv // nv == pv % nv, axis=1)   # every product vertex (m, m)
    assert np.all(cost[~diag] > 0.0) and np.all(cost[diag] == 0.0)


def test_confident_fixing_ranks_largest_score_first():
    """Hand-worked min-marginals: two exactly-one rows over x0, x1, x2 with
    multipliers (0, 1, 5) and (0, 2, 9), so c = (0, 3, 14).  In an
    exactly-one row M_i = lambda_i - min_{k != i} lambda_k, giving
    (-1, 1, 5) and (-2, 2, 9): sums -3, 3, 14, all three agreeing (x0 -> 1,
    x1, x2 -> 0).  Largest |sum| first with ties to the lower variable:
    x2, x0, x1.  Fixing floor(0.9 * 3) = 2 takes x2 = 0 and x0 = 1;
    floor(0.34 * 3) = 1 takes x2 = 0 only.  (Smallest first would take x0
    and x1.)"""
    rp = np.array([0, 3, 6], np.int32)
    S = O.Space.from_ilp(3, rp, np.array([0, 1, 2, 0, 1, 2]), np.ones(6, int), np.array([1, 1]))
    S.set_costs(np.array([0.0, 3.0, 14.0]))
    assert S.info["n_free"] == 3
    lam = np.array([0.0, 1.0, 5.0, 0.0, 2.0, 9.0])
    M, _, _ = S.min_marginals(lam)
    assert np.allclose(M, [-1, 1, 5, -2, 2, 9], atol=0)
    fix, na, nf = S.confident_fix(lam, 0.9)
    assert (na, nf) == (3, 2) and fix.tolist() == [1, -1, 0]
    fix, na, nf = S.confident_fix(lam, 0.34)
    assert (na, nf) == (3, 1) and fix.tolist() == [-1, -1, 0]
