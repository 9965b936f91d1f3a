"""GPU quasi-Newton layer (Sec. 4.1, Alg. 1) against the FP64 oracle.

Tolerances:
* subgradient: with FP64 messages the minimiser of every row is the oracle's
  (the inputs are continuous, so rows have no ties); with FP32 messages a row
  may pick another minimiser only when its objective is within FP32 rounding
  of the row minimum, so every GPU choice is checked for feasibility and for
  its objective, and the rows that differ are counted.
* direction: FP64 1e-12 relative to the largest entry (dots are FP64 on both
  sides, summed in different orders); FP32 messages 1e-5.
* full iterations with FP64 messages: the search decisions compare bounds that
  differ by far more than rounding on the instances used, so the trajectory is
  the oracle's: bounds 1e-9 relative, step sizes 1e-9, the same steps taken.
* full iterations with FP32 messages: the decisions may flip, so properties:
  dual feasibility, the trace ends at the bound of the returned multipliers,
  the bound beats the same number of plain Jacobi iterations.
"""
import numpy as np
import pytest
import torch

from gpu_common import both, dm, np_, rel_err, say
from oracle import oracle as O
from synth import make_pair

pytestmark = pytest.mark.gpu


def _perturbed(S, seed, scale=0.05):
    """A feasible lambda away from c/deg: add a per-variable zero-mean perturbation."""
    lam = S.init_lambda()
    rng = np.random.default_rng(seed)
    z = rng.normal(size=len(lam)) * scale
    rv = S.get("rent_var")
    mean = np.bincount(rv, weights=z, minlength=S.info["n_free"]) / np.bincount(rv)
    return lam + z - mean[rv]


def _row_checks(rp, coef, b, g, lam):
    """Per row: the assignment satisfies the row, and its objective."""
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    lhs = np.bincount(rows, weights=coef * g, minlength=len(rp) - 1)
    obj = np.bincount(rows, weights=g * lam, minlength=len(rp) - 1)
    return np.array_equal(lhs.astype(np.int64), b.astype(np.int64)), obj


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_subgradient_parity(prec):
    p = make_pair(1, 0, desc_noise=1.0)
    S, ctx = both(p, 16, "fp64")
    lam = _perturbed(S, 3)
    dt = torch.float64 if prec == "fp64" else torch.float32
    lam_t = torch.from_numpy(lam).to(dt).cuda()
    lam_seen = np_(lam_t).astype(np.float64)   # the oracle sees the same values
    g, lb = ctx.subgradient(lam_t)
    g = np_(g).astype(np.float64)
    gref = S.subgradient(lam_seen)
    _, rowmin, _ = S.min_marginals(lam_seen)
    rp, coef, b = S.get("rrow_ptr"), S.get("rent_coef"), S.get("rrow_b")
    ok, obj = _row_checks(rp, coef, b, g, lam_seen)
    assert ok, "a row's assignment violates its constraint"
    scale = np.abs(lam_seen).max()
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    differ = np.unique(rows[g != gref])
    say(f"  {prec}: rows {len(rp) - 1}, rows with another minimiser {len(differ)}, "
        f"bound {lb:.9f} vs {S.lower_bound(lam_seen):.9f}")
    if prec == "fp64":
        assert len(differ) == 0
        assert abs(lb - S.lower_bound(lam_seen)) <= 1e-12 * abs(lb)
        assert np.abs(obj - rowmin).max() <= 1e-12 * scale
    else:
        assert len(differ) <= max(2, (len(rp) - 1) // 1000)
        assert np.abs(obj - rowmin).max() <= 1e-5 * scale
        assert abs(lb - S.lower_bound(lam_seen)) <= 1e-5 * abs(lb)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("h", [0, 1, 3, 5])
def test_direction_parity(prec, h):
    p = make_pair(1, 1)
    S, ctx = both(p, 6, "fp64")
    nnz = S.info["nnz"]
    rng = np.random.default_rng(10 + h)
    Y = rng.integers(-1, 2, size=(h, nnz)).astype(np.int8)
    Sv = 0.01 * Y + 0.002 * rng.normal(size=(h, nnz))      # s^T y > 0
    g = rng.integers(0, 2, size=nnz).astype(np.uint8)
    dt = torch.float64 if prec == "fp64" else torch.float32
    S_t = torch.from_numpy(Sv).to(dt).cuda()
    S_seen = np_(S_t).astype(np.float64)
    d = np_(ctx.lbfgs_direction(S_t, torch.from_numpy(Y).cuda(), torch.from_numpy(g).cuda()))
    ref = S.project_feasible(O.lbfgs_direction(S_seen, Y.astype(np.float64), g.astype(np.float64)))
    err = np.abs(d - ref).max() / np.abs(ref).max()
    say(f"  h={h} {prec}: max err {err:.2e} (scale {np.abs(ref).max():.3e})")
    assert err <= (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("cfg,over,K,iters,m", [(1, {"desc_noise": 1.0}, 16, 10, 5),
                                                (1, {"desc_noise": 1.0}, 16, 6, 0),
                                                (2, {"desc_noise": 0.5}, 16, 4, 5)])
def test_lbfgs_fp64_parity(cfg, over, K, iters, m):
    p = make_pair(cfg, 0, **over)
    S, ctx = both(p, K, "fp64")
    lam, tr, gm, tk = ctx.lbfgs_solve(ctx.init_lambda("fp64"), iters, history=m)
    rlam, rtr, rgm, rtk = S.lbfgs_solve(iters, m=m)
    tr, gm, tk = np_(tr), np_(gm), np_(tk)
    say(f"  iters={iters} m={m}: bound {rtr[0]:.6f} -> {rtr[-1]:.6f}, steps taken {int(rtk.sum())}, "
        f"bound err {rel_err(tr, rtr):.2e}, gamma err {rel_err(gm, rgm):.2e}")
    assert np.array_equal(tk, rtk)
    assert rel_err(tr, rtr) <= 1e-9
    assert rel_err(gm, rgm) <= 1e-9
    assert np.abs(np_(lam) - rlam).max() <= 1e-8 * np.abs(rlam).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_zero_step_is_plain_mma(prec):
    """gamma0 = 0: no step is ever taken and the iteration is the Jacobi sweep;
    the multipliers are bit-identical to dm_dual_solve's, and so are the row
    minima behind the bounds (the bound totals are summed by different
    one-block kernels, in a different fixed order)."""
    p = make_pair(1, 0, desc_noise=1.0)
    S, ctx = both(p, 16, "fp64")
    lam, tr, gm, tk = ctx.lbfgs_solve(ctx.init_lambda(prec), 7, gamma0=0.0)
    lam_j, tr_j = ctx.dual_solve(ctx.init_lambda(prec), 7, 0.5)
    assert not np_(tk).any()
    assert torch.equal(lam, lam_j)
    assert rel_err(np_(tr[:7]), np_(tr_j)) <= 1e-13


def test_lbfgs_fp32_properties():
    p = make_pair(1, 0, desc_noise=1.0)
    S, ctx = both(p, 16, "fp32")
    lam, tr, gm, tk = ctx.lbfgs_solve(ctx.init_lambda("fp32"), 60)
    tr = np_(tr)
    _, rtr = S.dual_solve(60)
    _, otr, _, _ = S.lbfgs_solve(60)
    rv = S.get("rent_var")
    c = S.get("cost")[S.get("free_var")]
    sums = np.bincount(rv, weights=np_(lam).astype(np.float64), minlength=S.info["n_free"])
    say(f"  fp32 60 iters: bound {tr[0]:.4f} -> {tr.max():.4f} (oracle L-BFGS {otr.max():.4f}, "
        f"Jacobi {rtr.max():.4f}), steps taken {int(np_(tk).sum())}")
    assert np.abs(sums - c).max() <= 1e-5 * c.max()
    assert abs(tr[-1] - ctx.lower_bound(lam)) <= 1e-6 * abs(tr[-1])
    # the quasi-Newton steps beat plain Jacobi clearly on this instance
    best_gap_j = otr.max() - rtr.max()
    assert tr.max() >= rtr.max() + 0.5 * best_gap_j


def test_lbfgs_edge_cases():
    p = make_pair(1, 0, desc_noise=1.0)
    S, ctx = both(p, 16, "fp64")
    lam0 = ctx.init_lambda("fp64")
    lam, tr, gm, tk = ctx.lbfgs_solve(lam0.clone(), 0)
    assert torch.equal(lam, lam0) or torch.allclose(lam, lam0, rtol=0, atol=1e-15)
    assert abs(float(tr[0]) - S.lower_bound(S.init_lambda())) <= 1e-12 * abs(float(tr[0]))
    for bad in ({"history": -1}, {"max_search": 0}, {"step_up": 1.0}, {"step_down": 1.0},
                {"omega": 0.0}, {"gamma0": -1.0}):
        with pytest.raises(dm().DMError):
            ctx.lbfgs_solve(lam0.clone(), 2, **bad)


def test_subgradient_full_size_sampled():
    """Largest pair at full size: every row's GPU assignment satisfies its row;
    on a sample of rows its objective equals the oracle's row minimum,
    computed row by row."""
    p = make_pair(5, 0)
    import paper_2310_08230_amd as m
    ctx = m.Context(0)
    cxy, cyx = ctx.knn_candidates(torch.from_numpy(p.DX), torch.from_numpy(p.DY), p.spec.k, "bf16")
    ctx.build_product_space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    ctx.build_costs(torch.from_numpy(p.DX), torch.from_numpy(p.DY), "bf16")
    lam = ctx.init_lambda("fp32")
    lam, _, _, _ = ctx.lbfgs_solve(lam, 3)
    g, lb = ctx.subgradient(lam)
    rp = np_(ctx.get_space("rrow_ptr")).astype(np.int64)
    coef = np_(ctx.get_space("rent_coef")).astype(np.int64)
    b = np_(ctx.get_space("rrow_b")).astype(np.int64)
    lam_h = np_(lam).astype(np.float64)
    g = np_(g).astype(np.int64)
    ok, obj = _row_checks(rp, coef, b, g, lam_h)
    say(f"  config 5: rows {len(rp) - 1}, nnz {len(g)}, bound {lb:.4f}")
    assert ok
    rng = np.random.default_rng(0)
    for j in rng.choice(len(rp) - 1, size=300, replace=False):
        sl = slice(rp[j], rp[j + 1])
        v, _, _ = O.row_dp(coef[sl], int(b[j]), lam_h[sl])
        assert abs(obj[j] - v) <= 1e-5 * max(1.0, abs(v))


def test_resume_continues_the_search():
    """Four iterations, then six resumed, follow the ten-iteration run (FP64)."""
    p = make_pair(1, 0, desc_noise=1.0)
    S, ctx = both(p, 16, "fp64")
    lam, tr, gm, tk = ctx.lbfgs_solve(ctx.init_lambda("fp64"), 10)
    lam2, tr_a, gm_a, tk_a = ctx.lbfgs_solve(ctx.init_lambda("fp64"), 4)
    lam2, tr_b, gm_b, tk_b = ctx.lbfgs_solve(lam2, 6, resume=True)
    tr_s = np.concatenate([np_(tr_a)[:4], np_(tr_b)])
    say(f"  one call {np_(tr)[-1]:.9f}, resumed {tr_s[-1]:.9f}")
    assert rel_err(tr_s, np_(tr)) <= 1e-9
    assert rel_err(np.concatenate([np_(gm_a), np_(gm_b)]), np_(gm)) <= 1e-9
    assert np.array_equal(np.concatenate([np_(tk_a), np_(tk_b)]), np_(tk))
    assert np.abs(np_(lam2) - np_(lam)).max() <= 1e-9 * np.abs(np_(lam)).max()
    # resuming with another history length is refused
    with pytest.raises(dm().DMError):
        ctx.lbfgs_solve(lam2, 2, history=3, resume=True)
