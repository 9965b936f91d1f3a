"""GPU confident-variable fixing (Appendix "Coarse-to-fine solving strategy")
and presolve from fixings, against the FP64 oracle.

* Fixings from the same FP64 multipliers are identical (the scores are sums
  of four or five min-marginals; the instances have no ties at the cutoff).
* The residual problem after the same fixings is identical index by index
  (integer work, bit-exact), and so is the restored problem without fixings.
* The residual solve (dual + rounding) is a heuristic: the primal found is
  checked exactly and its objective against the oracle's flow.
"""
import numpy as np
import pytest
import torch

from gpu_common import both, dm, np_, rel_err, say
from synth import make_pair

pytestmark = pytest.mark.gpu

ARRAYS = ["state", "free_var", "rrow_orig", "rrow_ptr", "rent_var", "rent_coef", "rrow_b"]


def _same_space(S, ctx):
    for name in ARRAYS:
        a = np_(ctx.get_space(name)).astype(np.int64)
        b = np.asarray(S.get(name)).astype(np.int64)
        assert np.array_equal(a, b), name


def test_confident_fixing_parity_fp64():
    p = make_pair(1, 0, desc_noise=0.5)
    S, ctx = both(p, 16, "fp64")
    lam, _, _, _ = S.lbfgs_solve(20)
    fix_g, na_g, nf_g = ctx.confident_fixing(torch.from_numpy(lam).cuda(), 0.9)
    fix_o, na_o, nf_o = S.confident_fix(lam, 0.9)
    say(f"  agreeing {na_g} (oracle {na_o}), fixed {nf_g} (oracle {nf_o})")
    assert (na_g, nf_g) == (na_o, nf_o)
    assert np.array_equal(np_(fix_g), fix_o)


def test_confident_fixing_fp32_properties():
    p = make_pair(1, 0, desc_noise=0.5)
    S, ctx = both(p, 16, "fp32")
    lam, _, _, _ = ctx.lbfgs_solve(ctx.init_lambda("fp32"), 20)
    lam64 = np_(lam).astype(np.float64)
    fix_g, na_g, nf_g = ctx.confident_fixing(lam, 0.9)
    fix_o, na_o, nf_o = S.confident_fix(lam64, 0.9)
    fix_g = np_(fix_g)
    differ = int((fix_g != fix_o).sum())
    say(f"  fp32: agreeing {na_g} vs {na_o}, fixed {nf_g} vs {nf_o}, elements fixed differently {differ}")
    assert abs(na_g - na_o) <= max(2, na_o // 500)
    # where both fix an element they agree on its value
    both_fixed = (fix_g >= 0) & (fix_o >= 0)
    assert np.array_equal(fix_g[both_fixed], fix_o[both_fixed])
    assert differ <= max(4, nf_o // 100)


def test_fix_variables_parity_and_restore():
    p = make_pair(1, 0, desc_noise=0.5)
    S, ctx = both(p, 16, "fp64")
    info0 = dict(ctx.info)
    lam, _, _, _ = S.lbfgs_solve(20)
    fix, _, _ = S.confident_fix(lam, 0.9)
    ctx.fix_variables(torch.from_numpy(fix))
    S.fix_variables(fix)
    say(f"  residual: free {ctx.info['n_free']} of {info0['n_free']}, rows {ctx.info['n_rows']}")
    assert ctx.info["n_free"] == S.info["n_free"] and ctx.info["nnz"] == S.info["nnz"]
    _same_space(S, ctx)
    # the constant of fixed-to-1 costs follows the fixings
    lam_r = ctx.init_lambda("fp64")
    assert rel_err([ctx.lower_bound(lam_r)], [S.lower_bound(S.init_lambda())]) <= 1e-12
    ctx.fix_variables(None)
    S.fix_variables(None)
    assert ctx.info == info0
    _same_space(S, ctx)


def test_infeasible_fixings_restore_the_problem():
    p = make_pair(1, 0, desc_noise=1.0)
    S, ctx = both(p, 16, "fp64")
    info0 = dict(ctx.info)
    lam, _, _, _ = S.lbfgs_solve(60)
    fix, _, _ = S.confident_fix(lam, 0.9)
    with pytest.raises(dm().DMError):
        ctx.fix_variables(torch.from_numpy(fix))
    assert ctx.info == info0
    _same_space(S, ctx)


def test_fix_and_solve_residual_matches_oracle_flow():
    p = make_pair(1, 0, desc_noise=0.5)
    S, ctx = both(p, 16, "fp64")
    lam, _, _, _ = ctx.lbfgs_solve(ctx.init_lambda("fp64"), 60)
    fix, na, nf = ctx.confident_fixing(lam, 0.9)
    ctx.fix_variables(fix)
    lam_r, _ = ctx.dual_solve(ctx.init_lambda("fp64"), 100, 0.5)
    x, pobj, feas, _ = ctx.round_primal(lam_r)
    assert feas and ctx.check_primal(x) == 0
    rlam, _, _, _ = S.lbfgs_solve(60)
    rfix, _, _ = S.confident_fix(rlam, 0.9)
    S.fix_variables(rfix)
    rlam2, _ = S.dual_solve(100)
    _, rp, rfeas, _ = S.round(rlam2)
    say(f"  fixed {nf} of {na} agreeing, residual free {ctx.info['n_free']}; p {pobj:.6f} (oracle {rp:.6f})")
    assert rfeas and abs(pobj - rp) <= 1e-9 * abs(rp)


def test_fixing_full_size():
    """Largest pair: confident fixing and the residual problem at full size;
    the problem without fixings comes back unchanged."""
    p = make_pair(5, 0)
    import paper_2310_08230_amd as m
    ctx = m.Context(0)
    DX, DY = torch.from_numpy(p.DX), torch.from_numpy(p.DY)
    cxy, cyx = ctx.knn_candidates(DX, DY, p.spec.k, "bf16")
    info0 = dict(ctx.build_product_space(p.VX, p.FX, p.VY, p.FY, cxy, cyx))
    ctx.build_costs(DX, DY, "bf16")
    lam, tr, _, _ = ctx.lbfgs_solve(ctx.init_lambda("fp32"), 20)
    fix, na, nf = ctx.confident_fixing(lam, 0.9)
    f = np_(fix)
    say(f"  config 5: free {info0['n_free']}, agreeing {na}, fixed {nf}")
    assert int((f >= 0).sum()) == info0["n_prod_tri"] - info0["n_free"] + nf
    try:
        info = ctx.fix_variables(fix)
        say(f"  residual free {info['n_free']}, rows {info['n_rows']}")
        assert info["n_free"] <= info0["n_free"] - nf
        lam_r, _ = ctx.dual_solve(ctx.init_lambda("fp32"), 100, 0.5)
        x, pobj, feas, _ = ctx.round_primal(lam_r)
        say(f"  residual rounding feasible={feas} p={pobj:.4f} bound={float(tr.max()):.4f}")
        if feas:
            assert ctx.check_primal(x) == 0
    except dm().DMError as e:
        say(f"  fixings infeasible: {e}")
    ctx.fix_variables(None)
    assert ctx.info == info0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_everything_fixed_leaves_an_empty_residual(prec):
    """Fixing every variable to a feasible primal leaves no free variable and
    no row: multipliers are empty, every solver returns the constant bound
    (the primal objective itself), and rounding returns that primal."""
    p = make_pair(1, 0)
    S, ctx = both(p, 6, "fp64")
    lam, _ = ctx.dual_solve(ctx.init_lambda(prec), 50, 0.5)
    x, pobj, feas, _ = ctx.round_primal(lam)
    assert feas
    info = ctx.fix_variables(x.to(torch.int8))
    assert info["n_free"] == 0 and info["n_rows"] == 0 and info["nnz"] == 0
    lam0 = ctx.init_lambda(prec)
    assert lam0.numel() == 0
    _, tr = ctx.dual_solve(lam0, 3, 0.5)
    assert np.allclose(np_(tr), pobj, rtol=1e-12)
    _, qtr, _, qtk = ctx.lbfgs_solve(lam0, 3)
    assert np.allclose(np_(qtr), pobj, rtol=1e-12) and not np_(qtk).any()
    assert abs(ctx.lower_bound(lam0) - pobj) <= 1e-12 * abs(pobj)
    x2, p2, feas2, _ = ctx.round_primal(lam0)
    assert feas2 and torch.equal(x2, x) and abs(p2 - pobj) <= 1e-12 * abs(pobj)
    fix, na, nf = ctx.confident_fixing(lam0, 0.9)
    assert na == 0 and nf == 0 and torch.equal(fix, x.to(torch.int8))
    ctx.fix_variables(None)
    assert ctx.info["n_free"] == S.info["n_free"]
