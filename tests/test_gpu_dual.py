"""GPU costs, multipliers, Jacobi dual iterations and bounds against the FP64
oracle.

Tolerances:
* FP64 messages: the GPU and the oracle evaluate the same recursions in a
  different order (sorted prefix sums vs a partial-sum recursion, projection
  onto dual feasibility vs explicit averaging), so values agree to rounding,
  1e-10 relative on bounds after hundreds of iterations.
* FP32 messages: relative 1e-5 on the per-iteration bound (the stated
  tolerance for the FP32 bound), multipliers compared in absolute terms
  against the cost scale.
* costs: FP64 1e-12, FP32 1e-5, BF16 2e-2 relative.
"""
import numpy as np
import pytest
import torch

from gpu_common import both, dm, np_, rel_err, say
from oracle import oracle as O
from synth import make_pair

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg,prec,tol", [(1, "fp64", 1e-12), (2, "fp32", 1e-5), (2, "bf16", 2e-2),
                                          (3, "bf16", 2e-2), (3, "fp32", 1e-5)])
def test_costs(cfg, prec, tol):
    p = make_pair(cfg, 1)
    S, ctx = both(p, p.spec.k, prec)
    c = np_(ctx.build_costs(torch.from_numpy(p.DX), torch.from_numpy(p.DY), prec))
    ref = S.get("cost")
    err = rel_err(c.astype(np.float64), ref)
    say(f"  cost {prec}: max rel err {err:.3e} (float32 output)")
    # the output tensor is float32: its own rounding is 6e-8
    assert err <= max(tol, 1.2e-7)


def test_mixed_areas():
    p = make_pair(2, 0)
    ctx = dm().Context(0)
    for V, F in [(p.VX, p.FX), (p.VY, p.FY)]:
        a = np_(ctx.mixed_areas(V, F))
        assert rel_err(a, O.mixed_areas(V, F)) <= 1e-12


def test_init_lambda():
    p = make_pair(1, 0)
    S, ctx = both(p, 6)
    lam64 = np_(ctx.init_lambda("fp64"))
    assert rel_err(lam64, S.init_lambda()) <= 1e-15
    lam32 = np_(ctx.init_lambda("fp32"))
    assert rel_err(lam32, S.init_lambda()) <= 1e-7


@pytest.mark.parametrize("cfg,over,K,iters", [(1, {}, 6, 200), (1, {"desc_noise": 1.0}, 16, 150),
                                              (1, {"desc_noise": 0.3}, 6, 100)])
def test_dual_fp64_parity(cfg, over, K, iters):
    p = make_pair(cfg, 0, **over)
    S, ctx = both(p, K, "fp64")
    lam, tr = ctx.dual_solve(ctx.init_lambda("fp64"), iters, 0.5)
    rlam, rtr = S.dual_solve(iters)
    e_tr = rel_err(np_(tr), rtr)
    scale = np.abs(rlam).max()
    e_lam = float(np.abs(np_(lam) - rlam).max() / scale)
    say(f"  fp64 iters={iters}: bound rel err {e_tr:.2e}, lambda err {e_lam:.2e}, "
        f"bound {rtr[0]:.6f} -> {rtr[-1]:.6f}")
    assert e_tr <= 1e-10
    assert e_lam <= 1e-8
    assert abs(ctx.lower_bound(lam) - S.lower_bound(rlam)) <= 1e-10 * abs(rtr[-1])


@pytest.mark.parametrize("cfg,over,K,iters", [(2, {}, 16, 60), (1, {"desc_noise": 1.0}, 16, 300),
                                              (2, {"desc_noise": 0.5}, 16, 40), (2, {}, 16, 1000)])
def test_dual_fp32_parity(cfg, over, K, iters):
    p = make_pair(cfg, 0, **over)
    S, ctx = both(p, K, "fp32")
    lam, tr = ctx.dual_solve(ctx.init_lambda("fp32"), iters, 0.5)
    rlam, rtr = S.dual_solve(iters)
    e_tr = rel_err(np_(tr), rtr)
    cscale = float(S.get("cost").max())
    e_lam = float(np.abs(np_(lam).astype(np.float64) - rlam).max() / cscale)
    say(f"  fp32 iters={iters}: bound rel err {e_tr:.2e}, lambda err/cmax {e_lam:.2e}, "
        f"bound {rtr[0]:.6f} -> {rtr[-1]:.6f}")
    assert e_tr <= 1e-5
    assert e_lam <= 1e-4


def test_dual_full_size_largest_pair():
    # largest workload at full size: one build, three iterations, bound per
    # iteration and multipliers against the oracle
    p = make_pair(5, 0)
    S, ctx = both(p, p.spec.k, "fp32")
    say(f"  |P|={ctx.info['n_prod_tri']} nnz={ctx.info['nnz']}")
    lam, tr = ctx.dual_solve(ctx.init_lambda("fp32"), 3, 0.5)
    rlam, rtr = S.dual_solve(3)
    assert rel_err(np_(tr), rtr) <= 1e-5
    cscale = float(S.get("cost").max())
    assert float(np.abs(np_(lam).astype(np.float64) - rlam).max() / cscale) <= 1e-4


def test_warm_start_and_determinism():
    p = make_pair(1, 0, desc_noise=1.0)
    S, ctx = both(p, 16, "fp32")
    a, tra = ctx.dual_solve(ctx.init_lambda("fp32"), 40, 0.5)
    b, trb = ctx.dual_solve(ctx.init_lambda("fp32"), 40, 0.5)
    assert torch.equal(a, b) and torch.equal(tra, trb)
    c, _ = ctx.dual_solve(ctx.init_lambda("fp32"), 25, 0.5)
    c, trc = ctx.dual_solve(c, 15, 0.5)
    # resuming from the exported multipliers continues the same iteration
    assert rel_err(np_(trc), np_(tra)[25:]) <= 1e-6
    # dual feasibility of the exported multipliers
    rv = S.get("rent_var")
    sums = np.bincount(rv, weights=np_(a).astype(np.float64), minlength=S.info["n_free"])
    cf = S.get("cost")[S.get("free_var")]
    assert np.max(np.abs(sums - cf) / (1 + cf)) <= 1e-5


def test_bound_never_exceeds_lp():
    from scipy.optimize import linprog
    from scipy.sparse import csr_matrix
    p = make_pair(1, 0, desc_noise=1.0)
    S, ctx = both(p, 16, "fp64")
    lam, tr = ctx.dual_solve(ctx.init_lambda("fp64"), 200, 0.5)
    rp, rv, rc, rb = S.get("rrow_ptr"), S.get("rent_var"), S.get("rent_coef"), S.get("rrow_b")
    rows = np.repeat(np.arange(len(rb)), np.diff(rp))
    A = csr_matrix((rc.astype(float), (rows, rv)), shape=(len(rb), S.info["n_free"]))
    res = linprog(S.get("cost")[S.get("free_var")], A_eq=A, b_eq=rb, bounds=(0, 1), method="highs")
    lp = res.fun + S.offset
    assert np.all(np_(tr) <= lp + 1e-9 * abs(lp))
