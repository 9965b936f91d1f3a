"""The K = 144 scale point of the 2000/3000-face pair (52.7 M nonzeros, past
the row-tile limit: every short row runs in chunks, the kernel without
tiles) is too large for the whole oracle.  One Jacobi iteration (Sec. 3.2,
Eq. (D)) is checked there on sampled variables: every row of a sampled
variable is minimised by the oracle's row routine at the GPU's starting
multipliers (re-projected onto dual feasibility in FP64), the damped
min-marginal step and the averaging are applied in FP64, and the result
must equal the GPU's multipliers of that variable to FP32 rounding."""
import numpy as np
import pytest
import torch

from gpu_common import dm, np_, say
from oracle import oracle as O
from synth import make_pair

pytestmark = pytest.mark.gpu


def test_one_iteration_on_sampled_variables_at_k144():
    p = make_pair(5, 0, k=144)
    dev = torch.device("cuda", 0)
    D = lambda a: torch.from_numpy(a).to(dev)
    ctx = dm().Context(0)
    cxy, cyx = ctx.knn_candidates(D(p.DX), D(p.DY), 144, "bf16")
    ctx.build_product_space(D(p.VX), D(p.FX), D(p.VY), D(p.FY), cxy, cyx)
    cost = ctx.build_costs(D(p.DX), D(p.DY), "bf16")
    info = ctx.info
    say(f"[k144] |P|={info['n_prod_tri']} free={info['n_free']} nnz={info['nnz']} rows={info['n_rows']}")
    assert info["nnz"] > (24 << 20)   # beyond the row-tile limit
    omega = 0.5
    lam0 = ctx.init_lambda("fp32")
    lam1, _ = ctx.dual_solve(lam0.clone(), 1, omega)
    torch.cuda.synchronize()
    rp = np_(ctx.get_space("rrow_ptr"))
    rv = np_(ctx.get_space("rent_var"))
    rc = np_(ctx.get_space("rent_coef"))
    rb = np_(ctx.get_space("rrow_b"))
    fv = np_(ctx.get_space("free_var"))
    nfree = len(fv)
    c = np_(cost).astype(np.float64)[fv]
    l0 = np_(lam0).astype(np.float64)
    l1 = np_(lam1).astype(np.float64)
    del lam0, lam1
    deg = np.bincount(rv, minlength=nfree)
    # the records hold s = lam0 and every reader re-projects: lambda = s + (c - sum s) / |J|
    proj0 = l0 + ((c - np.bincount(rv, weights=l0, minlength=nfree)) / deg)[rv]
    order = np.argsort(rv, kind="stable")
    starts = np.searchsorted(rv[order], np.arange(nfree + 1))
    rng = np.random.default_rng(3)
    sample = rng.choice(nfree, 300, replace=False)
    cmax = float(np.abs(c).max())
    err = 0.0
    long_rows = 0
    for v in sample:
        ents = order[starts[v]:starts[v + 1]]
        s_new = np.empty(len(ents))
        for k, e in enumerate(ents):
            r = int(np.searchsorted(rp, e, side="right") - 1)
            a, b = int(rp[r]), int(rp[r + 1])
            long_rows += b - a > 64
            _, M, _ = O.row_dp(rc[a:b], int(rb[r]), proj0[a:b])
            s_new[k] = proj0[e] - omega * M[e - a]
        ref = s_new + (c[v] - s_new.sum()) / len(ents)
        err = max(err, float(np.abs(ref - l1[ents]).max()))
    say(f"  300 sampled variables ({long_rows} projection rows among their rows): max error / c_max {err / cmax:.2e}")
    assert long_rows > 0
    assert err <= 1e-4 * cmax
