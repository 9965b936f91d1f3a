"""A context reuses the device blocks its earlier calls freed (by size
class, on its own stream).  Rebuilding different problems in one context,
and switching the context to another stream between builds, must give
bit-identical arrays, multipliers and bound traces to fresh contexts."""
import pytest
import torch

from gpu_common import dm, say
from synth import make_pair

pytestmark = pytest.mark.gpu


def _run(ctx, cfg):
    p = make_pair(cfg, 0)
    dev = torch.device("cuda", 0)
    D = lambda a: torch.from_numpy(a).to(dev)
    cxy, cyx = ctx.knn_candidates(D(p.DX), D(p.DY), p.spec.k, "fp32")
    ctx.build_product_space(D(p.VX), D(p.FX), D(p.VY), D(p.FY), cxy, cyx)
    ctx.build_costs(D(p.DX), D(p.DY), "fp32")
    lam, tr = ctx.dual_solve(ctx.init_lambda("fp32"), 30, 0.5)
    x, pobj, feas, _ = ctx.round_primal(lam, seed=0)
    out = {"cxy": cxy, "rrow_ptr": ctx.get_space("rrow_ptr"), "rent_var": ctx.get_space("rent_var"),
           "lam": lam, "trace": tr, "x": x}
    torch.cuda.synchronize()
    return {k: v.clone() for k, v in out.items()}, (pobj, feas)


def _same(a, b):
    return all(torch.equal(a[0][k], b[0][k]) for k in a[0]) and a[1] == b[1]


def test_rebuilds_in_one_context_match_fresh_contexts():
    fresh = {cfg: _run(dm().Context(0), cfg) for cfg in (1, 2)}
    ctx = dm().Context(0)
    for cfg in (2, 1, 2, 1):
        say(f"[reuse] rebuild cfg={cfg}")
        assert _same(_run(ctx, cfg), fresh[cfg])


def test_stream_switch_between_builds():
    fresh = {cfg: _run(dm().Context(0), cfg) for cfg in (1, 2)}
    ctx = dm().Context(0)
    assert _same(_run(ctx, 2), fresh[2])
    side = torch.cuda.Stream()   # default priority
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        say("[reuse] cfg=1 on a second stream")
        r = _run(ctx, 1)
    torch.cuda.current_stream().wait_stream(side)
    assert _same(r, fresh[1])
    say("[reuse] cfg=2 back on the default stream")
    assert _same(_run(ctx, 2), fresh[2])
