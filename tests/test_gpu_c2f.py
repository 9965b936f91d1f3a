"""GPU coarse-to-fine pruning (Sec. 5.2) against the oracle: nearest-vertex
maps, the matched vertex pairs of a primal and the ring candidate lists are
integer results and must agree exactly; the pruned fine problem is then
solved by the same dual + rounding."""
import numpy as np
import pytest
import torch

from gpu_common import dm, np_, say
from oracle import oracle as O
from synth import make_pair

pytestmark = pytest.mark.gpu


def _coarse_solution(ctx, p):
    DX, DY = torch.from_numpy(p.DX).cuda(), torch.from_numpy(p.DY).cuda()
    cxy, cyx = ctx.knn_candidates(DX, DY, 32, "fp32")
    ctx.build_product_space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    ctx.build_costs(DX, DY, "fp32")
    lam, tr = ctx.lbfgs_solve(ctx.init_lambda("fp32"), 40)[:2]
    x, pobj, feas, _ = ctx.round_primal(lam)
    assert feas
    return x


@pytest.mark.parametrize("rings", [1, 2])
def test_c2f_pieces_match_the_oracle(rings):
    pc, pf = make_pair(3, 0, faces_x=500, faces_y=500), make_pair(3, 0)
    ctx = dm().Context(0)
    x = _coarse_solution(ctx, pc)
    pairs = ctx.matched_pairs(x)
    rp = O.matched_pairs(np_(ctx.get_space("pv")), np_(x), len(pc.VY))
    assert np.array_equal(np_(pairs), rp)
    RXc, RXf = pc.RX.astype(np.float32), pf.RX.astype(np.float32)
    RYc, RYf = pc.RY.astype(np.float32), pf.RY.astype(np.float32)
    mx, my = ctx.nearest_vertices(RXc, RXf), ctx.nearest_vertices(RYc, RYf)
    assert np.array_equal(np_(mx), O.nearest_vertices(RXc, RXf))
    assert np.array_equal(np_(my), O.nearest_vertices(RYc, RYf))
    seeds = np.stack([np_(mx)[rp[:, 0]], np_(my)[rp[:, 1]]], 1)
    cxy, cyx = ctx.ring_candidates(pf.VX, pf.FX, pf.VY, pf.FY, seeds, rings=rings)
    oxy, oyx = O.ring_candidates(pf.FX, len(pf.VX), pf.FY, len(pf.VY), seeds, rings)
    say(f"  rings {rings}: {len(rp)} coarse pairs, fine K = {cxy.shape[1]}")
    assert np.array_equal(np_(cxy), oxy) and np.array_equal(np_(cyx), oyx)


def test_c2f_fine_level_solves():
    pc, pf = make_pair(3, 0, faces_x=500, faces_y=500), make_pair(3, 0)
    ctx = dm().Context(0)
    x = _coarse_solution(ctx, pc)
    pairs = ctx.matched_pairs(x)
    mx = ctx.nearest_vertices(pc.RX.astype(np.float32), pf.RX.astype(np.float32))
    my = ctx.nearest_vertices(pc.RY.astype(np.float32), pf.RY.astype(np.float32))
    seeds = torch.stack([mx[pairs[:, 0].long()], my[pairs[:, 1].long()]], 1)
    cxy, cyx = ctx.ring_candidates(pf.VX, pf.FX, pf.VY, pf.FY, seeds, rings=2)
    ctx.build_product_space(pf.VX, pf.FX, pf.VY, pf.FY, cxy, cyx)
    DX, DY = torch.from_numpy(pf.DX).cuda(), torch.from_numpy(pf.DY).cuda()
    ctx.build_costs(DX, DY, "fp32")
    lam, tr = ctx.lbfgs_solve(ctx.init_lambda("fp32"), 60)[:2]
    xf, pobj, feas, _ = ctx.round_primal(lam)
    gap = (pobj - float(tr.max())) / pobj
    say(f"  fine: |C| {ctx.info['n_cand']}, |P| {ctx.info['n_prod_tri']}, feasible {feas}, gap {gap:.2e}")
    assert feas and ctx.check_primal(xf) == 0 and gap <= 1e-2
    # every fine vertex pair used by the fine solution is a ring candidate
    used = np_(ctx.matched_pairs(xf))
    cand = set(map(tuple, np.stack([np.repeat(np.arange(len(pf.VX)), cxy.shape[1]), np_(cxy).ravel()], 1).tolist()))
    assert all(tuple(u) in cand for u in used.tolist())


def test_c2f_errors_are_reported():
    """Bad inputs come back as errors (checked on the host or by the
    kernel's own range test), never as out-of-range accesses."""
    DMError = __import__("paper_2310_08230_amd").DMError
    pf = make_pair(3, 0, faces_x=500, faces_y=500)
    ctx = dm().Context(0)
    seeds = np.array([[0, 0], [5, 7]], np.int32)
    with pytest.raises(DMError) as e:   # a capacity below the needed K
        ctx.ring_candidates(pf.VX, pf.FX, pf.VY, pf.FY, np.stack([np.arange(252)] * 2, 1), rings=2, kcap=4)
    assert e.value.code == -6
    with pytest.raises(DMError):        # a seed outside the fine mesh
        ctx.ring_candidates(pf.VX, pf.FX, pf.VY, pf.FY, np.array([[0, 10 ** 6]], np.int32), rings=1)
    with pytest.raises(DMError) as e:   # a fine vertex left without candidates
        ctx.ring_candidates(pf.VX, pf.FX, pf.VY, pf.FY, seeds, rings=1, kcap=64)
    assert e.value.code == -4
    with pytest.raises(DMError):
        ctx.nearest_vertices(pf.RX.astype(np.float32), np.zeros((0, 3), np.float32))
