"""Shared set-up of the GPU parity tests: the same seeded inputs go to the
oracle and to the library; the oracle's candidates are used on both sides so
that index parity does not depend on distance rounding."""
import functools
import sys

import numpy as np

from oracle import oracle as O


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def dm():
    import paper_2310_08230_amd as m
    m.lib()
    return m


def both(pair, K, cost_prec="fp64"):
    import torch
    say(f"[setup] {pair.spec.name} seed={pair.seed} K={K} cost={cost_prec}")
    cxy, cyx = O.knn(pair.DX, pair.DY, K)
    S = O.Space(pair.VX, pair.FX, pair.VY, pair.FY, cxy, cyx)
    S.costs(pair.DX, pair.DY)
    ctx = dm().Context(0)
    ctx.build_product_space(pair.VX, pair.FX, pair.VY, pair.FY, cxy, cyx)
    ctx.build_costs(torch.from_numpy(pair.DX), torch.from_numpy(pair.DY), cost_prec)
    torch.cuda.synchronize()
    return S, ctx


def np_(t):
    return t.detach().cpu().numpy()


def rel_err(a, b, floor=1e-12):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor))) if a.size else 0.0
