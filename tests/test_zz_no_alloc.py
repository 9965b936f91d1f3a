"""The allocation-free candidate entry point (dm_knn_candidates_noalloc)
against dm_knn_candidates: identical candidate lists, bit for bit, on
consecutive calls of decreasing size through the C ABI, and the size limit
of its fixed scratch array."""
import numpy as np
import pytest
import torch

from gpu_common import dm, np_, say
from synth import make_pair

pytestmark = pytest.mark.gpu


def _pair_desc(cfg):
    p = make_pair(cfg, 0)
    return p.DX, p.DY, p.spec.k


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_candidates_equal_allocating_entry_point(prec):
    ctx = dm().Context(0)
    # largest pair first, then smaller ones: each call must see only its own data
    for cfg in (5, 2, 1):
        DX, DY, K = _pair_desc(cfg)
        say(f"[noalloc] cfg={cfg} prec={prec} nvx={DX.shape[0]} nvy={DY.shape[0]} D={DX.shape[1]} K={K}")
        ref_xy, ref_yx = ctx.knn_candidates(torch.from_numpy(DX), torch.from_numpy(DY), K, prec)
        got_xy, got_yx = ctx.knn_candidates_noalloc(torch.from_numpy(DX), torch.from_numpy(DY), K, prec)
        torch.cuda.synchronize()
        assert np.array_equal(np_(got_xy), np_(ref_xy)) and np.array_equal(np_(got_yx), np_(ref_yx))
    # the same small call again after the large ones, into caller-provided outputs
    DX, DY, K = _pair_desc(1)
    out = (torch.full((DX.shape[0], K), -7, dtype=torch.int32, device="cuda"),
           torch.full((DY.shape[0], K), -7, dtype=torch.int32, device="cuda"))
    ctx.knn_candidates_noalloc(torch.from_numpy(DX), torch.from_numpy(DY), K, prec, out=out)
    ref_xy, ref_yx = ctx.knn_candidates(torch.from_numpy(DX), torch.from_numpy(DY), K, prec)
    assert np.array_equal(np_(out[0]), np_(ref_xy)) and np.array_equal(np_(out[1]), np_(ref_yx))


def test_noalloc_rejects_sizes_beyond_its_scratch():
    ctx = dm().Context(0)
    g = torch.Generator().manual_seed(0)
    # 2100 x 2100 squared distances alone need 17.6 MB, more than the 16 MiB array
    DX = torch.randn(2100, 8, generator=g)
    DY = torch.randn(2100, 8, generator=g)
    with pytest.raises(dm().DMError) as e:
        ctx.knn_candidates_noalloc(DX, DY, 4, "fp32")
    assert e.value.code == -6 and "scratch" in str(e.value)
    # the context still works afterwards, on both entry points
    DX, DY, K = _pair_desc(1)
    a = ctx.knn_candidates_noalloc(torch.from_numpy(DX), torch.from_numpy(DY), K, "fp32")
    b = ctx.knn_candidates(torch.from_numpy(DX), torch.from_numpy(DY), K, "fp32")
    assert all(np.array_equal(np_(x), np_(y)) for x, y in zip(a, b))


def test_noalloc_reports_nonfinite_descriptors():
    ctx = dm().Context(0)
    DX, DY, K = _pair_desc(1)
    DX = DX.copy()
    DX[3, 2] = np.nan
    with pytest.raises(dm().DMError) as e:
        ctx.knn_candidates_noalloc(torch.from_numpy(DX), torch.from_numpy(DY), K, "bf16")
    assert e.value.code == -5
    # the error word is cleared by the next call
    a = ctx.knn_candidates_noalloc(torch.from_numpy(DY), torch.from_numpy(DY), K, "bf16")
    b = ctx.knn_candidates(torch.from_numpy(DY), torch.from_numpy(DY), K, "bf16")
    assert all(np.array_equal(np_(x), np_(y)) for x, y in zip(a, b))
