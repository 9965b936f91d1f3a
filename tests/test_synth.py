"""The seeded input generator is deterministic and produces the intended
shapes and sizes."""
import numpy as np
import pytest

from synth import CONFIGS, make_pair


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_pair_shapes_and_determinism(cfg):
    a, b = make_pair(cfg, 3), make_pair(cfg, 3)
    s = CONFIGS[cfg]
    assert len(a.FX) == s.faces_x and len(a.FY) == s.faces_y
    assert a.DX.shape == (len(a.VX), s.dim) and a.DX.dtype == np.float32
    for f in ("VX", "FX", "VY", "FY", "DX", "DY"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = make_pair(cfg, 4)
    assert not np.array_equal(a.DX, c.DX)


def test_descriptors_match_nearest_points():
    # matching rest points have close descriptors: the identity is the
    # descriptor-nearest neighbour for most vertices
    p = make_pair(2, 0)
    D = ((p.DX[:, None, :] - p.DY[None]) ** 2).sum(-1)
    assert np.mean(D.argmin(1) == np.arange(len(p.DX))) > 0.9
