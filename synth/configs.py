"""Seeded synthetic mesh pairs with per-vertex descriptors.

They stand in for the paper's shape pairs (FAUST_r, SMAL, SHREC'20, DT4D-H
downsampled to 450 faces, 500-1000 faces in the convergence study, 128-d
learned features; Sec. 5 "Datasets" and Sec. 5.1), which are not available
here.  Recipe per pair:

* rest surface: the unit sphere triangulated as an icosphere, optionally
  decimated shortest-edge-first to the requested face count;
* poses: X and Y are posed copies of the rest surface (noise, random
  rotation, a smooth bump field along the normal, anisotropic scale);
* descriptors: ``F = sin(P_rest W + beta) + N(0, 0.05^2)`` with W ~ N(0, 3^2)
  of shape [3, D] and beta ~ U(0, 2 pi)^D shared by X and Y, i.e. matching
  points of the rest surface get nearly equal descriptors.

Every random draw comes from numpy's PCG64 seeded by ``SeedSequence([cfg,
seed])`` and its spawned children, so a (config, seed) pair fixes the input
bit for bit.  This module holds none of the matching method's arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from functools import lru_cache

import numpy as np

from . import meshes


@dataclass
class PairSpec:
    name: str
    faces_x: int
    faces_y: int
    dim: int
    k: int
    iters: int
    pose: str            # "noise" | "rot_bumps" | "rot_scale_bumps" | "remesh"
    temperature: float = 0.0
    cost_prec: str = "fp32"   # "fp64" | "fp32" | "bf16"
    msg_prec: str = "fp32"    # "fp64" | "fp32"
    omega: float = 0.5
    desc_noise: float = 0.05  # std of the per-vertex descriptor noise
    notes: str = ""


# Workloads: shapes, sizes and distributions of the paper's instances (450 to
# 1000 faces per shape, 128-d features), at five scales.
CONFIGS = {
    1: PairSpec("small_fp64", 80, 80, 16, 6, 200, "noise", cost_prec="fp64",
                msg_prec="fp64", notes="icosphere L1 (42 verts), sigma=0.01 noise on X and Y"),
    2: PairSpec("plain_fp32_500", 500, 500, 64, 16, 1000, "rot_bumps",
                notes="500-face icosphere pair, random rotation + bumps (0.05)"),
    3: PairSpec("mixed_bf16_1000", 1000, 1000, 128, 32, 1000, "rot_scale_bumps",
                cost_prec="bf16", notes="1000-face pair, anisotropic scale + bumps"),
    4: PairSpec("diff_t0.1_1000", 1000, 1000, 128, 32, 1000, "rot_scale_bumps",
                temperature=0.1, cost_prec="bf16", notes="pair of config 3, smoothed"),
    5: PairSpec("largest_2000x3000", 2000, 3000, 128, 48, 1000, "remesh",
                cost_prec="bf16", notes="unequal resolutions, Y remeshed"),
}


@dataclass
class Pair:
    spec: PairSpec
    seed: int
    VX: np.ndarray          # float32 [nvx, 3] posed vertices
    FX: np.ndarray          # int32   [nfx, 3]
    VY: np.ndarray
    FY: np.ndarray
    DX: np.ndarray          # float32 [nvx, D] descriptors
    DY: np.ndarray
    RX: np.ndarray = field(repr=False, default=None)   # rest positions (float64)
    RY: np.ndarray = field(repr=False, default=None)


@lru_cache(maxsize=None)
def _base_mesh(faces: int, levels: int, jitter_key: tuple | None):
    V, F = meshes.icosphere(levels)
    if jitter_key is not None:
        seed, = jitter_key
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([0xD15C0, seed])))
        q = rng.normal(size=4)
        R = _quat_to_rot(q / np.linalg.norm(q))
        V = V @ R.T
        jitter = rng.uniform(0.85, 1.15, size=len(V))
    else:
        jitter = None
    if faces != len(F):
        V, F = meshes.decimate(V, F, faces, jitter=jitter)
    return V, F


def rest_mesh(faces: int, remesh_seed: int | None = None):
    """Unit-sphere mesh with ``faces`` faces (20 * 4^L, or decimated from
    the next finer icosphere).  ``remesh_seed`` yields a different
    triangulation of the same sphere."""
    lv = 0
    while 20 * 4 ** lv < faces:
        lv += 1
    key = None if remesh_seed is None else (int(remesh_seed),)
    V, F = _base_mesh(faces, lv, key)
    return V.copy(), F.copy()


def _quat_to_rot(q):
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _rotation(rng):
    q = rng.normal(size=4)
    return _quat_to_rot(q / np.linalg.norm(q))


def _bumps(rng, P):
    """Normal displacement field: 8 Gaussian bumps of width 0.35 on the unit
    sphere, normalised to a peak amplitude of 0.05."""
    c = rng.normal(size=(8, 3))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    g = rng.uniform(-1.0, 1.0, size=8)
    d2 = ((P[:, None, :] - c[None, :, :]) ** 2).sum(-1)
    b = (g[None, :] * np.exp(-d2 / (2 * 0.35 ** 2))).sum(1)
    return 0.05 * b / np.abs(b).max()


def _descriptors(rng_w, rng_n, P, D, noise=0.05):
    W = rng_w.normal(0.0, 3.0, size=(3, D))
    beta = rng_w.uniform(0.0, 2 * np.pi, size=D)
    return np.sin(P @ W + beta) + rng_n.normal(0.0, noise, size=(len(P), D))


def make_pair(cfg: int, seed: int = 0, spec: PairSpec | None = None, **over) -> Pair:
    """Pair of config ``cfg`` with ``seed``; keyword overrides (e.g.
    ``desc_noise=0.5``) change the spec for test variants."""
    spec = spec or CONFIGS[cfg]
    if over:
        from dataclasses import replace
        spec = replace(spec, **over)
    ss = np.random.SeedSequence([cfg, seed])
    r = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(8)]
    PX, FX = rest_mesh(spec.faces_x)
    if spec.pose == "remesh":
        PY, FY = rest_mesh(spec.faces_y, remesh_seed=seed)
    else:
        PY, FY = PX.copy(), FX.copy()
    if spec.pose == "noise":
        VX = PX + r[0].normal(0.0, 0.01, size=PX.shape)
        VY = (PY + r[1].normal(0.0, 0.01, size=PY.shape)) @ _rotation(r[2]).T
    elif spec.pose == "rot_bumps":
        VX = PX.copy()
        nY = PY / np.linalg.norm(PY, axis=1, keepdims=True)
        VY = (PY + _bumps(r[3], PY)[:, None] * nY) @ _rotation(r[2]).T
    elif spec.pose in ("rot_scale_bumps", "remesh"):
        VX = PX.copy()
        nY = PY / np.linalg.norm(PY, axis=1, keepdims=True)
        S = np.diag(r[4].uniform(0.8, 1.2, size=3))
        Q = PY + _bumps(r[3], PY)[:, None] * nY
        if spec.pose == "remesh":
            Q = Q + r[1].normal(0.0, 0.01, size=Q.shape)
        VY = Q @ (_rotation(r[2]) @ S).T
    else:
        raise ValueError(spec.pose)
    W_rng = r[5]
    state = W_rng.bit_generator.state
    DX = _descriptors(W_rng, r[6], PX, spec.dim, spec.desc_noise)
    W_rng.bit_generator.state = state          # same W, beta for Y
    DY = _descriptors(W_rng, r[7], PY, spec.dim, spec.desc_noise)
    return Pair(spec, seed,
                VX.astype(np.float32), FX.astype(np.int32),
                VY.astype(np.float32), FY.astype(np.int32),
                DX.astype(np.float32), DY.astype(np.float32), PX, PY)


def tiny_pair(kind_x: str, kind_y: str, dim: int = 8, seed: int = 0, noise: float = 0.0,
              desc_noise: float = 0.05):
    """Pairs of platonic solids for exhaustive checks (tetra/octa/icosa)."""
    make = {"tetra": meshes.tetrahedron, "octa": meshes.octahedron, "icosa": meshes.icosahedron}
    PX, FX = make[kind_x]()
    PY, FY = make[kind_y]()
    ss = np.random.SeedSequence([0x7171, seed])
    r = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(4)]
    VX = PX + r[0].normal(0.0, noise, size=PX.shape) if noise else PX.copy()
    VY = (PY + r[1].normal(0.0, noise, size=PY.shape)) if noise else PY.copy()
    st = r[2].bit_generator.state
    DX = _descriptors(r[2], r[3], PX, dim, desc_noise)
    r[2].bit_generator.state = st
    DY = _descriptors(r[2], r[3], PY, dim, desc_noise)
    spec = PairSpec(f"{kind_x}_{kind_y}", len(FX), len(FY), dim, 0, 0, "tiny",
                    cost_prec="fp64", msg_prec="fp64")
    return Pair(spec, seed, VX.astype(np.float32), FX.astype(np.int32),
                VY.astype(np.float32), FY.astype(np.int32),
                DX.astype(np.float32), DY.astype(np.float32), PX, PY)
