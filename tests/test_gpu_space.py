"""GPU product space, incidence, presolve and candidates against the oracle:
bit-exact for every index array."""
import numpy as np
import pytest
import torch

from gpu_common import both, dm, np_, say
from helpers import bf16_rne, full_candidates
from oracle import oracle as O
from synth import make_pair, meshes, tiny_pair

pytestmark = pytest.mark.gpu

EXACT = ["pv", "code", "state", "row_key", "row_ptr", "ent_var", "ent_coef", "row_b", "free_var",
         "rrow_orig", "rrow_ptr", "rent_var", "rent_coef", "rrow_b", "cand"]


def _compare_space(S, ctx):
    i = ctx.info
    o = S.info
    assert (i["n_prod_tri"], i["n_rows_full"], i["nnz_full"], i["n_closed_full"], i["n_free"],
            i["n_fixed1"], i["n_rows"], i["nnz"]) == (o["nP"], o["n_rows_full"], o["nnz_full"],
                                                      o["n_closed_full"], o["n_free"], o["n_fixed1"],
                                                      o["n_rows"], o["nnz"])
    for name in EXACT:
        g = np_(ctx.get_space(name))
        r = S.get(name)
        assert g.dtype == r.dtype and g.shape == r.shape, name
        assert np.array_equal(g, r), name


@pytest.mark.parametrize("cfg,seed", [(1, 0), (1, 3), (2, 0), (2, 1)])
def test_space_parity_configs(cfg, seed):
    p = make_pair(cfg, seed)
    S, ctx = both(p, p.spec.k)
    say(f"  |P|={ctx.info['n_prod_tri']} nnz={ctx.info['nnz']} rounds={ctx.info['presolve_rounds']}")
    _compare_space(S, ctx)


def test_space_parity_config3_full_size():
    p = make_pair(3, 0)
    S, ctx = both(p, p.spec.k, "fp32")
    _compare_space(S, ctx)


@pytest.mark.parametrize("kx,ky", [("tetra", "tetra"), ("octa", "icosa"), ("icosa", "icosa")])
def test_space_parity_unpruned(kx, ky):
    p = tiny_pair(kx, ky)
    cxy, cyx, _ = full_candidates(len(p.VX), len(p.VY))
    S = O.Space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    ctx = dm().Context(0)
    ctx.build_product_space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    _compare_space(S, ctx)
    assert ctx.info["n_prod_tri"] == O.unpruned_count(len(p.VX), len(p.VX) + len(p.FX) - 2, len(p.FX),
                                                      len(p.VY), len(p.VY) + len(p.FY) - 2, len(p.FY))


def test_space_with_fixed_variables():
    # harder pruning leaves variables fixed to 1 and closedness rows with b != 0
    p = make_pair(1, 0)
    S, ctx = both(p, 6)
    assert ctx.info["n_fixed1"] > 0
    assert np.any(S.get("rrow_b")[: ctx.info["n_short_rows"]] != 0) or ctx.info["n_fixed1"] > 0
    _compare_space(S, ctx)


def test_edges_match_oracle():
    p = make_pair(2, 0)
    ctx = dm().Context(0)
    cxy, cyx = O.knn(p.DX, p.DY, 16)
    ctx.build_product_space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    for F, V, name in [(p.FX, p.VX, "edges_x"), (p.FY, p.VY, "edges_y")]:
        E, _ = O.mesh_edges(F, len(V))
        assert np.array_equal(np_(ctx.get_space(name)), E)


def test_errors():
    ctx = dm().Context(0)
    p = make_pair(1, 0, desc_noise=0.6)
    cxy, cyx = O.knn(p.DX, p.DY, 6)
    with pytest.raises(dm().DMError) as e:
        ctx.build_product_space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    assert e.value.code == -4
    V, F = meshes.icosahedron()
    bad = F.copy()
    bad[0] = bad[0][[0, 2, 1]]
    cxy, cyx, _ = full_candidates(12, 12)
    with pytest.raises(dm().DMError) as e:
        ctx.build_product_space(V, bad, V, F, cxy, cyx)
    assert e.value.code == -2
    V2, F2 = meshes.octahedron()
    n = 3
    T = []
    for a in range(n):
        for b in range(n):
            i, j = a * n + b, a * n + (b + 1) % n
            k, l_ = ((a + 1) % n) * n + b, ((a + 1) % n) * n + (b + 1) % n
            T += [[i, j, l_], [i, l_, k]]
    cxy, cyx, _ = full_candidates(6, 9)
    with pytest.raises(dm().DMError) as e:
        ctx.build_product_space(V2, F2, np.zeros((9, 3), np.float32), np.array(T), cxy, cyx)
    assert e.value.code == -3
    bad_c = cxy.copy()
    bad_c[0, 0] = 99
    with pytest.raises(dm().DMError) as e:
        ctx.build_product_space(V2, F2, V2, F2, bad_c[:, :6], full_candidates(6, 6)[1])
    assert e.value.code == -1


def test_mesh_errors_name_the_first_fault():
    """Malformed meshes are rejected with the fault named, in a fixed order
    (non-finite vertex, index out of range, repeated vertex, orientation),
    also where one mesh has several faults; the context stays usable."""
    V, F = meshes.icosahedron()
    cxy, cyx, _ = full_candidates(12, 12)
    ctx = dm().Context(0)
    out_of_range = F.copy()
    out_of_range[3, 1] = 12
    repeated = F.copy()
    repeated[5, 2] = repeated[5, 0]
    both_faults = out_of_range.copy()
    both_faults[7] = both_faults[7][[0, 2, 1]]   # also flipped
    nan_v = V.copy()
    nan_v[4, 1] = np.nan
    cases = [(V, out_of_range, -2, "out of range"), (V, repeated, -2, "repeats a vertex"),
             (V, both_faults, -2, "out of range"), (nan_v, F, -5, "non-finite vertex"),
             (nan_v, both_faults, -5, "non-finite vertex")]
    for Vb, Fb, code, msg in cases:
        with pytest.raises(dm().DMError, match=msg) as e:
            ctx.build_product_space(Vb, Fb, V, F, cxy, cyx)
        assert e.value.code == code, msg
        with pytest.raises(dm().DMError, match=msg):
            ctx.build_product_space(V, F, Vb, Fb, cxy, cyx)
    S = O.Space(V, F, V, F, cxy, cyx)
    ctx.build_product_space(V, F, V, F, cxy, cyx)
    assert ctx.info["n_prod_tri"] == S.info["nP"]


def test_nonfinite_descriptors_are_rejected():
    """A NaN or an infinity in either shape's descriptors is reported as
    DM_ERR_NONFINITE by the candidate and cost builders in every precision,
    and the context stays usable."""
    p = make_pair(1, 0)
    DX, DY = torch.from_numpy(p.DX), torch.from_numpy(p.DY)
    ctx = dm().Context(0)
    cxy, cyx = O.knn(p.DX, p.DY, 6)
    ctx.build_product_space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    for side, val in (("X", float("nan")), ("Y", float("inf")), ("Y", float("nan"))):
        bx, by = DX.clone(), DY.clone()
        (bx if side == "X" else by)[len(bx if side == "X" else by) - 1, 3] = val
        for prec in ("fp32", "bf16"):
            with pytest.raises(dm().DMError) as e:
                ctx.knn_candidates(bx, by, 6, prec)
            assert e.value.code == -5, (side, prec)
        for prec in ("fp64", "fp32", "bf16"):
            with pytest.raises(dm().DMError) as e:
                ctx.build_costs(bx, by, prec)
            assert e.value.code == -5, (side, prec)
    gx, gy = ctx.knn_candidates(DX, DY, 6, "fp32")
    assert np.array_equal(np_(gx), cxy) and np.array_equal(np_(gy), cyx)
    ctx.build_costs(DX, DY, "fp64")


@pytest.mark.parametrize("cfg,prec", [(1, "fp32"), (2, "fp32"), (2, "bf16"), (3, "bf16")])
def test_knn_candidates(cfg, prec):
    p = make_pair(cfg, 0)
    K = p.spec.k
    ctx = dm().Context(0)
    cxy, cyx = ctx.knn_candidates(torch.from_numpy(p.DX), torch.from_numpy(p.DY), K, prec)
    rxy, ryx = O.knn(p.DX, p.DY, K)
    D = np.sqrt(((p.DX.astype(np.float64)[:, None, :] - p.DY.astype(np.float64)[None]) ** 2).sum(-1))
    # distance error bound of the form: FP32 ~1e-5 relative; BF16 from the
    # rounding of the inputs (2^-9 per component)
    tol = 1e-4 if prec == "fp32" else 3e-2
    near_ties = 0
    for G, R, Dm in [(np_(cxy), rxy, D), (np_(cyx), ryx, D.T)]:
        for q in range(len(G)):
            if set(G[q]) == set(R[q]):
                continue
            # differences only where the K-th and (K+1)-th distances are within tol
            srt = np.sort(Dm[q])
            assert srt[K] - srt[K - 1] <= tol * srt[K], (q, srt[K - 1], srt[K])
            near_ties += 1
    say(f"  {prec} candidate sets differing at near ties: {near_ties}")
    assert near_ties <= (2 if prec == "fp32" else 0.2 * (len(p.DX) + len(p.DY)))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_knn_rows_longer_than_one_lds_table(prec):
    """Both sides above the top-K kernel's 4096-key LDS table (5000 and 4500
    vertices), so every query row goes through the table in chunks that keep
    the best K so far: the sets must equal the oracle's K nearest (on the
    BF16-rounded descriptors for the BF16 form) except where the K-th and
    (K+1)-th squared distances lie within the FP32 error of the distance
    computation.  K = 2049 is refused at this size."""
    rng = np.random.default_rng(5)
    DX = rng.standard_normal((5000, 24)).astype(np.float32)
    DY = rng.standard_normal((4500, 24)).astype(np.float32)
    K = 40
    say(f"[knn-long] prec={prec} nvx=5000 nvy=4500 D=24 K={K}")
    ctx = dm().Context(0)
    cxy, cyx = ctx.knn_candidates(torch.from_numpy(DX), torch.from_numpy(DY), K, prec)
    BX, BY = (bf16_rne(DX), bf16_rne(DY)) if prec == "bf16" else (DX, DY)
    rxy, ryx = O.knn(BX, BY, K)
    bx, by = BX.astype(np.float64), BY.astype(np.float64)
    D2 = (bx ** 2).sum(1)[:, None] + (by ** 2).sum(1)[None] - 2.0 * bx @ by.T
    nx, ny = (bx ** 2).sum(1), (by ** 2).sum(1)
    eps = 4.0 * bx.shape[1] * 2.0 ** -24
    differ = 0
    for G, R, Dm, nq, nc in [(np_(cxy), rxy, D2, nx, ny), (np_(cyx), ryx, D2.T, ny, nx)]:
        assert G.min() >= 0 and G.max() < Dm.shape[1]
        for q in range(len(G)):
            assert len(set(G[q])) == K
            if set(G[q]) == set(R[q]):
                continue
            srt = np.sort(Dm[q])
            assert srt[K] - srt[K - 1] <= eps * (nq[q] + nc.max()), (q, srt[K - 1], srt[K])
            differ += 1
    say(f"  candidate sets differing at FP32 near ties: {differ} of 9500")
    assert differ <= 0.01 * 9500
    with pytest.raises(dm().DMError):
        ctx.knn_candidates(torch.from_numpy(DX), torch.from_numpy(DY), 2049, prec)


@pytest.mark.parametrize("case", ["cfg2", "cfg3", "d16", "d72", "d200"])
def test_knn_bf16_matches_rounded_inputs(case):
    """BF16 candidates against the oracle run on the same BF16-rounded
    descriptors: products of BF16 values are exact in FP32, so the candidate
    sets may differ only where the K-th and (K+1)-th squared distances lie
    within the FP32 accumulation error (D terms, norms included).  The custom
    widths cover the distance kernel's K loop with a remainder only (16), one
    64-wide group plus a remainder (72) and three groups plus a remainder
    (200), on side lengths that leave ragged 64-row tiles."""
    if case.startswith("cfg"):
        p = make_pair(int(case[3:]), 0)
        DX, DY, K = p.DX, p.DY, p.spec.k
    else:
        rng = np.random.default_rng(17)
        D = int(case[1:])
        DX = rng.standard_normal((300, D)).astype(np.float32)
        DY = rng.standard_normal((261, D)).astype(np.float32)
        K = 8
    ctx = dm().Context(0)
    cxy, cyx = ctx.knn_candidates(torch.from_numpy(DX), torch.from_numpy(DY), K, "bf16")
    BX, BY = bf16_rne(DX), bf16_rne(DY)
    rxy, ryx = O.knn(BX, BY, K)
    bx, by = BX.astype(np.float64), BY.astype(np.float64)
    D2 = (bx ** 2).sum(1)[:, None] + (by ** 2).sum(1)[None] - 2.0 * bx @ by.T
    nx, ny = (bx ** 2).sum(1), (by ** 2).sum(1)
    eps = 4.0 * bx.shape[1] * 2.0 ** -24
    differ = 0
    for G, R, Dm, nq, nc in [(np_(cxy), rxy, D2, nx, ny), (np_(cyx), ryx, D2.T, ny, nx)]:
        for q in range(len(G)):
            if set(G[q]) == set(R[q]):
                continue
            srt = np.sort(Dm[q])
            assert srt[K] - srt[K - 1] <= eps * (nq[q] + nc.max()), (case, q, srt[K - 1], srt[K])
            differ += 1
    say(f"  {case}: candidate sets differing at FP32 near ties: {differ} of {len(DX) + len(DY)}")
    assert differ <= 0.02 * (len(DX) + len(DY))
