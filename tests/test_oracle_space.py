"""Pins of the oracle's meshes, mixed areas, candidates, product space and
presolve against closed forms, invariants and independent computations."""
import json
import os

import numpy as np
import pytest

from helpers import full_candidates, full_rows, matching_violations
from oracle import oracle as O
from synth import make_pair, meshes, rest_mesh, tiny_pair

GOLD = os.path.join(os.path.dirname(__file__), "golden")

SOLIDS = {"tetra": meshes.tetrahedron, "octa": meshes.octahedron, "icosa": meshes.icosahedron,
          "icosphere1": lambda: meshes.icosphere(1)}


# ---------------------------------------------------------------- meshes
def test_icosphere_counts_and_euler():
    V, F = meshes.icosphere(1)
    st, ne = O.mesh_check(F, len(V))
    assert st == 0 and (len(V), ne, len(F)) == (42, 120, 80)
    assert len(V) - ne + len(F) == 2


@pytest.mark.parametrize("faces", [500, 1000])
def test_decimated_meshes_are_manifold(faces):
    V, F = rest_mesh(faces)
    st, ne = O.mesh_check(F, len(V))
    assert st == 0 and len(F) == faces and ne == 3 * faces // 2 and len(V) - ne + faces == 2


def test_mesh_errors():
    V, F = meshes.icosahedron()
    bad = F.copy()
    bad[0] = bad[0][[0, 2, 1]]                     # flipped face
    assert O.mesh_check(bad, len(V))[0] == O.E_MESH
    assert O.mesh_check(F[1:], len(V))[0] == O.E_MESH      # open boundary
    dup = np.vstack([F, F[:1]])
    assert O.mesh_check(dup, len(V))[0] == O.E_MESH
    # two octahedra sharing one vertex: edge-manifold but not vertex-manifold
    V1, F1 = meshes.octahedron()
    F2 = F1 + 5                                    # vertex 5 of the first = vertex 0 of the second
    assert O.mesh_check(np.vstack([F1, F2]), 11)[0] == O.E_MESH


def test_edge_table_sorted_and_face_map():
    V, F = meshes.icosphere(1)
    E, FE = O.mesh_edges(F, len(V))
    keys = E[:, 0].astype(np.int64) * 1000 + E[:, 1]
    assert np.all(E[:, 0] < E[:, 1]) and np.all(np.diff(keys) > 0)
    for f in range(len(F)):
        for k in range(3):
            a, b = F[f, k], F[f, (k + 1) % 3]
            assert tuple(E[FE[f, k]]) == (min(a, b), max(a, b))


# ---------------------------------------------------------------- areas
def _circumcenter(a, b, c):
    ab, ac = b - a, c - a
    n = np.cross(ab, ac)
    return a + (np.dot(ac, ac) * np.cross(n, ab) + np.dot(ab, ab) * np.cross(ac, n)) / (2 * np.dot(n, n))


def _quad_area(p, q, r, s):
    return 0.5 * np.linalg.norm(np.cross(r - p, s - q))


def _mixed_areas_geometric(V, F):
    """Independent construction: in a non-obtuse triangle a vertex owns the
    quadrilateral (vertex, edge midpoint, circumcentre, edge midpoint); in an
    obtuse one the obtuse vertex gets half the area and the others a
    quarter."""
    A = np.zeros(len(V))
    for t in F:
        P = V[t].astype(np.float64)
        area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
        ang = [np.dot(P[(k + 1) % 3] - P[k], P[(k + 2) % 3] - P[k]) for k in range(3)]
        if min(ang) >= 0:
            cc = _circumcenter(*P)
            for k in range(3):
                p, q, r = P[k], P[(k + 1) % 3], P[(k + 2) % 3]
                A[t[k]] += _quad_area(p, (p + q) / 2, cc, (p + r) / 2)
        else:
            for k in range(3):
                A[t[k]] += area / 2 if ang[k] < 0 else area / 4
    return A


def test_mixed_areas_regular_solids():
    for make, share in [(meshes.icosahedron, 12), (meshes.octahedron, 6), (meshes.tetrahedron, 4)]:
        V, F = make()
        A = O.mixed_areas(V, F)
        tot = sum(0.5 * np.linalg.norm(np.cross(V[b] - V[a], V[c] - V[a])) for a, b, c in F)
        # float32 vertex input: allow its rounding
        assert np.allclose(A, tot / share, rtol=1e-6)


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_mixed_areas_sum_and_geometry(cfg):
    p = make_pair(cfg, 1)
    for V, F in [(p.VX, p.FX), (p.VY, p.FY)]:
        A = O.mixed_areas(V, F)
        V64 = V.astype(np.float64)
        tot = 0.5 * np.linalg.norm(np.cross(V64[F[:, 1]] - V64[F[:, 0]], V64[F[:, 2]] - V64[F[:, 0]]),
                                   axis=1).sum()
        assert abs(A.sum() - tot) <= 1e-12 * tot
        assert np.allclose(A, _mixed_areas_geometric(V64, F), rtol=1e-9, atol=1e-13)


def test_mixed_areas_obtuse_branch():
    """Decimated meshes contain obtuse triangles, so the geometric comparison
    above covers both branches of the mixed-area rule; here the obtuse
    triangles of one mesh are checked on their own."""
    p = make_pair(2, 1)
    V, F = p.VX.astype(np.float64), p.FX
    P = V[F]
    dots = np.stack([((P[:, (k + 1) % 3] - P[:, k]) * (P[:, (k + 2) % 3] - P[:, k])).sum(1)
                     for k in range(3)], 1)
    obtuse = np.nonzero(dots.min(1) < 0)[0]
    assert len(obtuse) > 50
    A = O.mixed_areas(V, F)
    # removing one obtuse triangle's share must change exactly its corners'
    # areas by area/2 (obtuse corner) and area/4 (the others)
    t = F[obtuse[0]]
    area = 0.5 * np.linalg.norm(np.cross(V[t[1]] - V[t[0]], V[t[2]] - V[t[0]]))
    ref = _mixed_areas_geometric(V, F)
    G = np.delete(F, obtuse[0], axis=0)
    rest = _mixed_areas_geometric(V, G)
    share = ref - rest
    k_obt = int(np.argmin(dots[obtuse[0]]))
    assert np.isclose(share[t[k_obt]], area / 2) and np.isclose(share[t[(k_obt + 1) % 3]], area / 4)
    assert np.allclose(A, ref, rtol=1e-9)


# ---------------------------------------------------------------- candidates
def test_knn_definition():
    p = make_pair(2, 0)
    K = 16
    cxy, cyx = O.knn(p.DX, p.DY, K)
    D = np.sqrt(((p.DX.astype(np.float64)[:, None, :] - p.DY.astype(np.float64)[None]) ** 2).sum(-1))
    for m in range(len(p.DX)):
        order = np.lexsort((np.arange(D.shape[1]), D[m]))[:K]
        assert list(order) == list(cxy[m])
    for n in range(len(p.DY)):
        order = np.lexsort((np.arange(D.shape[0]), D[:, n]))[:K]
        assert list(order) == list(cyx[n])


def test_knn_errors():
    p = make_pair(1, 0)
    with pytest.raises(O.OracleError):
        O.knn(p.DX, p.DY, 100)
    bad = p.DX.copy()
    bad[3, 2] = np.nan
    with pytest.raises(O.OracleError):
        O.knn(bad, p.DY, 4)


# ---------------------------------------------------------------- product space
def _load_cases():
    with open(os.path.join(GOLD, "closed_forms.json")) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _load_cases(), ids=lambda c: f"{c['x']}-{c['y']}")
def test_unpruned_closed_forms(case):
    VX, FX = SOLIDS[case["x"]]()
    VY, FY = SOLIDS[case["y"]]()
    cxy, cyx, _ = full_candidates(len(VX), len(VY))
    S = O.Space(VX, FX, VY, FY, cxy, cyx)
    i = S.info
    assert i["nP"] == case["nP"]
    assert i["n_closed_full"] == case["closed_rows"]
    assert i["nnz_full"] == case["nnz"]
    assert i["n_rows_full"] == case["closed_rows"] + len(FX) + len(FY)
    rp = S.get("row_ptr")
    L = np.diff(rp)
    nc = i["n_closed_full"]
    ex, ey = case["E"]
    vx, vy = case["V"]
    assert np.all(L[nc:nc + len(FX)] == 3 * len(FY) + 6 * ey + vy)
    assert np.all(L[nc + len(FX):] == 3 * len(FX) + 6 * ex + vx)
    assert O.unpruned_count(vx, ex, len(FX), vy, ey, len(FY)) == case["nP"]


def test_exact_count_vs_paper_estimate():
    # the paper's "about 21 |T_M||T_N|" against the exact 22 F^2 + 4 F
    for F in (450, 500, 1000):
        E, V = 3 * F // 2, F // 2 + 2
        n = O.unpruned_count(V, E, F, V, E, F)
        assert n == 22 * F * F + 4 * F
        assert abs(n / (F * F) - 21) < 1.1


def test_elements_distinct_and_canonical():
    VX, FX = meshes.octahedron()
    VY, FY = meshes.tetrahedron()
    cxy, cyx, _ = full_candidates(len(VX), len(VY))
    S = O.Space(VX, FX, VY, FY, cxy, cyx)
    pv, code = S.get("pv"), S.get("code")
    # three distinct product vertices, no repeated element
    assert np.all((pv[:, 0] != pv[:, 1]) & (pv[:, 1] != pv[:, 2]) & (pv[:, 0] != pv[:, 2]))
    cyc = [tuple(np.roll(t, -int(np.argmin(t)))) for t in pv]
    assert len(set(cyc)) == len(cyc)
    # canonical order: (x class, x id, y class, y id, pattern) ascending
    key = [(c[0], c[1], c[2] // 8, c[3], c[2] % 8) for c in code]
    assert key == sorted(key)
    # orientation anchored on the face side: the projected X sequence of a
    # face element equals the stored face, for Y faces a rotation of it
    for p, c in zip(pv, code):
        xs, ys = p // len(VY), p % len(VY)
        if c[0] == 0:
            assert list(xs) == list(FX[c[1]])
        if c[2] // 8 == 0:
            assert any(list(np.roll(ys, r)) == list(FY[c[3]]) for r in range(3))


@pytest.mark.parametrize("kind", ["tetra", "octa", "icosa"])
def test_identity_matching_is_feasible(kind):
    V, F = SOLIDS[kind]()
    cxy, cyx, _ = full_candidates(len(V), len(V))
    S = O.Space(V, F, V, F, cxy, cyx)
    code = S.get("code")
    x = ((code[:, 0] == 0) & (code[:, 2] == 0) & (code[:, 1] == code[:, 3])).astype(np.uint8)
    assert x.sum() == len(F)
    assert S.check_primal(x) == 0
    assert matching_violations(S.get("pv"), code, len(F), len(F), x) == 0
    # a single wrong rotation breaks closedness
    y = x.copy()
    f0 = np.nonzero(x)[0][0]
    y[f0] = 0
    y[f0 + 1] = 1
    assert S.check_primal(y) > 0 and matching_violations(S.get("pv"), code, len(F), len(F), y) > 0


def test_constraint_rows_match_definition():
    """Rows of A rebuilt from the element list by a direct reading of the
    constraints (dict keyed by product edge / face) equal the oracle's CSR."""
    p = tiny_pair("octa", "icosa", desc_noise=0.3)
    cxy, cyx = O.knn(p.DX, p.DY, 4)
    S = O.Space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    pv, code = S.get("pv"), S.get("code")
    rows = {}
    for q in range(len(pv)):
        for k in range(3):
            a, b = int(pv[q, k]), int(pv[q, (k + 1) % 3])
            rows.setdefault(("c", min(a, b), max(a, b)), []).append((q, 1 if a < b else -1))
        if code[q, 0] == 0:
            rows.setdefault(("x", int(code[q, 1])), []).append((q, 1))
        if code[q, 2] // 8 == 0:
            rows.setdefault(("y", int(code[q, 3])), []).append((q, 1))
    got = full_rows(S)
    keys = S.get("row_key")
    nc = S.info["n_closed_full"]
    npv = len(p.VX) * len(p.VY)
    for j, (vs, cs, b) in enumerate(got):
        if j < nc:
            key = ("c", int(keys[j] // npv), int(keys[j] % npv))
            assert b == 0
        elif j < nc + len(p.FX):
            key = ("x", j - nc)
            assert b == 1
        else:
            key = ("y", j - nc - len(p.FX))
            assert b == 1
        assert sorted(rows.pop(key, [])) == sorted(zip(vs.tolist(), cs.tolist()))
    assert not rows


def test_pruning_keeps_exactly_candidate_elements():
    p = make_pair(1, 2)
    cxy, cyx = O.knn(p.DX, p.DY, 6)
    S = O.Space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    cand = S.get("cand")
    ref = np.zeros_like(cand)
    for m in range(len(cxy)):
        ref[m, cxy[m]] = 1
    for n in range(len(cyx)):
        ref[cyx[n], n] = 1
    assert np.array_equal(cand, ref)
    full = O.Space(p.VX, p.FX, p.VY, p.FY, *full_candidates(42, 42)[:2])
    fpv = full.get("pv")
    keep = cand.reshape(-1)[fpv].all(axis=1)
    assert keep.sum() == S.info["nP"]
    assert np.array_equal(fpv[keep], S.get("pv"))


# ---------------------------------------------------------------- presolve
def _implied(rows, state):
    """Fixings some row still implies under ``state`` (independent reading)."""
    out = []
    for vs, cs, b in rows:
        r = b - sum(a for v, a in zip(vs, cs) if state[v] == 1)
        free = [(v, a) for v, a in zip(vs, cs) if state[v] < 0]
        for v, a in free:
            rest = [c for u, c in free if u != v]
            lo, hi = -sum(1 for c in rest if c < 0), sum(1 for c in rest if c > 0)
            if not (lo <= r - a <= hi) or not (lo <= r <= hi):
                out.append(v)
    return out


@pytest.mark.parametrize("cfg,seed", [(1, 0), (1, 3), (2, 0)])
def test_presolve_fixpoint(cfg, seed):
    p = make_pair(cfg, seed)
    cxy, cyx = O.knn(p.DX, p.DY, p.spec.k)
    S = O.Space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    state = S.get("state")
    assert _implied(full_rows(S), state) == []
    # every kept row has at least two free entries; free variables keep all
    # of their 3 closedness rows plus their projection rows
    rp = S.get("rrow_ptr")
    assert np.all(np.diff(rp) >= 2)
    code = S.get("code")[S.get("free_var")]
    expect = 3 + (code[:, 0] == 0) + (code[:, 2] // 8 == 0)
    assert np.array_equal(S.get("deg"), expect)


def test_presolve_preserves_lp_and_ilp():
    from scipy.optimize import Bounds, LinearConstraint, linprog, milp
    from scipy.sparse import csr_matrix
    p = tiny_pair("icosa", "icosa", desc_noise=0.5)
    cxy, cyx = O.knn(p.DX, p.DY, 3)
    S = O.Space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    c = S.costs(p.DX, p.DY)
    assert S.info["n_free"] < S.info["nP"]

    def solve(rows, n, cost, integral):
        r = np.concatenate([[j] * len(vs) for j, (vs, _, _) in enumerate(rows)])
        cidx = np.concatenate([vs for vs, _, _ in rows])
        val = np.concatenate([cs for _, cs, _ in rows]).astype(float)
        A = csr_matrix((val, (r, cidx)), shape=(len(rows), n))
        b = np.array([b for _, _, b in rows], float)
        if integral:
            res = milp(cost, constraints=LinearConstraint(A, b, b), integrality=np.ones(n),
                       bounds=Bounds(0, 1))
        else:
            res = linprog(cost, A_eq=A, b_eq=b, bounds=(0, 1), method="highs")
        assert res.status == 0
        return res.fun

    from helpers import reduced_rows
    fv = S.get("free_var")
    for integral in (False, True):
        full = solve(full_rows(S), S.info["nP"], c, integral)
        red = solve(reduced_rows(S), S.info["n_free"], c[fv], integral) + S.offset
        assert abs(full - red) <= 1e-9 * abs(full)


def test_infeasible_pruning_is_reported():
    p = make_pair(1, 0, desc_noise=0.6)
    cxy, cyx = O.knn(p.DX, p.DY, 6)
    with pytest.raises(O.OracleError) as e:
        O.Space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    assert e.value.code == O.E_INFEASIBLE


def test_genus_mismatch():
    VX, FX = meshes.octahedron()
    # a torus-like closed mesh: 3x3 grid torus
    n = 3
    V = np.zeros((n * n, 3))
    F = []
    for i in range(n):
        for j in range(n):
            a, b = i * n + j, i * n + (j + 1) % n
            c, d = ((i + 1) % n) * n + j, ((i + 1) % n) * n + (j + 1) % n
            F += [[a, b, d], [a, d, c]]
    F = np.array(F)
    st, ne = O.mesh_check(F, n * n)
    assert st == 0 and n * n - ne + len(F) == 0
    cxy, cyx, _ = full_candidates(6, 9)
    with pytest.raises(O.OracleError) as e:
        O.Space(VX, FX, V, F, cxy, cyx)
    assert e.value.code == O.E_GENUS
