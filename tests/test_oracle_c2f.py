"""Oracle of the coarse-to-fine pruning (Sec. 5.2) pinned against closed
forms on regular solids, graph distances from scipy's shortest paths, a k-d
tree for nearest points, and the identity matching."""
import numpy as np
import pytest

from helpers import full_candidates
from oracle import oracle as O
from synth import meshes

SOLIDS = {"tetra": meshes.tetrahedron, "octa": meshes.octahedron, "icosa": meshes.icosahedron}


def _hops(F, nv):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    F = np.asarray(F)
    a = np.concatenate([F[:, 0], F[:, 1], F[:, 2]])
    b = np.concatenate([F[:, 1], F[:, 2], F[:, 0]])
    A = csr_matrix((np.ones(len(a)), (a, b)), shape=(nv, nv))
    return shortest_path(A, unweighted=True, directed=False)


@pytest.mark.parametrize("kind,r1,r2", [("tetra", 4, 4), ("octa", 5, 6), ("icosa", 6, 11)])
def test_ring_sizes_on_regular_solids(kind, r1, r2):
    V, F = SOLIDS[kind]()
    assert {len(r) for r in O.vertex_rings(F, len(V), 1)} == {r1}
    assert {len(r) for r in O.vertex_rings(F, len(V), 2)} == {r2}


def test_rings_are_graph_balls():
    from synth.configs import rest_mesh
    P, F = rest_mesh(500)
    H = _hops(F, len(P))
    for rings in (1, 2):
        R = O.vertex_rings(F, len(P), rings)
        for v in range(0, len(P), 7):
            assert R[v] == set(np.nonzero(H[v] <= rings)[0].tolist())


def test_nearest_vertices_against_a_kd_tree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(3)
    Q = rng.normal(size=(400, 3)).astype(np.float32)
    P = rng.normal(size=(300, 3)).astype(np.float32)
    got = O.nearest_vertices(P, Q)
    assert np.array_equal(got, cKDTree(Q.astype(np.float64)).query(P.astype(np.float64))[1])
    # exact ties go to the lower index
    Q2 = np.array([[1, 0, 0], [0, 1, 0], [-1, 0, 0]], np.float32)
    assert O.nearest_vertices(np.zeros((1, 3), np.float32), Q2)[0] == 0
    assert np.array_equal(O.nearest_vertices(Q, Q), np.arange(len(Q)))


@pytest.mark.parametrize("kind", ["octa", "icosa"])
def test_matched_pairs_of_the_identity_matching(kind):
    V, F = SOLIDS[kind]()
    cxy, cyx, _ = full_candidates(len(V), len(V))
    S = O.Space(V, F, V, F, cxy, cyx)
    code = S.get("code")
    x = ((code[:, 0] == 0) & (code[:, 2] == 0) & (code[:, 1] == code[:, 3])).astype(np.uint8)
    pairs = O.matched_pairs(S.get("pv"), x, len(V))
    assert np.array_equal(pairs, np.stack([np.arange(len(V))] * 2, 1))


@pytest.mark.parametrize("rings,hops", [(1, 2), (2, 4)])
def test_ring_candidates_closed_form(rings, hops):
    """Identity seeds on an icosahedron: (u, w) is a candidate iff some v has
    u and w in its ring, i.e. u and w are at most 2 * rings edges apart."""
    V, F = meshes.icosahedron()
    H = _hops(F, len(V))
    seeds = np.stack([np.arange(len(V))] * 2, 1)
    cxy, cyx = O.ring_candidates(F, len(V), F, len(V), seeds, rings)
    want = [np.nonzero(H[u] <= hops)[0] for u in range(len(V))]
    K = max(len(w) for w in want)
    assert cxy.shape == (len(V), K) and cyx.shape == (len(V), K)
    for u in range(len(V)):
        assert np.array_equal(np.unique(cxy[u]), want[u]) and np.array_equal(np.unique(cyx[u]), want[u])
        assert np.all(np.diff(cxy[u]) >= 0)   # ascending, padded with the last entry
