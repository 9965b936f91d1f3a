"""Seeded synthetic triangle meshes: platonic solids, icospheres and a
deterministic shortest-edge decimator.

These are *inputs* only (the stand-in for the paper's remeshed shape datasets,
which are downsampled to a few hundred faces before matching, Sec. 5
"Datasets").  Nothing here computes any part of the matching method: no areas,
no distances, no product space.  Faces are stored counter-clockwise seen from
outside (outward normals).
"""
from __future__ import annotations

import heapq

import numpy as np

PHI = (1.0 + 5.0 ** 0.5) / 2.0


def _orient_outward(V: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Flip faces whose normal points towards the origin (star-shaped solids)."""
    F = F.copy()
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    n = np.cross(b - a, c - a)
    flip = (n * (a + b + c)).sum(1) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return F


def _canonical_faces(F: np.ndarray) -> np.ndarray:
    """Rotate each face so its smallest vertex comes first (cyclic order kept),
    then sort faces lexicographically.  Makes generated meshes independent of
    enumeration order."""
    F = np.asarray(F, dtype=np.int64)
    out = np.empty_like(F)
    for i, f in enumerate(F):
        k = int(np.argmin(f))
        out[i] = np.roll(f, -k)
    order = np.lexsort((out[:, 2], out[:, 1], out[:, 0]))
    return out[order]


def _faces_from_edge_length(V: np.ndarray, edge_len: float) -> np.ndarray:
    """All vertex triples whose three pairwise distances equal ``edge_len``."""
    n = len(V)
    D = np.linalg.norm(V[:, None, :] - V[None, :, :], axis=-1)
    adj = np.abs(D - edge_len) < 1e-6 * edge_len
    faces = []
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    faces.append((i, j, k))
    return np.array(faces, dtype=np.int64)


def tetrahedron():
    V = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = _faces_from_edge_length(V, np.linalg.norm(V[0] - V[1]))
    return V, _canonical_faces(_orient_outward(V, F))


def octahedron():
    V = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                 dtype=np.float64)
    F = _faces_from_edge_length(V, 2 ** 0.5)
    return V, _canonical_faces(_orient_outward(V, F))


def icosahedron():
    V = []
    for s1 in (-1, 1):
        for s2 in (-1, 1):
            V.append((0, s1, s2 * PHI))
            V.append((s1, s2 * PHI, 0))
            V.append((s2 * PHI, 0, s1))
    V = np.array(V, dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = _faces_from_edge_length(V, _min_pair_dist(V))
    return V, _canonical_faces(_orient_outward(V, F))


def _min_pair_dist(V):
    D = np.linalg.norm(V[:, None, :] - V[None, :, :], axis=-1)
    D[np.arange(len(V)), np.arange(len(V))] = np.inf
    return float(D.min())


def subdivide(V: np.ndarray, F: np.ndarray, levels: int):
    """Midpoint 1-to-4 subdivision, new vertices projected to the unit sphere."""
    V = [tuple(v) for v in V]
    F = [tuple(int(x) for x in f) for f in F]
    for _ in range(levels):
        mid = {}

        def midpoint(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in mid:
                p = (np.asarray(V[a]) + np.asarray(V[b])) * 0.5
                p /= np.linalg.norm(p)
                mid[key] = len(V)
                V.append(tuple(p))
            return mid[key]

        nf = []
        for a, b, c in F:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = nf
    return np.array(V, dtype=np.float64), _canonical_faces(np.array(F, dtype=np.int64))


def icosphere(levels: int):
    V, F = icosahedron()
    return subdivide(V, F, levels)


def decimate(V: np.ndarray, F: np.ndarray, target_faces: int,
             jitter: np.ndarray | None = None):
    """Shortest-edge-first collapse to ``target_faces`` faces on the unit sphere.

    Each collapse merges an edge (u, v) into u, placed at the re-projected
    midpoint.  Ties are broken by vertex ids.  A collapse is skipped when it
    would break the link condition (non-manifold result) or fold a face
    inwards.  ``jitter`` (one factor per original vertex pair hashing, or
    None) multiplies edge priorities so that the same sphere yields a
    different triangulation.  Returns compacted (V, F).
    """
    V = np.array(V, dtype=np.float64)
    faces = {i: list(map(int, f)) for i, f in enumerate(F)}
    vfaces = [set() for _ in range(len(V))]
    for fi, f in faces.items():
        for x in f:
            vfaces[x].add(fi)
    alive = np.ones(len(V), dtype=bool)
    version = np.zeros(len(V), dtype=np.int64)

    def prio(u, v):
        d = float(np.linalg.norm(V[u] - V[v]))
        if jitter is not None:
            d *= float(jitter[u] * jitter[v])
        return d

    def neighbours(u):
        s = set()
        for fi in vfaces[u]:
            s.update(faces[fi])
        s.discard(u)
        return s

    heap = []
    seen = set()
    for f in faces.values():
        for k in range(3):
            a, b = f[k], f[(k + 1) % 3]
            key = (min(a, b), max(a, b))
            if key not in seen:
                seen.add(key)
                heapq.heappush(heap, (prio(*key), key[0], key[1], 0, 0))
    nf = len(faces)
    while nf > target_faces and heap:
        p, u, v, vu, vv = heapq.heappop(heap)
        if not (alive[u] and alive[v]) or version[u] != vu or version[v] != vv:
            continue
        shared = vfaces[u] & vfaces[v]
        if len(shared) != 2:
            continue
        opp = set()
        for fi in shared:
            opp.update(faces[fi])
        opp -= {u, v}
        if neighbours(u) & neighbours(v) != opp:
            continue  # link condition violated
        newp = (V[u] + V[v]) * 0.5
        newp /= np.linalg.norm(newp)
        # orientation check on every face that survives around u and v
        ok = True
        for fi in (vfaces[u] | vfaces[v]) - shared:
            f = [u if x == v else x for x in faces[fi]]
            P = [newp if x == u else V[x] for x in f]
            n = np.cross(P[1] - P[0], P[2] - P[0])
            if float(n @ (P[0] + P[1] + P[2])) <= 1e-12:
                ok = False
                break
        if not ok:
            continue
        # perform collapse v -> u
        for fi in shared:
            for x in faces[fi]:
                vfaces[x].discard(fi)
            del faces[fi]
        for fi in list(vfaces[v]):
            faces[fi] = [u if x == v else x for x in faces[fi]]
            vfaces[u].add(fi)
        vfaces[v].clear()
        alive[v] = False
        V[u] = newp
        version[u] += 1
        nf -= 2
        for w in neighbours(u):
            a, b = min(u, w), max(u, w)
            heapq.heappush(heap, (prio(a, b), a, b, int(version[a]), int(version[b])))
    if nf != target_faces:
        raise RuntimeError(f"decimation stalled at {nf} faces (target {target_faces})")
    keep = np.nonzero(alive)[0]
    remap = -np.ones(len(V), dtype=np.int64)
    remap[keep] = np.arange(len(keep))
    Fo = np.array([[remap[x] for x in f] for f in faces.values()], dtype=np.int64)
    return V[keep].copy(), _canonical_faces(Fo)
