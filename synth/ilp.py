"""Seeded synthetic 0-1 ILPs with +-1 rows (input generator only)."""
import numpy as np


def generic_ilp(n, n_side, seed, side_len=(3, 6)):
    """Seeded 0-1 ILP with +-1 rows: an n x n assignment (x_ij, exactly-one
    rows per i and per j) plus n_side rows of 3 to 6 random +-1 entries whose
    right-hand sides a planted permutation satisfies (so the ILP is
    feasible), costs uniform in [0, 1).  Returns (n_vars, row_ptr, cols,
    coefs, b, cost)."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    xstar = np.zeros(n * n, np.int64)
    xstar[np.arange(n) * n + perm] = 1
    rows = [([i * n + j for j in range(n)], [1] * n, 1) for i in range(n)]
    rows += [([i * n + j for i in range(n)], [1] * n, 1) for j in range(n)]
    deg = np.full(n * n, 2)
    for _ in range(n_side):
        k = int(rng.integers(side_len[0], side_len[1] + 1))
        pool = np.nonzero(deg < 5)[0]
        vs = rng.choice(pool, size=min(k, len(pool)), replace=False)
        cs = rng.choice([-1, 1], size=len(vs))
        deg[vs] += 1
        rows.append((vs.tolist(), cs.tolist(), int(cs @ xstar[vs])))
    rp = np.cumsum([0] + [len(r[0]) for r in rows]).astype(np.int32)
    cols = np.concatenate([r[0] for r in rows]).astype(np.int32)
    coefs = np.concatenate([r[1] for r in rows]).astype(np.int8)
    b = np.array([r[2] for r in rows], np.int32)
    return n * n, rp, cols, coefs, b, rng.uniform(0.0, 1.0, n * n)
