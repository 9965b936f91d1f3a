"""Independent checkers used by the tests: exhaustive search over tiny ILPs,
a from-scratch check of the matching constraints, and small utilities.

Nothing here imports the library; nothing here shares code with the oracle.
"""
from __future__ import annotations

import numpy as np


def reduced_rows(S):
    """Rows of an oracle space's presolved problem as (vars, coefs, b)."""
    rp = S.get("rrow_ptr")
    rv = S.get("rent_var")
    rc = S.get("rent_coef")
    rb = S.get("rrow_b")
    return [(rv[rp[j]:rp[j + 1]].copy(), rc[rp[j]:rp[j + 1]].copy(), int(rb[j]))
            for j in range(len(rb))]


def full_rows(S):
    rp = S.get("row_ptr")
    rv = S.get("ent_var")
    rc = S.get("ent_coef")
    rb = S.get("row_b")
    return [(rv[rp[j]:rp[j + 1]].copy(), rc[rp[j]:rp[j + 1]].copy(), int(rb[j]))
            for j in range(len(rb))]


def _propagate(s, rows, var_rows, start=None):
    """Unit propagation on 0/1 equality rows (from the rows in ``start``, all
    rows if None); returns False on conflict."""
    queue = list(range(len(rows))) if start is None else list(start)
    inq = [False] * len(rows)
    for j in queue:
        inq[j] = True
    while queue:
        j = queue.pop()
        inq[j] = False
        vs, cs, b = rows[j]
        r = b
        P = N = 0
        for v, a in zip(vs, cs):
            if s[v] == 1:
                r -= a
            elif s[v] < 0:
                if a > 0:
                    P += 1
                else:
                    N += 1
        if r < -N or r > P:
            return False
        for v, a in zip(vs, cs):
            if s[v] >= 0:
                continue
            Pr, Nr = P - (a > 0), N - (a < 0)
            one = -Nr <= r - a <= Pr
            zero = -Nr <= r <= Pr
            if not one and not zero:
                return False
            if one != zero:
                s[v] = 1 if one else 0
                if one:
                    r -= a
                if a > 0:
                    P -= 1
                else:
                    N -= 1
                for k in var_rows[v]:
                    if not inq[k]:
                        inq[k] = True
                        queue.append(k)
    return True


def enumerate_ilp(rows, nvar, cost, limit=200000):
    """All 0/1 solutions of the rows by depth-first search with propagation.

    Returns (optimum, number of optimal solutions within 1e-9, number of
    feasible solutions, list of optimal assignments)."""
    var_rows = [[] for _ in range(nvar)]
    for j, (vs, _, _) in enumerate(rows):
        for v in vs:
            var_rows[v].append(j)
    best = [np.inf]
    opts = []
    count = [0]

    def rec(s, start):
        if not _propagate(s, rows, var_rows, start):
            return
        free_rows = []
        for j, (vs, _, _) in enumerate(rows):
            nf = int(np.sum(s[vs] < 0))
            if nf:
                free_rows.append((nf, j))
        if not free_rows:
            if np.any(s < 0):   # variable in no row: c >= 0 -> 0
                s = s.copy()
                s[s < 0] = 0
            count[0] += 1
            if count[0] > limit:
                raise RuntimeError("too many solutions")
            val = float(cost @ s)
            if val < best[0] - 1e-9:
                best[0] = val
                opts.clear()
                opts.append(s.copy())
            elif abs(val - best[0]) <= 1e-9:
                opts.append(s.copy())
            return
        _, j = min(free_rows)
        vs = rows[j][0]
        v = next(int(x) for x in vs if s[x] < 0)
        for val in (1, 0):
            t = s.copy()
            t[v] = val
            rec(t, var_rows[v])

    rec(-np.ones(nvar, dtype=np.int64), None)
    return best[0], len(opts), count[0], opts


def matching_violations(pv, code, nfx, nfy, x):
    """Check a 0/1 selection of product triangles against the definition of a
    discrete diffeomorphism, from scratch: every face of X and of Y covered
    exactly once, and every undirected product edge traversed equally often
    in both directions.  Returns the number of violated conditions."""
    sel = np.nonzero(np.asarray(x) != 0)[0]
    bad = 0
    covx = np.zeros(nfx, np.int64)
    covy = np.zeros(nfy, np.int64)
    for p in sel:
        if code[p, 0] == 0:
            covx[code[p, 1]] += 1
        if code[p, 2] // 8 == 0:
            covy[code[p, 3]] += 1
    bad += int(np.sum(covx != 1)) + int(np.sum(covy != 1))
    bal = {}
    for p in sel:
        for k in range(3):
            a, b = int(pv[p, k]), int(pv[p, (k + 1) % 3])
            key = (min(a, b), max(a, b))
            bal[key] = bal.get(key, 0) + (1 if a < b else -1)
    bad += sum(1 for v in bal.values() if v != 0)
    return bad


def full_candidates(nvx, nvy):
    """Candidate lists whose union is every vertex pair (K = min(nvx, nvy))."""
    K = min(nvx, nvy)
    cxy = np.array([[(m + k) % nvy for k in range(K)] for m in range(nvx)], np.int32)
    cyx = np.array([[(n + k) % nvx for k in range(K)] for n in range(nvy)], np.int32)
    return cxy, cyx, K


def milp_optimum(S):
    """Exact ILP optimum of the oracle space's current (reduced) problem by
    HiGHS, offset included; None when HiGHS finds it infeasible."""
    from scipy.optimize import Bounds, LinearConstraint, milp
    from scipy.sparse import csr_matrix
    n = S.info["n_free"]
    if n == 0:
        return S.offset
    rows = reduced_rows(S)
    c = S.get("cost")[S.get("free_var")]
    r = np.concatenate([[j] * len(vs) for j, (vs, _, _) in enumerate(rows)])
    A = csr_matrix((np.concatenate([cs for _, cs, _ in rows]).astype(float),
                    (r, np.concatenate([vs for vs, _, _ in rows]))), shape=(len(rows), n))
    b = np.array([b for _, _, b in rows], float)
    res = milp(c, constraints=LinearConstraint(A, b, b), integrality=np.ones(n), bounds=Bounds(0, 1))
    return res.fun + S.offset if res.status == 0 else None



def bf16_rne(a):
    """Round float32 values to bfloat16 (round to nearest, ties to even),
    returned as float32."""
    u = np.ascontiguousarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + (((u >> 16) & 1) + 0x7FFF)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)
