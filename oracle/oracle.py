"""ctypes wrapper of the FP64 CPU oracle (oracle.cpp).

Test infrastructure only: the tests, the smoke check and the benchmark's
CPU-baseline leg may import it; the library never does.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OK, E_ARG, E_MESH, E_GENUS, E_INFEASIBLE, E_NONFINITE = 0, -1, -2, -3, -4, -5


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b  # noqa: F401  (package import)
        _LIB = C.CDLL(path)
        L = _LIB
        P = C.c_void_p
        L.or_mesh_check.argtypes = [C.c_int, C.c_int, P, P]
        L.or_mesh_edges.argtypes = [C.c_int, C.c_int, P, P, P]
        L.or_mixed_areas.argtypes = [C.c_int, C.c_int, P, P, P]
        L.or_knn.argtypes = [C.c_int, P, C.c_int, P, C.c_int, C.c_int, P, P]
        L.or_desc_dist.argtypes = [C.c_int, P, P, P, P, C.c_int, P]
        L.or_space_build.argtypes = [C.c_int, C.c_int, P, P, C.c_int, C.c_int, P, P, P, P,
                                     C.c_int, P]
        L.or_space_build.restype = C.c_void_p
        L.or_ilp_build.argtypes = [C.c_int, C.c_int, P, P, P, P, P]
        L.or_ilp_build.restype = C.c_void_p
        L.or_space_free.argtypes = [P]
        L.or_space_info.argtypes = [P, P]
        L.or_space_get.argtypes = [P, C.c_int, P]
        L.or_space_costs.argtypes = [P, P, P, C.c_int]
        L.or_space_set_costs.argtypes = [P, P]
        L.or_init_lambda.argtypes = [P, P]
        L.or_dual_solve.argtypes = [P, C.c_int, C.c_double, C.c_double, P, P, C.c_int]
        L.or_lower_bound.argtypes = [P, P, C.c_double]
        L.or_lower_bound.restype = C.c_double
        L.or_min_marginals.argtypes = [P, P, C.c_double, P, P, P]
        L.or_row_dp.argtypes = [C.c_int, P, C.c_int, P, C.c_double, P, P]
        L.or_row_dp.restype = C.c_double
        L.or_check_primal.argtypes = [P, P]
        L.or_check_primal.restype = C.c_int64
        L.or_round.argtypes = [P, P, C.c_int, C.c_int, C.c_double, C.c_double, C.c_uint64,
                               C.c_double, P, P, P, P]
        L.or_uniform_pm1.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32]
        L.or_uniform_pm1.restype = C.c_double
        L.or_smoothed_grad.argtypes = [P, P, C.c_double, P, P, C.c_int, P, P, P, P]
        L.or_smoothed_value_phi.argtypes = [P, P, P, C.c_double]
        L.or_smoothed_value_phi.restype = C.c_double
        L.or_costs_for.argtypes = [P, P, P, C.c_int, P]
        L.or_lbfgs_solve.argtypes = [P, C.c_int, C.c_double, C.c_int, C.c_int, C.c_double,
                                     C.c_double, C.c_double, C.c_double, P, P, P, P]
        L.or_subgradient.argtypes = [P, P, P]
        L.or_project_feasible.argtypes = [P, P]
        L.or_confident_fix.argtypes = [P, P, C.c_double, P, P, P]
        L.or_fix_variables.argtypes = [P, P]
        L.or_lbfgs_direction.argtypes = [C.c_int, C.c_int, P, P, P, P]
        L.or_find_step_parabola.argtypes = [C.c_double, C.c_double, C.c_int, C.c_double,
                                            C.c_double, C.c_double, P]
        L.or_find_step_parabola.restype = C.c_double
    return _LIB


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle status {code}")
        self.code = code


def mesh_check(F, nv):
    F = _c(F, np.int32)
    ne = C.c_int(0)
    st = lib().or_mesh_check(nv, len(F), _p(F), C.byref(ne))
    return st, ne.value


def mesh_edges(F, nv):
    F = _c(F, np.int32)
    st, ne = mesh_check(F, nv)
    if st:
        raise OracleError(st)
    E = np.zeros((ne, 2), np.int32)
    FE = np.zeros((len(F), 3), np.int32)
    lib().or_mesh_edges(nv, len(F), _p(F), _p(E), _p(FE))
    return E, FE


def mixed_areas(V, F):
    V = _c(V, np.float32)
    F = _c(F, np.int32)
    out = np.zeros(len(V), np.float64)
    st = lib().or_mixed_areas(len(V), len(F), _p(V), _p(F), _p(out))
    if st:
        raise OracleError(st)
    return out


def knn(DX, DY, K):
    DX = _c(DX, np.float32)
    DY = _c(DY, np.float32)
    cxy = np.zeros((len(DX), K), np.int32)
    cyx = np.zeros((len(DY), K), np.int32)
    st = lib().or_knn(len(DX), _p(DX), len(DY), _p(DY), DX.shape[1], K, _p(cxy), _p(cyx))
    if st:
        raise OracleError(st)
    return cxy, cyx


def desc_dist(DX, DY, m_idx, n_idx):
    DX = _c(DX, np.float32)
    DY = _c(DY, np.float32)
    m_idx = _c(m_idx, np.int32)
    n_idx = _c(n_idx, np.int32)
    out = np.zeros(len(m_idx), np.float64)
    lib().or_desc_dist(len(m_idx), _p(m_idx), _p(n_idx), _p(DX), _p(DY), DX.shape[1], _p(out))
    return out


def row_dp(coef, b, lam, T=0.0):
    coef = _c(coef, np.int32)
    lam = _c(lam, np.float64)
    M = np.zeros(len(lam))
    mu = np.zeros(len(lam))
    v = lib().or_row_dp(len(lam), _p(coef), int(b), _p(lam), float(T), _p(M), _p(mu))
    return v, M, mu


def uniform_pm1(seed, r, i):
    return lib().or_uniform_pm1(seed, r, i)


def lbfgs_direction(S, Y, g):
    """Two-loop recursion d = H g over history pairs S[j], Y[j] (oldest first)."""
    g = _c(g, np.float64)
    S = _c(np.reshape(S, (-1, len(g))), np.float64)
    Y = _c(np.reshape(Y, (-1, len(g))), np.float64)
    d = np.zeros(len(g))
    lib().or_lbfgs_direction(len(g), S.shape[0], _p(S), _p(Y), _p(g), _p(d))
    return d


def find_step_parabola(c, gamma, K=5, a_up=1.1, a_down=0.8, dmin=float("inf")):
    """FindStepSize on E(gamma) = -(gamma - c)^2 starting from gamma (E_init = E(0))."""
    e = C.c_double(0)
    gm = lib().or_find_step_parabola(float(c), float(gamma), int(K), float(a_up),
                                     float(a_down), float(dmin), C.byref(e))
    return gm, e.value


class Space:
    """Product space + presolved ILP + costs, held by the oracle."""

    INFO = ("nP", "n_rows_full", "nnz_full", "n_closed_full", "n_free", "n_fixed1",
            "n_rows", "nnz")

    def __init__(self, VX, FX, VY, FY, cand_xy, cand_yx):
        self._keep = [_c(VX, np.float32), _c(FX, np.int32), _c(VY, np.float32),
                      _c(FY, np.int32), _c(cand_xy, np.int32), _c(cand_yx, np.int32)]
        VX, FX, VY, FY, cxy, cyx = self._keep
        st = C.c_int(0)
        self.h = lib().or_space_build(len(VX), len(FX), _p(VX), _p(FX), len(VY), len(FY),
                                      _p(VY), _p(FY), _p(cxy), _p(cyx), cxy.shape[1],
                                      C.byref(st))
        if not self.h:
            raise OracleError(st.value)
        self.info = self._read_info()
        self.nvx, self.nvy = len(VX), len(VY)
        self.nfx, self.nfy = len(FX), len(FY)

    @classmethod
    def from_ilp(cls, n_vars, row_ptr, cols, coefs, b):
        """Generic 0-1 ILP with +-1 rows (CSR): one subproblem per input
        row, rows reordered [other rows | exactly-one rows], presolved (see
        or_ilp_build)."""
        S = cls.__new__(cls)
        S._keep = [_c(row_ptr, np.int32), _c(cols, np.int32), _c(coefs, np.int32), _c(b, np.int32)]
        rp, cl, cf, bb = S._keep
        st = C.c_int(0)
        S.h = lib().or_ilp_build(int(n_vars), len(rp) - 1, _p(rp), _p(cl), _p(cf), _p(bb), C.byref(st))
        if not S.h:
            raise OracleError(st.value)
        S.info = S._read_info()
        S.nvx = S.nvy = S.nfx = S.nfy = 0
        return S

    def _read_info(self):
        info = np.zeros(8, np.int64)
        lib().or_space_info(self.h, _p(info))
        return dict(zip(self.INFO, (int(x) for x in info)))

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_space_free(self.h)
            self.h = None

    def get(self, name):
        i = self.info
        spec = {
            "pv": (0, np.int32, (i["nP"], 3)),
            "code": (1, np.int32, (i["nP"], 4)),
            "state": (2, np.int8, (i["nP"],)),
            "row_key": (3, np.int64, (i["n_rows_full"],)),
            "row_ptr": (4, np.int64, (i["n_rows_full"] + 1,)),
            "ent_var": (5, np.int64, (i["nnz_full"],)),
            "ent_coef": (6, np.int32, (i["nnz_full"],)),
            "row_b": (7, np.int32, (i["n_rows_full"],)),
            "free_var": (8, np.int64, (i["n_free"],)),
            "rrow_orig": (9, np.int64, (i["n_rows"],)),
            "rrow_ptr": (10, np.int64, (i["n_rows"] + 1,)),
            "rent_var": (11, np.int64, (i["nnz"],)),
            "rent_coef": (12, np.int32, (i["nnz"],)),
            "rrow_b": (13, np.int32, (i["n_rows"],)),
            "deg": (14, np.int32, (i["n_free"],)),
            "cost": (15, np.float64, (i["nP"],)),
            "offset": (16, np.float64, (1,)),
            "cand": (17, np.uint8, (self.nvx, self.nvy)),
        }[name]
        out = np.zeros(spec[2], spec[1])
        st = lib().or_space_get(self.h, spec[0], _p(out))
        if st:
            raise OracleError(st)
        return out

    def costs(self, DX, DY):
        DX = _c(DX, np.float32)
        DY = _c(DY, np.float32)
        st = lib().or_space_costs(self.h, _p(DX), _p(DY), DX.shape[1])
        if st:
            raise OracleError(st)
        return self.get("cost")

    def costs_for(self, DX, DY):
        """Element costs for other descriptors, without changing the state."""
        DX = _c(DX, np.float32)
        DY = _c(DY, np.float32)
        out = np.zeros(self.info["nP"])
        st = lib().or_costs_for(self.h, _p(DX), _p(DY), DX.shape[1], _p(out))
        if st:
            raise OracleError(st)
        return out

    def set_costs(self, cost):
        cost = _c(cost, np.float64)
        lib().or_space_set_costs(self.h, _p(cost))

    @property
    def offset(self):
        return float(self.get("offset")[0])

    def init_lambda(self):
        lam = np.zeros(self.info["nnz"])
        st = lib().or_init_lambda(self.h, _p(lam))
        if st:
            raise OracleError(st)
        return lam

    def dual_solve(self, iters, omega=0.5, T=0.0, lam=None):
        init = lam is None
        lam = np.zeros(self.info["nnz"]) if init else _c(lam, np.float64).copy()
        trace = np.zeros(max(iters, 1))
        st = lib().or_dual_solve(self.h, iters, omega, T, _p(lam), _p(trace), int(init))
        if st:
            raise OracleError(st)
        return lam, trace[:iters]

    def lbfgs_solve(self, iters, lam=None, omega=0.5, m=5, K=5, eps=1e-8, a_up=1.1,
                    a_down=0.8, gamma0=0.1):
        """Quasi-newton powered MMA (Alg. 1); returns lambda, E per iteration
        (iters + 1 values: before each iteration and at the end), the step size
        after each FindStepSize and whether the step was taken."""
        lam = self.init_lambda() if lam is None else _c(lam, np.float64).copy()
        tE = np.zeros(iters + 1)
        tg = np.zeros(max(iters, 1))
        tk = np.zeros(max(iters, 1), np.int32)
        st = lib().or_lbfgs_solve(self.h, int(iters), float(omega), int(m), int(K), float(eps),
                                  float(a_up), float(a_down), float(gamma0), _p(lam), _p(tE),
                                  _p(tg), _p(tk))
        if st:
            raise OracleError(st)
        return lam, tE, tg[:iters], tk[:iters].astype(bool)

    def subgradient(self, lam):
        """Per entry: 1 where the row's minimising assignment sets the variable."""
        lam = _c(lam, np.float64)
        g = np.zeros(self.info["nnz"])
        lib().or_subgradient(self.h, _p(lam), _p(g))
        return g

    def confident_fix(self, lam, frac=0.9):
        """Fixings of the coarse-to-fine appendix: per element -1 (free) or the
        value it is fixed to (presolve fixings and the newly fixed confident
        variables); also the numbers of agreeing and of newly fixed variables."""
        lam = _c(lam, np.float64)
        fix = np.zeros(self.info["nP"], np.int8)
        na, nf = C.c_int64(0), C.c_int64(0)
        st = lib().or_confident_fix(self.h, _p(lam), float(frac), _p(fix), C.byref(na), C.byref(nf))
        if st:
            raise OracleError(st)
        return fix, na.value, nf.value

    def fix_variables(self, fix=None):
        """Re-presolve from the fixings (None: the original problem); the
        reduced problem becomes the residual one."""
        f = None if fix is None else _c(fix, np.int8)
        st = lib().or_fix_variables(self.h, _p(f) if f is not None else None)
        if st:
            raise OracleError(st)
        self.info = self._read_info()

    def project_feasible(self, d):
        """Subtract from every entry the mean over its variable's entries."""
        d = _c(d, np.float64).copy()
        lib().or_project_feasible(self.h, _p(d))
        return d

    def lower_bound(self, lam, T=0.0):
        lam = _c(lam, np.float64)
        return lib().or_lower_bound(self.h, _p(lam), float(T))

    def min_marginals(self, lam, T=0.0):
        lam = _c(lam, np.float64)
        M = np.zeros(self.info["nnz"])
        rm = np.zeros(self.info["n_rows"])
        mu = np.zeros(self.info["nnz"])
        lib().or_min_marginals(self.h, _p(lam), float(T), _p(M), _p(rm), _p(mu))
        return M, rm, mu

    def check_primal(self, x):
        x = _c(x, np.uint8)
        return int(lib().or_check_primal(self.h, _p(x)))

    def round(self, lam, R=30, T_iters=25, delta0=0.0, gamma=1.5, seed=0, omega=0.5):
        lam = _c(lam, np.float64)
        x = np.zeros(self.info["nP"], np.uint8)
        p = C.c_double(0)
        feas = C.c_int(0)
        rounds = C.c_int(0)
        st = lib().or_round(self.h, _p(lam), R, T_iters, float(delta0), float(gamma),
                            C.c_uint64(seed), float(omega), _p(x), C.byref(p), C.byref(feas),
                            C.byref(rounds))
        if st:
            raise OracleError(st)
        return x, p.value, bool(feas.value), rounds.value

    def smoothed_grad(self, lam, T, DX, DY):
        lam = _c(lam, np.float64)
        DX = _c(DX, np.float32)
        DY = _c(DY, np.float32)
        gc = np.zeros(self.info["nP"])
        gX = np.zeros(DX.shape)
        gY = np.zeros(DY.shape)
        v = C.c_double(0)
        st = lib().or_smoothed_grad(self.h, _p(lam), float(T), _p(DX), _p(DY), DX.shape[1],
                                    _p(gc), _p(gX), _p(gY), C.byref(v))
        if st:
            raise OracleError(st)
        return v.value, gc, gX, gY

    def smoothed_value_phi(self, cost, phi, T):
        cost = _c(cost, np.float64)
        phi = _c(phi, np.float64)
        return lib().or_smoothed_value_phi(self.h, _p(cost), _p(phi), float(T))


def unpruned_count(nvx, nex, nfx, nvy, ney, nfy):
    """Closed-form size of the unpruned product space (tri-tri 3 FxFy,
    tri-edge / edge-tri 6 per pair, tri-vertex / vertex-tri 1 per pair)."""
    return 3 * nfx * nfy + 6 * (nfx * ney + nex * nfy) + nfx * nvy + nvx * nfy


# ---------------------------------------------------------------- coarse-to-fine pruning (Sec. 5.2)
# Plain set logic: a coarse vertex match (m, n) admits every fine pair
# (u, v) with u in the ring neighbourhood of m's location on X and v in that
# of n's location on Y.

def nearest_vertices(P, Q):
    """Index of the nearest point of Q for every point of P: squared
    distances in FP64 (exact for FP32 coordinates), ties to the lower index
    (argmin returns the first minimum)."""
    P = np.asarray(P, np.float32).astype(np.float64)
    Q = np.asarray(Q, np.float32).astype(np.float64)
    out = np.empty(len(P), np.int32)
    for i, p in enumerate(P):
        d = Q - p
        out[i] = int(np.argmin((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]))
    return out


def matched_pairs(pv, x, nvy):
    """Vertex pairs (m, n) used by the elements with x = 1 (their product
    vertices m * nvy + n), ascending."""
    ids = np.unique(np.asarray(pv)[np.asarray(x).astype(bool)].ravel())
    return np.stack([ids // nvy, ids % nvy], axis=1).astype(np.int32)


def vertex_rings(F, nv, rings):
    """Ring neighbourhood of every vertex of a closed mesh: the vertex and its
    edge neighbours (rings = 1), and theirs (rings = 2), as sets."""
    nb = [set() for _ in range(nv)]
    for a, b, c in np.asarray(F):
        for u, v in ((a, b), (b, c), (c, a)):
            nb[u].add(int(v))
            nb[v].add(int(u))
    out = []
    for v in range(nv):
        r = {v} | nb[v]
        if rings >= 2:
            for u in list(nb[v]):
                r |= nb[u]
        out.append(r)
    return out


def ring_candidates(FX, nvx, FY, nvy, seeds, rings):
    """Union over seed pairs (a, b) of ring(a) x ring(b); per-vertex lists in
    ascending order both ways, padded to the common length K by repeating
    the last entry.  Returns (cand_xy [nvx, K], cand_yx [nvy, K])."""
    rx, ry = vertex_rings(FX, nvx, rings), vertex_rings(FY, nvy, rings)
    xs = [set() for _ in range(nvx)]
    ys = [set() for _ in range(nvy)]
    for a, b in np.asarray(seeds):
        for u in rx[int(a)]:
            xs[u] |= ry[int(b)]
        for v in ry[int(b)]:
            ys[v] |= rx[int(a)]
    K = max(max(len(s) for s in xs), max(len(s) for s in ys))

    def lists(sets):
        out = np.empty((len(sets), K), np.int32)
        for i, s in enumerate(sets):
            srt = sorted(s)
            if not srt:
                raise OracleError(E_INFEASIBLE)
            out[i] = srt + [srt[-1]] * (K - len(srt))
        return out
    return lists(xs), lists(ys)
