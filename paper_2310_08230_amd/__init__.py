"""Python binding of libdiscomatch (gfx950): argument marshalling only.

Every step of the solver runs in the HIP library; this module passes device
pointers of torch tensors and the current torch stream through the C ABI of
include/discomatch.h and raises on any error.  The library must have been
built (paper_2310_08230_amd/build.py); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdiscomatch.so")

DM_OK = 0
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
ERRORS = {-1: "invalid argument", -2: "mesh", -3: "genus", -4: "infeasible", -5: "non-finite",
          -6: "workspace", -7: "hip", -8: "state"}
ARRAYS = ["pv", "code", "state", "row_key", "row_ptr", "ent_var", "ent_coef", "row_b", "free_var",
          "rrow_orig", "rrow_ptr", "rent_var", "rent_coef", "rrow_b", "edges_x", "edges_y", "cand"]

_lib = None


class DMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"discomatch error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class dm_mesh(C.Structure):
    _fields_ = [("nv", C.c_int32), ("nf", C.c_int32), ("verts", C.c_void_p), ("faces", C.c_void_p)]


class dm_space_info(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_prod_tri", "n_rows_full", "nnz_full", "n_closed_full",
                                         "n_free", "n_fixed1", "n_rows", "nnz", "n_short_rows",
                                         "n_edges_x", "n_edges_y", "n_cand")] + \
               [("presolve_rounds", C.c_int32), ("max_short_row", C.c_int32)]


class dm_round_params(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("iters_per_round", C.c_int32), ("delta0", C.c_double),
                ("gamma", C.c_double), ("seed", C.c_uint64), ("omega", C.c_double),
                ("msg_prec", C.c_int32)]


class dm_search_params(C.Structure):
    _fields_ = [("max_nodes", C.c_int32), ("dual_iters", C.c_int32), ("omega", C.c_double),
                ("rel_tol", C.c_double), ("round", dm_round_params)]


SEARCH_STATUS = {-1: "infeasible", 0: "limit", 1: "optimal"}


class dm_lbfgs_params(C.Structure):
    _fields_ = [("history", C.c_int32), ("max_search", C.c_int32), ("omega", C.c_double),
                ("eps", C.c_double), ("step_up", C.c_double), ("step_down", C.c_double),
                ("gamma0", C.c_double), ("resume", C.c_int32)]


def lib():
    """Load libdiscomatch.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built; run paper_2310_08230_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, F, D = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_double
        sig = {
            "dm_create": [I32, P, P],
            "dm_destroy": [P],
            "dm_set_stream": [P, P],
            "dm_knn_candidates": [P, P, I32, P, I32, I32, I32, I32, P, P],
            "dm_knn_candidates_noalloc": [P, P, I32, P, I32, I32, I32, I32, P, P],
            "dm_build_product_space": [P, P, P, P, P, I32, P],
            "dm_get_space": [P, I32, P],
            "dm_build_costs": [P, P, P, I32, I32, P],
            "dm_init_lambda": [P, I32, P],
            "dm_dual_solve": [P, I32, D, D, I32, P, P],
            "dm_lower_bound": [P, P, D, I32, P],
            "dm_round_primal": [P, P, P, P, P, P, P],
            "dm_check_primal": [P, P, P],
            "dm_smoothed_backward": [P, P, D, I32, D, P, P, I32, P, P, P, P],
            "dm_mixed_areas": [P, P, P],
            "dm_timing_enable": [P, I32],
            "dm_timing_read": [P, P, P],
            "dm_lbfgs_solve": [P, I32, P, I32, P, P, P, P],
            "dm_subgradient": [P, I32, P, P, P],
            "dm_lbfgs_direction": [P, I32, I32, P, P, P, P],
            "dm_confident_fixing": [P, I32, P, D, P, P, P],
            "dm_fix_variables": [P, P, P],
            "dm_build_ilp": [P, I32, I32, P, P, P, P, P],
            "dm_set_costs": [P, P],
            "dm_nearest_vertices": [P, P, I32, P, I32, P],
            "dm_matched_pairs": [P, P, P, I32, P],
            "dm_ring_candidates": [P, P, P, P, I32, I32, I32, P, P, P],
            "dm_exact_search": [P, P, P, P, P, P, P, P, P],
            "dm_repair_primal": [P, P, I32, P, P, P, P, P],
            "dm_workspace_query": [P, I32, P],
            "dm_set_workspace": [P, I32, P, C.c_size_t],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = I32
        L.dm_last_error.argtypes = [P]
        L.dm_last_error.restype = C.c_char_p
        L.dm_version.argtypes = []
        L.dm_version.restype = C.c_char_p
        _lib = L
    return _lib


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, device):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    return t.to(device=device, dtype=dtype).contiguous()


class Context:
    """One library context on one GPU; work goes on the current torch stream."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("discomatch needs a ROCm GPU")
        self.device = torch.device("cuda", device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            st = lib().dm_create(device, C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(h))
        if st != DM_OK:
            raise DMError(st, "dm_create failed")
        self.h = h
        self.info = None
        self._keep = []
        # counts the calls that replace the problem or its costs; a smoothed
        # bound's backward pass must see the problem its forward pass solved
        self.generation = 0

    def close(self):
        if getattr(self, "h", None):
            lib().dm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    _CHANGES_PROBLEM = frozenset(("dm_build_product_space", "dm_build_ilp", "dm_build_costs", "dm_set_costs",
                                  "dm_fix_variables", "dm_exact_search"))

    def _call(self, name, *args):
        if name in self._CHANGES_PROBLEM:
            self.generation += 1
        L = lib()
        L.dm_set_stream(self.h, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))
        st = getattr(L, name)(self.h, *args)
        if st != DM_OK:
            raise DMError(st, L.dm_last_error(self.h).decode())

    # -- caller-owned solver state ----------------------------------------
    WS_STAGE = {"fp32": 0, "fp64": 1}

    def workspace_bytes(self, msg_prec="fp32"):
        """Bytes of the Jacobi solver state of one message precision for the
        current problem (dm_workspace_query)."""
        n = C.c_size_t(0)
        st = lib().dm_workspace_query(self.h, self.WS_STAGE[msg_prec], C.byref(n))
        if st != DM_OK:
            raise DMError(st, "dm_workspace_query failed (is a problem built?)")
        return n.value

    def set_workspace(self, msg_prec="fp32", buf=None):
        """Keep the solver state of one message precision in ``buf``, a device
        tensor owned by the caller (at least workspace_bytes(msg_prec) bytes,
        256-byte aligned, e.g. torch.empty(n, dtype=torch.uint8, device=...));
        None detaches.  The context holds a reference while attached."""
        if buf is None:
            self._call("dm_set_workspace", self.WS_STAGE[msg_prec], None, 0)
            self._ws = {k: v for k, v in getattr(self, "_ws", {}).items() if k != msg_prec}
            return
        nbytes = buf.numel() * buf.element_size()
        self._call("dm_set_workspace", self.WS_STAGE[msg_prec], C.c_void_p(buf.data_ptr()), nbytes)
        self._ws = dict(getattr(self, "_ws", {}))
        self._ws[msg_prec] = buf

    # -- A2 -------------------------------------------------------------
    def knn_candidates(self, DX, DY, K, prec="fp32"):
        DX = _dev(DX, torch.float32, self.device)
        DY = _dev(DY, torch.float32, self.device)
        cxy = torch.empty((DX.shape[0], K), dtype=torch.int32, device=self.device)
        cyx = torch.empty((DY.shape[0], K), dtype=torch.int32, device=self.device)
        self._call("dm_knn_candidates", _ptr(DX), DX.shape[0], _ptr(DY), DY.shape[0], DX.shape[1], K,
                   PREC[prec], _ptr(cxy), _ptr(cyx))
        return cxy, cyx

    def knn_candidates_noalloc(self, DX, DY, K, prec="fp32", out=None):
        """As knn_candidates, through the entry point that allocates nothing
        (its temporaries live in the library's fixed per-GPU scratch array);
        out = (cand_xy, cand_yx) int32 tensors to write, else new ones."""
        DX = _dev(DX, torch.float32, self.device)
        DY = _dev(DY, torch.float32, self.device)
        if out is None:
            out = (torch.empty((DX.shape[0], K), dtype=torch.int32, device=self.device),
                   torch.empty((DY.shape[0], K), dtype=torch.int32, device=self.device))
        cxy, cyx = out
        self._call("dm_knn_candidates_noalloc", _ptr(DX), DX.shape[0], _ptr(DY), DY.shape[0], DX.shape[1], K,
                   PREC[prec], _ptr(cxy), _ptr(cyx))
        return cxy, cyx

    # -- A1, A3 ---------------------------------------------------------
    def build_product_space(self, VX, FX, VY, FY, cand_xy, cand_yx):
        VX = _dev(VX, torch.float32, self.device)
        VY = _dev(VY, torch.float32, self.device)
        FX = _dev(FX, torch.int32, self.device)
        FY = _dev(FY, torch.int32, self.device)
        cxy = _dev(cand_xy, torch.int32, self.device)
        cyx = _dev(cand_yx, torch.int32, self.device)
        mx = dm_mesh(VX.shape[0], FX.shape[0], VX.data_ptr(), FX.data_ptr())
        my = dm_mesh(VY.shape[0], FY.shape[0], VY.data_ptr(), FY.data_ptr())
        info = dm_space_info()
        self._call("dm_build_product_space", C.byref(mx), C.byref(my), _ptr(cxy), _ptr(cyx),
                   cxy.shape[1], C.byref(info))
        self.info = {n: getattr(info, n) for n, _ in dm_space_info._fields_}
        self.nvx, self.nvy = VX.shape[0], VY.shape[0]
        return self.info

    # -- coarse-to-fine pruning (Sec. 5.2) ------------------------------
    def nearest_vertices(self, P, Q):
        """For each point of P the index of the nearest point of Q (FP64
        squared distances, ties to the lower index)."""
        P = _dev(P, torch.float32, self.device)
        Q = _dev(Q, torch.float32, self.device)
        out = torch.empty(P.shape[0], dtype=torch.int32, device=self.device)
        self._call("dm_nearest_vertices", _ptr(P), P.shape[0], _ptr(Q), Q.shape[0], _ptr(out))
        return out

    def matched_pairs(self, x):
        """Vertex pairs (m, n) used by the selected elements of x, as an
        int32 [k, 2] tensor in ascending order of m * nvY + n."""
        x = _dev(x, torch.uint8, self.device)
        cap = 3 * max(int(x.sum().item()), 1)
        pairs = torch.empty((cap, 2), dtype=torch.int32, device=self.device)
        n = C.c_int32(0)
        self._call("dm_matched_pairs", _ptr(x), _ptr(pairs), cap, C.byref(n))
        return pairs[:n.value]

    def ring_candidates(self, VX, FX, VY, FY, seeds, rings=2, kcap=512):
        """Candidate lists of the fine meshes (VX, FX), (VY, FY) from seed
        vertex pairs: ring(a) x ring(b) for every seed (a, b); returns
        (cand_xy [nvX, K], cand_yx [nvY, K])."""
        VX = _dev(VX, torch.float32, self.device)
        VY = _dev(VY, torch.float32, self.device)
        FX = _dev(FX, torch.int32, self.device)
        FY = _dev(FY, torch.int32, self.device)
        sd = _dev(seeds, torch.int32, self.device)
        mx = dm_mesh(VX.shape[0], FX.shape[0], VX.data_ptr(), FX.data_ptr())
        my = dm_mesh(VY.shape[0], FY.shape[0], VY.data_ptr(), FY.data_ptr())
        cxy = torch.empty(VX.shape[0] * kcap, dtype=torch.int32, device=self.device)
        cyx = torch.empty(VY.shape[0] * kcap, dtype=torch.int32, device=self.device)
        K = C.c_int32(0)
        self._call("dm_ring_candidates", C.byref(mx), C.byref(my), _ptr(sd), sd.shape[0], int(rings), int(kcap),
                   _ptr(cxy), _ptr(cyx), C.byref(K))
        k = K.value
        return cxy[:VX.shape[0] * k].view(VX.shape[0], k), cyx[:VY.shape[0] * k].view(VY.shape[0], k)

    # -- generic 0-1 ILPs ------------------------------------------------
    def build_ilp(self, n_vars, row_ptr, cols, coefs, b):
        """min c^T x, A x = b, x in {0,1}^n with +-1 rows given as CSR
        (row_ptr [n_rows + 1], cols, coefs [nnz], b [n_rows])."""
        rp = _dev(row_ptr, torch.int32, self.device)
        cl = _dev(cols, torch.int32, self.device)
        cf = _dev(coefs, torch.int8, self.device)
        bb = _dev(b, torch.int32, self.device)
        info = dm_space_info()
        self._call("dm_build_ilp", int(n_vars), rp.shape[0] - 1, _ptr(rp), _ptr(cl) if cl.numel() else None,
                   _ptr(cf) if cf.numel() else None, _ptr(bb) if bb.numel() else None, C.byref(info))
        self.info = {n: getattr(info, n) for n, _ in dm_space_info._fields_}
        self.nvx = self.nvy = 0
        return self.info

    def set_costs(self, cost):
        """Costs of the current problem's variables (float64)."""
        c = _dev(cost, torch.float64, self.device)
        self._call("dm_set_costs", _ptr(c))

    def get_space(self, name):
        i = self.info
        shapes = {
            "pv": (torch.int32, (i["n_prod_tri"], 3)), "code": (torch.int32, (i["n_prod_tri"], 4)),
            "state": (torch.int8, (i["n_prod_tri"],)), "row_key": (torch.int64, (i["n_rows_full"],)),
            "row_ptr": (torch.int64, (i["n_rows_full"] + 1,)), "ent_var": (torch.int64, (i["nnz_full"],)),
            "ent_coef": (torch.int32, (i["nnz_full"],)), "row_b": (torch.int32, (i["n_rows_full"],)),
            "free_var": (torch.int64, (i["n_free"],)), "rrow_orig": (torch.int64, (i["n_rows"],)),
            "rrow_ptr": (torch.int64, (i["n_rows"] + 1,)), "rent_var": (torch.int64, (i["nnz"],)),
            "rent_coef": (torch.int32, (i["nnz"],)), "rrow_b": (torch.int32, (i["n_rows"],)),
            "edges_x": (torch.int32, (i["n_edges_x"], 2)), "edges_y": (torch.int32, (i["n_edges_y"], 2)),
            "cand": (torch.uint8, (self.nvx, self.nvy)),
        }
        dt, shp = shapes[name]
        out = torch.empty(shp, dtype=dt, device=self.device)
        self._call("dm_get_space", ARRAYS.index(name), _ptr(out))
        return out

    # -- A4 -------------------------------------------------------------
    def build_costs(self, DX, DY, prec="fp32"):
        DX = _dev(DX, torch.float32, self.device)
        DY = _dev(DY, torch.float32, self.device)
        cost = torch.empty(self.info["n_prod_tri"], dtype=torch.float32, device=self.device)
        self._call("dm_build_costs", _ptr(DX), _ptr(DY), DX.shape[1], PREC[prec], _ptr(cost))
        self._desc = (DX, DY)
        return cost

    # -- A5-A8 ----------------------------------------------------------
    def init_lambda(self, msg_prec="fp32"):
        dt = torch.float32 if msg_prec == "fp32" else torch.float64
        lam = torch.empty(self.info["nnz"], dtype=dt, device=self.device)
        self._call("dm_init_lambda", PREC[msg_prec], _ptr(lam))
        return lam

    def dual_solve(self, lam, iters, omega=0.5, temperature=0.0, msg_prec=None, trace=True):
        msg_prec = msg_prec or ("fp32" if lam.dtype == torch.float32 else "fp64")
        tr = torch.empty(max(iters, 1), dtype=torch.float64, device=self.device) if trace else None
        self._call("dm_dual_solve", int(iters), float(omega), float(temperature), PREC[msg_prec],
                   _ptr(lam), _ptr(tr) if trace else None)
        return lam, (tr[:iters] if trace else None)

    def lbfgs_solve(self, lam, iters, history=5, max_search=5, omega=0.5, eps=1e-8, step_up=1.1,
                    step_down=0.8, gamma0=0.1, resume=False):
        """Quasi-Newton powered MMA (Alg. 1), in place on lam.  Returns lam, the
        bound before every iteration and at the end (iters + 1 values), the
        step sizes and whether each quasi-Newton step was taken.  resume=True
        continues the previous call's history, step size and Delta_min."""
        msg_prec = "fp32" if lam.dtype == torch.float32 else "fp64"
        P = dm_lbfgs_params(int(history), int(max_search), float(omega), float(eps), float(step_up),
                            float(step_down), float(gamma0), int(bool(resume)))
        tr = torch.empty(iters + 1, dtype=torch.float64, device=self.device)
        gm = torch.empty(max(iters, 1), dtype=torch.float64, device=self.device)
        tk = torch.empty(max(iters, 1), dtype=torch.int32, device=self.device)
        self._call("dm_lbfgs_solve", int(iters), C.byref(P), PREC[msg_prec], _ptr(lam), _ptr(tr),
                   _ptr(gm), _ptr(tk))
        return lam, tr, gm[:iters], tk[:iters].bool()

    def subgradient(self, lam):
        """Per multiplier 1 where its row's minimiser sets the variable, and the bound."""
        msg_prec = "fp32" if lam.dtype == torch.float32 else "fp64"
        g = torch.empty(self.info["nnz"], dtype=torch.uint8, device=self.device)
        lb = C.c_double(0)
        self._call("dm_subgradient", PREC[msg_prec], _ptr(lam), _ptr(g), C.byref(lb))
        return g, lb.value

    def lbfgs_direction(self, S, Y, g):
        """Projected two-loop direction over the pairs S[k], Y[k] (oldest first)."""
        S = S.contiguous()
        msg_prec = "fp32" if S.dtype == torch.float32 else "fp64"
        Y = Y.to(torch.int8).contiguous()
        g = g.to(torch.uint8).contiguous()
        d = torch.empty(self.info["nnz"], dtype=S.dtype, device=self.device)
        h = S.shape[0] if S.dim() == 2 else 0
        self._call("dm_lbfgs_direction", PREC[msg_prec], int(h), _ptr(S) if h else None,
                   _ptr(Y) if h else None, _ptr(g), _ptr(d))
        return d

    # -- confident fixing (coarse-to-fine appendix) ----------------------
    def confident_fixing(self, lam, frac=0.9):
        """Per element -1 (free) or its fixed value, and the numbers of
        agreeing and of newly fixed variables."""
        msg_prec = "fp32" if lam.dtype == torch.float32 else "fp64"
        fix = torch.empty(self.info["n_prod_tri"], dtype=torch.int8, device=self.device)
        na, nf = C.c_int64(0), C.c_int64(0)
        self._call("dm_confident_fixing", PREC[msg_prec], _ptr(lam), float(frac), _ptr(fix), C.byref(na),
                   C.byref(nf))
        return fix, na.value, nf.value

    def fix_variables(self, fix=None):
        """Presolve from the fixings; the context then holds the residual
        problem (None restores the problem without fixings)."""
        f = None if fix is None else _dev(fix, torch.int8, self.device)
        info = dm_space_info()
        try:
            self._call("dm_fix_variables", _ptr(f) if f is not None else None, C.byref(info))
        finally:   # on infeasible fixings the problem without fixings is back
            self.info = {n: getattr(info, n) for n, _ in dm_space_info._fields_}
        return self.info

    def lower_bound(self, lam, temperature=0.0):
        msg_prec = "fp32" if lam.dtype == torch.float32 else "fp64"
        out = C.c_double(0)
        self._call("dm_lower_bound", _ptr(lam), float(temperature), PREC[msg_prec], C.byref(out))
        return out.value

    # -- A9, A10 --------------------------------------------------------
    def round_primal(self, lam, rounds=30, iters_per_round=25, delta0=0.0, gamma=1.5, seed=0, omega=0.5):
        msg_prec = "fp32" if lam.dtype == torch.float32 else "fp64"
        P = dm_round_params(rounds, iters_per_round, delta0, gamma, seed, omega, PREC[msg_prec])
        x = torch.empty(self.info["n_prod_tri"], dtype=torch.uint8, device=self.device)
        p, feas, r = C.c_double(0), C.c_int32(0), C.c_int32(0)
        self._call("dm_round_primal", C.byref(P), _ptr(lam), _ptr(x), C.byref(p), C.byref(feas), C.byref(r))
        return x, p.value, bool(feas.value), r.value

    def exact_search(self, base_fix=None, max_nodes=1000, dual_iters=100, omega=0.5, rel_tol=1e-9,
                     msg_prec="fp64", rounds=10, iters_per_round=25, delta0=0.0, gamma=1.5, seed=0):
        """Depth-first branch and bound on the problem with the fixings
        base_fix (None: none); returns (x, primal objective, bound, nodes,
        status) with status "optimal", "infeasible" or "limit".  The
        problem with base_fix is in place afterwards."""
        f = None if base_fix is None else _dev(base_fix, torch.int8, self.device)
        R = dm_round_params(rounds, iters_per_round, delta0, gamma, seed, omega, PREC[msg_prec])
        P = dm_search_params(max_nodes, dual_iters, omega, rel_tol, R)
        x = torch.empty(self.info["n_prod_tri"], dtype=torch.uint8, device=self.device)
        p, b, n, st = C.c_double(0), C.c_double(0), C.c_int32(0), C.c_int32(0)
        info = dm_space_info()
        try:
            self._call("dm_exact_search", C.byref(P), _ptr(f) if f is not None else None, _ptr(x), C.byref(p),
                       C.byref(b), C.byref(n), C.byref(st), C.byref(info))
        finally:   # the problem with base_fix is in place afterwards
            self.info = {k: getattr(info, k) for k, _ in dm_space_info._fields_}
        return x, p.value, b.value, n.value, SEARCH_STATUS[st.value]

    def repair_primal(self, x, max_hops=8, max_nodes=200, dual_iters=100, omega=0.5, rel_tol=1e-9,
                      msg_prec="fp32", rounds=10, iters_per_round=25, delta0=0.0, gamma=1.5, seed=0):
        """Local exact repair of x around the rows it violates; returns (x,
        primal objective, feasible, steps of the last neighbourhood, its free
        elements).  x is repaired in place when it is a uint8 device tensor."""
        x = _dev(x, torch.uint8, self.device)
        R = dm_round_params(rounds, iters_per_round, delta0, gamma, seed, omega, PREC[msg_prec])
        P = dm_search_params(max_nodes, dual_iters, omega, rel_tol, R)
        p, feas, hops, nfree = C.c_double(0), C.c_int32(0), C.c_int32(0), C.c_int64(0)
        self._call("dm_repair_primal", C.byref(P), int(max_hops), _ptr(x), C.byref(p), C.byref(feas),
                   C.byref(hops), C.byref(nfree))
        return x, p.value, bool(feas.value), hops.value, nfree.value

    def check_primal(self, x):
        x = _dev(x, torch.uint8, self.device)
        v = C.c_int64(0)
        self._call("dm_check_primal", _ptr(x), C.byref(v))
        return v.value

    # -- A11 ------------------------------------------------------------
    def smoothed_backward(self, lam, temperature, DX, DY, grad_out=1.0):
        msg_prec = "fp32" if lam.dtype == torch.float32 else "fp64"
        DX = _dev(DX, torch.float32, self.device)
        DY = _dev(DY, torch.float32, self.device)
        gc = torch.empty(self.info["n_prod_tri"], dtype=torch.float32, device=self.device)
        gX = torch.empty_like(DX)
        gY = torch.empty_like(DY)
        v = C.c_double(0)
        self._call("dm_smoothed_backward", _ptr(lam), float(temperature), PREC[msg_prec], float(grad_out),
                   _ptr(DX), _ptr(DY), DX.shape[1], _ptr(gc), _ptr(gX), _ptr(gY), C.byref(v))
        return gc, gX, gY, v.value

    def timing(self, enable: bool):
        self._call("dm_timing_enable", int(enable))

    def timing_read(self):
        n, ms = C.c_int64(0), C.c_double(0)
        self._call("dm_timing_read", C.byref(n), C.byref(ms))
        return n.value, ms.value

    def mixed_areas(self, V, F):
        V = _dev(V, torch.float32, self.device)
        F = _dev(F, torch.int32, self.device)
        m = dm_mesh(V.shape[0], F.shape[0], V.data_ptr(), F.data_ptr())
        out = torch.empty(V.shape[0], dtype=torch.float64, device=self.device)
        self._call("dm_mixed_areas", C.byref(m), _ptr(out))
        return out


# Module-level names matching the C ABI -------------------------------------
def build_product_space(ctx: Context, *a, **k):
    return ctx.build_product_space(*a, **k)


def build_costs(ctx: Context, *a, **k):
    return ctx.build_costs(*a, **k)


def dual_solve(ctx: Context, *a, **k):
    return ctx.dual_solve(*a, **k)


def lbfgs_solve(ctx: Context, *a, **k):
    return ctx.lbfgs_solve(*a, **k)


def round_primal(ctx: Context, *a, **k):
    return ctx.round_primal(*a, **k)


def lower_bound(ctx: Context, *a, **k):
    return ctx.lower_bound(*a, **k)


class SmoothedBound(torch.autograd.Function):
    """L_T of the smoothed dual as a function of the descriptors.

    forward(DX, DY, ctx_obj, iters, T, omega) builds the costs from DX, DY
    (FP32), runs ``iters`` smoothed Jacobi iterations from c/|J_i| and returns
    L_T as a 0-d float64 tensor; backward calls dm_smoothed_backward with the
    final multipliers held as c/|J_i| + phi, phi fixed.  The backward pass
    reads the context's costs and problem, so it refuses to run when the
    context changed after the forward pass (Context.generation)."""

    @staticmethod
    def forward(fctx, DX, DY, dm: Context, iters: int, T: float, omega: float = 0.5, prec: str = "fp32"):
        dm.build_costs(DX.detach(), DY.detach(), prec)
        lam = dm.init_lambda("fp32")
        dm.dual_solve(lam, iters, omega, T, trace=False)
        val = dm.lower_bound(lam, T)
        fctx.dm, fctx.T, fctx.generation = dm, T, dm.generation
        fctx.save_for_backward(DX, DY, lam)
        return torch.tensor(val, dtype=torch.float64, device=DX.device)

    @staticmethod
    def backward(fctx, g):
        DX, DY, lam = fctx.saved_tensors
        if fctx.dm.generation != fctx.generation:
            raise RuntimeError("SmoothedBound.backward: the context's problem or costs changed after this "
                               "forward pass (another forward, build or fixing on the same Context); use one "
                               "Context per smoothed bound in a graph")
        _, gX, gY, _ = fctx.dm.smoothed_backward(lam, fctx.T, DX.detach(), DY.detach(), float(g))
        return gX.to(DX.dtype), gY.to(DY.dtype), None, None, None, None, None
