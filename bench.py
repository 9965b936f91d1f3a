"""Benchmark of the dual-solver hot path on one MI355X.

One step is one pass of the whole path over one synthetic mesh pair that is
already resident in HBM: candidates (A2), product space + presolve (A1, A3),
costs (A4), initial multipliers (A5), the Jacobi dual iterations with the FP64
bound trace (A6-A8), rounding to an exactly checked primal and the gap
(A9, A10).  The default workload is the 500-face plain-FP32 pair (64-d
descriptors, K = 16, 1000 iterations).  ``value`` is dual iterations per
second of whole-step wall time.  Gaps use a certified bound: the FP64 dual
objective at the multipliers re-projected onto dual feasibility.

Also reported (same JSON line): the dominant kernel's roofline (the sweep
kernel: algorithmic bytes per launch / its average launch duration from HIP
events around each launch), the sweep at the other pairs (the smoothed
sweep against the VALU issue peak), time-to-1%-gap of
the plain FP32, mixed (BF16 costs) and differentiable (smoothed T = 0.1 with
the backward pass) forms on the same pairs, the largest pair's full pipeline
timed end to end, a plain copy's bandwidth against the HBM peak, and the
FP64 oracle on the host (seconds per iteration and time to a 1 % gap).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue peak: a wave64 VALU instruction holds its SIMD's issue port for
# 4 cycles, so 256 CUs x 4 SIMDs x 2.4 GHz / 4 = 614.4 G wave-instructions/s
VALU_ISSUE_PEAK_G = 256 * 4 * 2.4 / 4
BYTES_PER_NNZ = 12     # read lambda 4 + write lambda 4 + one int32 routing word 4
BYTES_PER_ROW = 4      # row pointer


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--k", type=int, default=None, help="candidates per vertex (default: the config's K)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gap", action="store_true")
    ap.add_argument("--no-pairs", action="store_true", help="skip the per-pair sweep rooflines")
    ap.add_argument("--no-search", action="store_true", help="skip the exact-search timing")
    ap.add_argument("--cpu-sample-iters", type=int, default=80)
    ap.add_argument("--gap-seeds", default="0,1,2", help="seeds of the time-to-1%%-gap runs (median reported)")
    return ap.parse_args()


class Workload:
    def __init__(self, cfg, seed, iters=None, **over):
        import torch

        import paper_2310_08230_amd as dm
        from synth import CONFIGS, make_pair
        self.dm = dm
        self.pair = make_pair(cfg, seed, **over)
        self.spec = self.pair.spec
        self.cfg = cfg
        self.iters = iters or self.spec.iters
        dev = torch.device("cuda", 0)
        p = self.pair
        self.VX = torch.from_numpy(p.VX).to(dev)
        self.FX = torch.from_numpy(p.FX).to(dev)
        self.VY = torch.from_numpy(p.VY).to(dev)
        self.FY = torch.from_numpy(p.FY).to(dev)
        self.DX = torch.from_numpy(p.DX).to(dev)
        self.DY = torch.from_numpy(p.DY).to(dev)
        self.ctx = dm.Context(0)
        self.msg = self.spec.msg_prec
        self.cost = self.spec.cost_prec
        self.knn_prec = "bf16" if self.cost == "bf16" else "fp32"

    def step(self, with_round=True):
        c = self.ctx
        cxy, cyx = c.knn_candidates(self.DX, self.DY, self.spec.k, self.knn_prec)
        c.build_product_space(self.VX, self.FX, self.VY, self.FY, cxy, cyx)
        c.build_costs(self.DX, self.DY, self.cost)
        lam = c.init_lambda(self.msg)
        lam, tr = c.dual_solve(lam, self.iters, self.spec.omega, self.spec.temperature)
        out = {"lam": lam, "trace": tr}
        if with_round:
            x, pobj, feas, rounds = c.round_primal(lam, seed=0)
            # certified bound: the FP64 dual objective at the multipliers
            # re-projected onto dual feasibility with the FP64 costs
            dmax = c.lower_bound(lam.double())
            out.update(pobj=pobj, feasible=feas, rounds=rounds, bound=dmax,
                       gap=(pobj - dmax) / pobj if pobj else 0.0)
        return out


def c2f_run(seed=0, levels=(500, 1000, 2000, 4000), K0=32, qn_iters=60, rings=2):
    """Coarse-to-fine pipeline (Sec. 5.2) on the pose of the 1000-face pair
    at 500 -> 1000 -> 2000 -> 4000 faces: the coarsest level takes K0 nearest
    candidates, every finer one the ring candidates of the previous level's
    matching; each level runs qn_iters quasi-Newton iterations and one
    rounding, followed by the local repair if it leaves rows violated.
    Wall time per level (candidates, build, costs, solve, rounding), sizes
    and gap."""
    import numpy as np
    import torch

    import paper_2310_08230_amd as dm
    from synth import make_pair
    ctx = dm.Context(0)
    out, prev, total = [], None, 0.0
    for F in levels:
        p = make_pair(3, seed, faces_x=F, faces_y=F)
        DX, DY = torch.from_numpy(p.DX).cuda(), torch.from_numpy(p.DY).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if prev is None:
            cxy, cyx = ctx.knn_candidates(DX, DY, K0, "fp32")
        else:
            pp, xp = prev
            pairs = ctx.matched_pairs(xp)
            mx = ctx.nearest_vertices(pp.RX.astype(np.float32), p.RX.astype(np.float32))
            my = ctx.nearest_vertices(pp.RY.astype(np.float32), p.RY.astype(np.float32))
            seeds = torch.stack([mx[pairs[:, 0].long()], my[pairs[:, 1].long()]], 1)
            cxy, cyx = ctx.ring_candidates(p.VX, p.FX, p.VY, p.FY, seeds, rings=rings)
        ctx.build_product_space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
        ctx.build_costs(DX, DY, "fp32")
        lam, tr = ctx.lbfgs_solve(ctx.init_lambda("fp32"), qn_iters)[:2]
        x, pobj, feas, _ = ctx.round_primal(lam)
        if not feas:   # local exact repair around the violated rows
            x, pobj, feas, _, _ = ctx.repair_primal(x, max_hops=8)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        total += dt
        d = float(tr.max())
        out.append({"faces": F, "K": int(cxy.shape[1]), "n_cand": ctx.info["n_cand"],
                    "n_prod_tri": ctx.info["n_prod_tri"], "seconds": round(dt, 4), "feasible": feas,
                    "gap": (pobj - d) / pobj if feas and pobj else None})
        prev = (p, x)
    return {"levels": out, "total_seconds": round(total, 4)}


def generic_ilp_run(n=200, n_side=4000, seed=0, iters=500, search_n=20, search_side=60):
    """Generic 0-1 ILP path: an n x n assignment with n_side random +-1 side
    rows (planted feasible), FP32 Jacobi iterations per second and the bound
    reached; then the exact search to a proved optimum on a 20 x 20 instance
    with 60 side rows."""
    import torch

    import paper_2310_08230_amd as dm
    from synth import generic_ilp
    ctx = dm.Context(0)
    nv, rp, cols, coefs, b, c = generic_ilp(n, n_side, seed)
    info = ctx.build_ilp(nv, rp, cols, coefs, b)
    ctx.set_costs(torch.from_numpy(c))
    lam = ctx.init_lambda("fp32")
    ctx.dual_solve(lam, 20, 0.5, trace=False)   # untimed: loads the kernels
    lam = ctx.init_lambda("fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam, tr = ctx.dual_solve(lam, iters, 0.5)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"instance": f"{n}x{n} assignment + {n_side} +-1 side rows, seed {seed}", "n_vars": nv,
           "rows": info["n_rows"], "nnz": info["nnz"], "jacobi_iters_per_s": round(iters / dt, 1),
           "bound": float(tr.max())}
    nv, rp, cols, coefs, b, c = generic_ilp(search_n, search_side, seed + 1)
    ctx.build_ilp(nv, rp, cols, coefs, b)
    ctx.set_costs(torch.from_numpy(c))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, pobj, bound, nodes, status = ctx.exact_search(max_nodes=3000, dual_iters=60)
    torch.cuda.synchronize()
    out["exact_search"] = {"instance": f"{search_n}x{search_n} assignment + {search_side} side rows",
                           "status": status, "optimum": pobj, "nodes": nodes,
                           "seconds": round(time.perf_counter() - t0, 4)}
    return out


def exact_search_run(seed=0, max_nodes=3000, dual_iters=60):
    """Branch and bound on a pair whose LP relaxation leaves an integrality
    gap (the 80-face pair, descriptor noise 1.0, K = 16): wall time to a
    proved optimum, nodes, and the root bound for the size of the gap."""
    import torch
    w = Workload(1, seed, desc_noise=1.0, k=16)
    c = w.ctx
    cxy, cyx = c.knn_candidates(w.DX, w.DY, 16, "fp32")
    info = c.build_product_space(w.VX, w.FX, w.VY, w.FY, cxy, cyx)
    c.build_costs(w.DX, w.DY, "fp64")
    root = c.lower_bound(c.dual_solve(c.init_lambda("fp64"), dual_iters, 0.5)[0])
    c.exact_search(max_nodes=2, dual_iters=dual_iters)   # untimed: loads the kernels
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, pobj, bound, nodes, status = c.exact_search(max_nodes=max_nodes, dual_iters=dual_iters)
    torch.cuda.synchronize()
    return {"instance": "80-face pair, descriptor noise 1.0, K=16, seed %d" % seed, "free": info["n_free"],
            "status": status, "optimum": pobj, "root_bound": root, "nodes": nodes,
            "seconds": round(time.perf_counter() - t0, 4), "violations": c.check_primal(x)}


def sweep_roofline(cfg, seed, iters=200, temperature=0.0, **over):
    """Sweep kernel of one pair, timed per launch by the kernel's own events
    over ``iters`` Jacobi iterations: microseconds per launch and algorithmic
    GB/s (12 B per nonzero + 4 B per row) against the HBM peak.  With a
    temperature the smoothed sweep is timed instead; its partial-sum
    recursion is bound by vector-instruction issue, so on the 1000-face pair
    at T = 0.1 (seed 0) its instructions per launch, from the committed SQ
    counter summary, are set against the VALU issue peak.
    ``over`` changes the pair's spec (e.g. ``k=96``).  The working set is the
    two record buffers, the routing words and the row pointers."""
    w = Workload(cfg, seed, **over)
    c = w.ctx
    cxy, cyx = c.knn_candidates(w.DX, w.DY, w.spec.k, w.knn_prec)
    info = c.build_product_space(w.VX, w.FX, w.VY, w.FY, cxy, cyx)
    c.build_costs(w.DX, w.DY, w.cost)
    lam = c.init_lambda(w.msg)
    c.dual_solve(lam, 20, w.spec.omega, temperature, trace=False)
    c.timing(True)
    c.dual_solve(lam, iters, w.spec.omega, temperature)
    n, ms = c.timing_read()
    c.timing(False)
    us = ms * 1e3 / max(n, 1)
    if temperature > 0:
        out = {"pair": f"{w.spec.faces_x}/{w.spec.faces_y} faces", "temperature": temperature,
               "nnz": info["nnz"], "rows": info["n_rows"], "avg_launch_us": round(us, 2), "bound": "alu"}
        valu = _smoothed_valu() if (cfg, seed, temperature, not over) == (4, 0, 0.1, True) else None
        if valu:
            # instructions per launch from the committed SQ counter summary,
            # over this run's launch time, against the VALU issue peak
            g = valu["valu_insts_per_launch"] / (us * 1e-6) / 1e9
            out.update(achieved=round(g, 1), peak=VALU_ISSUE_PEAK_G, unit="G VALU wave-instructions/s",
                       frac=round(g / VALU_ISSUE_PEAK_G, 4), valu_insts_per_launch=valu["valu_insts_per_launch"],
                       trans_insts_per_launch=valu["trans_insts_per_launch"])
        return out
    nbytes = BYTES_PER_NNZ * info["nnz"] + BYTES_PER_ROW * info["n_rows"]
    gbs = nbytes / (us * 1e-6) / 1e9
    rec_bytes = 4 if w.msg == "fp32" else 8
    working_set = 2 * 8 * rec_bytes * info["n_free"] + 4 * info["nnz"] + 4 * (info["n_rows"] + 1)
    out = {"pair": f"{w.spec.faces_x}/{w.spec.faces_y} faces, K={w.spec.k}", "nnz": info["nnz"],
           "rows": info["n_rows"], "working_set_bytes": working_set,
           "avg_launch_us": round(us, 2), "bytes_per_launch": nbytes, "achieved_GBps": round(gbs, 1),
           "frac": round(gbs / HBM_PEAK_GBS, 4)}
    prof = TRAFFIC_PROFILES.get((cfg, seed, tuple(sorted(over.items()))))
    traffic = _traffic(prof) if prof and w.msg == "fp32" else None
    if traffic:
        # bytes through the L2s per launch (counters, copy-calibrated) over
        # this run's launch time, and their ratio to the algorithmic bytes
        out.update(traffic=traffic, traffic_GBps=round(traffic / (us * 1e-6) / 1e9, 1),
                   traffic_over_algorithmic=round(traffic / nbytes, 2))
    return out


FORMS = {
    # name: (distance / cost precision, smoothed start with the backward pass)
    "plain_fp32": ("fp32", False),
    "mixed_bf16": ("bf16", False),
    "diff_t0.1": ("bf16", True),
}


def time_to_gap(cfg, seed, form="plain_fp32", check_every=10, max_iters=3000, smooth_iters=50, solver="jacobi",
                qn_check_every=10, qn_max_iters=400, rounds=10, repair=True, **over):
    """Wall time from the first dual iteration until a rounding reaches a
    primal-dual gap <= 1e-2 (roundings and bound checks included; build
    excluded), for one of the three forms on one pair:

      plain_fp32  FP32 distances and costs, FP32 messages;
      mixed_bf16  BF16 MFMA distances (FP32 accumulation), FP32 messages;
      diff_t0.1   as mixed, preceded by ``smooth_iters`` smoothed iterations
                  at T = 0.1 and one backward pass to the descriptors (their
                  time included), hard iterations from the smoothed
                  multipliers.

    Every ``check_every`` Jacobi iterations (solver "jacobi") or
    ``qn_check_every`` quasi-Newton iterations (solver "lbfgs", the search
    state resumed between checks) the multipliers are rounded with ``rounds``
    perturbation rounds; with ``repair``, a rounding that leaves rows violated
    is followed by the local exact repair (dm_repair_primal, at most 8
    steps), whose time is included.  The bound is certified: the FP64 dual objective at
    the FP32 multipliers re-projected onto dual feasibility with the FP64
    costs (Eq. (D) holds at any feasible multipliers), maximised over the
    checks; d_max and p are both in FP64."""
    import torch
    prec, smoothed = FORMS[form]
    w = Workload(cfg, seed, **over)
    c = w.ctx
    cxy, cyx = c.knn_candidates(w.DX, w.DY, w.spec.k, "bf16" if prec == "bf16" else "fp32")
    c.build_product_space(w.VX, w.FX, w.VY, w.FY, cxy, cyx)
    c.build_costs(w.DX, w.DY, prec)
    lam = c.init_lambda("fp32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = {"form": form, "solver": solver}
    if smoothed:
        T = 0.1
        lam, _ = c.dual_solve(lam, smooth_iters, w.spec.omega, T, trace=False)
        _, gX, gY, LT = c.smoothed_backward(lam, T, w.DX, w.DY)
        torch.cuda.synchronize()
        out.update(smooth_seconds=round(time.perf_counter() - t0, 6), smooth_iters=smooth_iters, L_T=LT)
    dmax = -float("inf")
    it = 0
    best = None
    repaired = 0
    cap = qn_max_iters if solver == "lbfgs" else max_iters
    while it < cap:
        if solver == "lbfgs":
            lam, _, _, _ = c.lbfgs_solve(lam, qn_check_every, omega=w.spec.omega, resume=it > 0)
            it += qn_check_every
        else:
            lam, _ = c.dual_solve(lam, check_every, w.spec.omega, 0.0, trace=False)
            it += check_every
        dmax = max(dmax, c.lower_bound(lam.double()))
        x, pobj, feas, _ = c.round_primal(lam, rounds=rounds, seed=0)
        if not feas and repair:
            _, pobj, feas, _, _ = c.repair_primal(x, max_hops=8)
            repaired += bool(feas)
        if feas:
            g = (pobj - dmax) / pobj
            best = g if best is None else min(best, g)
            if g <= 1e-2:
                torch.cuda.synchronize()
                out.update(seconds=round(time.perf_counter() - t0, 6), iters=it, gap=g, bound=dmax, primal=pobj,
                           repaired_checks=repaired)
                return out
    torch.cuda.synchronize()
    out.update(seconds=None, iters=it, gap=None, best_gap=best, bound=dmax, repaired_checks=repaired,
               note="1% gap not reached within the iteration cap")
    return out


def pipeline_run(cfg=5, seed=0, iters=None, T=0.1, rounds=10):
    """The full pipeline on one pair, timed end to end with a synchronisation
    after each stage: BF16 candidates, product space + presolve, BF16 costs,
    FP32 Jacobi iterations with the FP64 bound trace, the certified FP64
    bound, rounding (at most ``rounds`` perturbation rounds, as at every
    time-to-gap check), and the smoothed backward pass (one soft sweep at the
    final multipliers and the chain to both descriptor sets).  A rounding
    that leaves rows violated is followed by the local exact repair."""
    import torch
    w = Workload(cfg, seed, iters)
    c = w.ctx
    stages = {}

    def mark(name, t):
        torch.cuda.synchronize()
        now = time.perf_counter()
        stages[name] = round(now - t, 6)
        return now

    torch.cuda.synchronize()
    t0 = t = time.perf_counter()
    cxy, cyx = c.knn_candidates(w.DX, w.DY, w.spec.k, "bf16")
    t = mark("candidates_bf16", t)
    info = c.build_product_space(w.VX, w.FX, w.VY, w.FY, cxy, cyx)
    t = mark("product_space_presolve", t)
    c.build_costs(w.DX, w.DY, "bf16")
    t = mark("costs_bf16", t)
    lam, tr = c.dual_solve(c.init_lambda("fp32"), w.iters, w.spec.omega)
    t = mark("jacobi_fp32", t)
    lb = c.lower_bound(lam.double())
    t = mark("certified_bound_fp64", t)
    x, pobj, feas, _ = c.round_primal(lam, rounds=rounds, seed=0)
    t = mark("rounding", t)
    rounded_feasible = feas
    if not feas:   # local exact repair around the violated rows
        x, pobj, feas, hops, nfree = c.repair_primal(x, max_hops=8)
        t = mark("repair", t)
    _, gX, gY, LT = c.smoothed_backward(lam, T, w.DX, w.DY)
    t = mark("smoothed_backward", t)
    return {"pair": f"{w.spec.faces_x}/{w.spec.faces_y} faces, K={w.spec.k}, D={w.spec.dim}, seed {seed}",
            "nnz": info["nnz"], "jacobi_iters": w.iters, "seconds": round(t - t0, 6), "stages": stages,
            "bound_certified": lb, "bound_trace_max": float(tr.max()), "primal": pobj, "feasible": feas,
            "rounding_feasible": rounded_feasible,
            "gap": (pobj - lb) / pobj if feas and pobj else None, "L_T": LT,
            "grad_finite": bool(torch.isfinite(gX).all() and torch.isfinite(gY).all())}


def copy_bandwidth(nbytes=1 << 31, reps=10):
    """Achieved bandwidth of a plain device-to-device copy (the runtime's copy
    kernel) of ``nbytes`` bytes: read + written bytes over the time of
    ``reps`` copies between HIP events; the reference for the 8 TB/s HBM
    peak."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3
    gbs = 2 * nbytes * reps / s / 1e9
    return {"bytes": nbytes, "reps": reps, "achieved_GBps": round(gbs, 1), "peak_GBps": HBM_PEAK_GBS,
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


# committed FETCH/WRITE summaries per sweep workload: (config, seed, spec changes) -> file
TRAFFIC_PROFILES = {(2, 0, ()): "sweep_plain_fp32_500_hbm_traffic.json",
                    (5, 0, ()): "sweep_largest_2000x3000_hbm_traffic.json",
                    (5, 0, (("k", 144),)): "sweep_k144_hbm_point_hbm_traffic.json"}


def _traffic(name="sweep_plain_fp32_500_hbm_traffic.json"):
    """HBM bytes per sweep launch from a committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by its reading on a
    plain copy kernel), used only while the sweep source is the one that was
    profiled; otherwise None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    src = os.path.join(ROOT, "paper_2310_08230_amd", "csrc", "dual.hip")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("dual_hip_sha256") != h:
        return None
    return rec.get("bytes_per_launch")


def _smoothed_valu():
    """VALU and transcendental wave-instructions per launch of the smoothed
    sweep on the 1000-face pair at T = 0.1, from the committed rocprofv3 SQ
    counter summary, used only while the sweep source is the one that was
    profiled; otherwise None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "sweep_smoothed_t0.1_1000_valu.json")
    src = os.path.join(ROOT, "paper_2310_08230_amd", "csrc", "dual.hip")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("dual_hip_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return rec


def summarize_valu(counter_csv, out_json, workload, command=""):
    """Median SQ_INSTS_VALU and SQ_INSTS_VALU_TRANS_F32 per dispatch of the
    smoothed FP32 update sweep (k_sweep<float, true, 0, ...>) from a
    rocprofv3 --pmc collection; writes the summary the smoothed entry's
    roofline reads."""
    import csv
    import hashlib
    import statistics
    rows = [r for r in csv.DictReader(open(counter_csv)) if "k_sweep<float, true, 0" in r["Kernel_Name"]]

    def med(counter):
        v = [float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == counter]
        return statistics.median(v), len(v)

    valu, n = med("SQ_INSTS_VALU")
    trans, _ = med("SQ_INSTS_VALU_TRANS_F32")
    waves, _ = med("SQ_WAVES")
    src = os.path.join(ROOT, "paper_2310_08230_amd", "csrc", "dual.hip")
    rec = {"kernel": sorted({r["Kernel_Name"].strip() for r in rows})[0] if rows else "", "workload": workload,
           "dispatches": n, "waves_per_launch": waves, "valu_insts_per_launch": valu,
           "trans_insts_per_launch": trans, "valu_issue_peak_G_per_s": VALU_ISSUE_PEAK_G, "commands": command,
           "dual_hip_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest()}
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def cpu_baseline(cfg, seed, iters, runs=3, gap_cap_s=3600.0, check_every=10, rounds=10):
    """The FP64 oracle (single thread, its build excluded) on the same pair:
    seconds per Jacobi iteration as the median of ``runs`` runs of ``iters``
    iterations, reported as iterations per second; and its time to a 1 %
    gap with the GPU's schedule (rounding with ``rounds`` rounds every
    ``check_every`` iterations), capped at ``gap_cap_s`` seconds."""
    import statistics

    from oracle import oracle as O
    from synth import make_pair
    p = make_pair(cfg, seed)
    cxy, cyx = O.knn(p.DX, p.DY, p.spec.k)
    S = O.Space(p.VX, p.FX, p.VY, p.FY, cxy, cyx)
    S.costs(p.DX, p.DY)
    per_it = []
    for _ in range(runs):
        t0 = time.perf_counter()
        S.dual_solve(iters)
        per_it.append((time.perf_counter() - t0) / iters)
    s_it = statistics.median(per_it)
    # time to a 1 % gap
    t0 = time.perf_counter()
    lam, dmax, it, gap = None, -float("inf"), 0, None
    while time.perf_counter() - t0 < gap_cap_s:
        lam, tr = S.dual_solve(check_every, lam=lam)
        it += check_every
        dmax = max(dmax, float(tr.max()))
        _, pobj, feas, _ = S.round(lam, R=rounds)
        if feas and (pobj - dmax) / pobj <= 1e-2:
            gap = (pobj - dmax) / pobj
            break
    ttg = time.perf_counter() - t0
    return {"value": round(1.0 / s_it, 3), "unit": "dual iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 oracle on the same pair (config {cfg}, seed {seed}), build excluded: median of "
                      f"{runs} runs of {iters} Jacobi iterations, {s_it:.4f} s per iteration "
                      f"({', '.join(f'{x:.4f}' for x in per_it)})",
            "seconds_per_iteration": round(s_it, 6),
            "time_to_1pct_gap": {"seconds": round(ttg, 3) if gap is not None else None, "iters": it, "gap": gap,
                                 "schedule": f"rounding ({rounds} rounds) every {check_every} iterations",
                                 "cap_seconds": gap_cap_s},
            "host": host_cpu()}


def host_cpu():
    """CPU model of this host and the cores this process may run on (the
    oracle itself is single-threaded, built -O2 -ffp-contract=off)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "cores_available": len(os.sched_getaffinity(0))}


def copy_calibration(nbytes, reps=5):
    """A plain device-to-device copy of ``nbytes`` bytes (the runtime's copy
    kernel), the reference that scales the FETCH_SIZE / WRITE_SIZE counters to
    bytes."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {nbytes} bytes {reps} times", flush=True)


def summarize_counters(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, out_json, copy_bytes,
                       command="", workload="plain_fp32_500 (config 2, seed 0)"):
    """Turn rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE collections (KiB per
    dispatch) of the sweep kernel and of a plain copy of ``copy_bytes`` bytes
    into HBM bytes per sweep launch; writes the summary JSON used by the
    roofline's ``traffic`` field."""
    import csv
    import hashlib
    import statistics

    names = set()

    def per_kernel(path, counter, name_has):
        rows = [r for r in csv.DictReader(open(path))
                if r["Counter_Name"] == counter and name_has in r["Kernel_Name"]]
        if name_has.startswith("k_sweep"):
            names.update(r["Kernel_Name"].strip() for r in rows)
        return statistics.median(float(r["Counter_Value"]) for r in rows), len(rows)

    cf, _ = per_kernel(copy_fetch_csv, "FETCH_SIZE", "copyBuffer")
    cw, _ = per_kernel(copy_write_csv, "WRITE_SIZE", "copyBuffer")
    # the hard FP32 update sweep, with or without row tiles: k_sweep<float, false, 0, ...>
    f, nf = per_kernel(fetch_csv, "FETCH_SIZE", "k_sweep<float, false, 0")
    wv, nw = per_kernel(write_csv, "WRITE_SIZE", "k_sweep<float, false, 0")
    kib = copy_bytes / 1024.0
    ffac, wfac = kib / cf, kib / cw
    fetch_b = f * ffac * 1024.0
    write_b = wv * wfac * 1024.0
    src = os.path.join(ROOT, "paper_2310_08230_amd", "csrc", "dual.hip")
    rec = {"kernel": " / ".join(sorted(names)), "workload": workload,
           "fetch_kib_median": f, "write_kib_median": wv, "dispatches": [nf, nw],
           "copy_calibration": {"bytes": copy_bytes, "fetch_kib": cf, "write_kib": cw,
                                "fetch_factor": ffac, "write_factor": wfac},
           "bytes_per_launch": int(fetch_b + write_b), "fetch_bytes": int(fetch_b), "write_bytes": int(write_b),
           "commands": command,
           "dual_hip_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest()}
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def summarize_trace(stats_csv, out_txt, command):
    """Short text summary of a rocprofv3 --kernel-trace --stats run: the
    command that made it and the kernels by total time."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"command: {command}", "",
             f"{'kernel':70s} {'calls':>7s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'total_ms':>9s} {'pct':>6s}"]
    for r in rows[:20]:
        name = r["Name"].replace("(anonymous namespace)::", "")
        name = name.split("(")[0] if not name.startswith("void rocprim") else "rocprim (sort/scan)"
        lines.append(f"{name[:70]:70s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:9.2f} "
                     f"{float(r['MinNs']) / 1e3:9.2f} {float(r['MaxNs']) / 1e3:9.2f} "
                     f"{float(r['TotalDurationNs']) / 1e6:9.2f} {float(r['Percentage']):6.1f}")
    open(out_txt, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-counters":
        # fetch write copy_fetch copy_write out_json copy_bytes workload command...
        summarize_counters(*sys.argv[2:7], int(sys.argv[7]), " ".join(sys.argv[9:]), sys.argv[8])
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--copy-calibration":
        copy_calibration(int(sys.argv[2]))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-valu":
        # counter_csv out_json workload command...
        summarize_valu(sys.argv[2], sys.argv[3], sys.argv[4], " ".join(sys.argv[5:]))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-trace":
        summarize_trace(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
        return
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported "
              "(the solver runs on one GPU and has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    w = Workload(a.config, a.seed, a.iters, **({"k": a.k} if a.k else {}))
    log(f"[bench] config {a.config} ({w.spec.name}) iters={w.iters} warmup={a.warmup} steps={a.steps}")
    for i in range(a.warmup):
        r = w.step()
        log(f"[bench] warmup {i}: gap={r['gap']:.2e} feasible={r['feasible']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        r = w.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / a.steps * 1e3
    value = a.steps * w.iters / dt
    info = w.ctx.info
    log(f"[bench] timed: {ms_per_step:.2f} ms/step, {value:.0f} dual it/s, gap={r['gap']:.2e}")

    # dominant kernel: the sweep, timed per launch with HIP events on its stream
    c = w.ctx
    lam = c.init_lambda(w.msg)
    c.dual_solve(lam, 20, w.spec.omega, w.spec.temperature, trace=False)
    # the solve alone (bound trace on, no per-launch events): iterations/s
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c.dual_solve(lam, w.iters, w.spec.omega, w.spec.temperature)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t1
    # the same solve with start/stop events around every sweep launch
    c.timing(True)
    c.dual_solve(lam, w.iters, w.spec.omega, w.spec.temperature)
    torch.cuda.synchronize()
    c.timing(False)
    n_launch, tot_ms = c.timing_read()
    avg_s = tot_ms / 1e3 / max(n_launch, 1)
    bytes_per_launch = BYTES_PER_NNZ * info["nnz"] + BYTES_PER_ROW * info["n_rows"]
    achieved = bytes_per_launch / avg_s / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            # the committed counters describe the seed-0 pair at its own K
            "traffic": _traffic() if (a.config, a.seed, a.k) == (2, 0, None) and w.iters > 0 else None,
            "kernel": "k_sweep<float,false,MODE_UPDATE>", "avg_launch_us": round(avg_s * 1e6, 3),
            "bytes_per_launch": bytes_per_launch}
    log(f"[bench] sweep kernel: {n_launch} launches, avg {avg_s * 1e6:.2f} us, {achieved:.0f} GB/s algorithmic")

    out = {"metric": "dual iterations/sec + time-to-1% gap, plain FP32 vs mixed/diff form, 1 MI355X",
           "value": round(value, 2), "unit": "dual iterations/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32" if w.msg == "fp32" else "f64",
           "data": "synthetic",
           "config": {"workload": f"{w.spec.name}: {w.spec.faces_x}-face vs {w.spec.faces_y}-face icosphere "
                                  f"pair ({w.spec.notes}), {w.spec.dim}-d descriptors, K={w.spec.k}, "
                                  f"{w.iters} Jacobi iterations, rounding",
                      "config_id": a.config, "seed": a.seed, "n_prod_tri": info["n_prod_tri"],
                      "nnz": info["nnz"], "n_rows": info["n_rows"]},
           "roofline": roof,
           "sweep_iters_per_s": round(w.iters / solve_s, 1),
           "gap_at_end": r["gap"], "primal_feasible": r["feasible"]}
    out["sweep_by_pair"] = {}
    for cfg in (() if a.no_pairs else (3, 5)):
        log(f"[bench] sweep roofline, config {cfg}")
        out["sweep_by_pair"][f"config_{cfg}"] = sweep_roofline(cfg, a.seed)
        log(f"[bench]   {out['sweep_by_pair'][f'config_{cfg}']}")
    if not a.no_pairs:
        from synth import CONFIGS
        T4 = CONFIGS[4].temperature
        log(f"[bench] smoothed sweep, config 4, T={T4}")
        out["sweep_by_pair"]["config_4_smoothed"] = sweep_roofline(4, a.seed, temperature=T4)
        log(f"[bench]   {out['sweep_by_pair']['config_4_smoothed']}")
        # extra scale point (not one of the workload configs): the largest
        # pair's geometry with K raised until the working set is well past
        # the 256 MB Infinity Cache, so the sweep streams from HBM
        log("[bench] sweep roofline, config 5 geometry with K = 144 (HBM-resident scale point)")
        out["sweep_by_pair"]["config_5_k144_hbm_point"] = sweep_roofline(5, a.seed, iters=50, k=144)
        log(f"[bench]   {out['sweep_by_pair']['config_5_k144_hbm_point']}")
    if not a.no_gap:
        import statistics
        gaps = {}
        seeds = [int(x) for x in a.gap_seeds.split(",")]
        # the three forms on the same pairs: the 1000-face pair (Jacobi) and
        # the largest pair (Jacobi and quasi-Newton)
        runs = [(3, "jacobi", FORMS, True), (5, "jacobi", FORMS, True), (5, "lbfgs", FORMS, True),
                (5, "jacobi", ("mixed_bf16",), False)]   # the last: rounding alone, for comparison
        for cfg, solver, forms, repair in runs:
            for form in forms:
                key = f"config_{cfg}_{form}_{solver}" + ("" if repair else "_rounding_only")
                per_seed = {}
                for sd in seeds:
                    log(f"[bench] time-to-1%-gap {key}, seed {sd}")
                    kw = dict(form=form, solver=solver, check_every=10, qn_check_every=10, repair=repair)
                    try:
                        if sd == seeds[0]:
                            time_to_gap(cfg, sd, max_iters=10, qn_max_iters=10, **kw)   # untimed: loads the kernels
                        per_seed[str(sd)] = time_to_gap(cfg, sd, **kw)
                    except RuntimeError as e:   # e.g. a pair that presolve proves infeasible
                        per_seed[str(sd)] = {"error": str(e)}
                    log(f"[bench]   {per_seed[str(sd)]}")
                ok = [v for v in per_seed.values() if v.get("seconds") is not None]
                gaps[key] = {"median_seconds": round(statistics.median([v["seconds"] for v in ok]), 6) if ok else None,
                             "median_iters": statistics.median([v["iters"] for v in ok]) if ok else None,
                             "seeds_reaching_1pct": len(ok), "per_seed": per_seed}
        out["time_to_1pct_gap"] = gaps
        log("[bench] full pipeline, largest pair")
        pipeline_run(5, a.seed, iters=20)   # untimed: loads the kernels
        out["pipeline_largest"] = pipeline_run(5, a.seed)
        log(f"[bench]   {out['pipeline_largest']}")
    if not a.no_gap:
        log("[bench] coarse-to-fine 500 -> 1000 -> 2000 -> 4000 faces")
        c2f_run(a.seed, levels=(500, 1000))   # untimed: loads the kernels
        out["coarse_to_fine"] = c2f_run(a.seed)
        log(f"[bench]   {out['coarse_to_fine']}")
    if not a.no_gap:
        log("[bench] generic 0-1 ILP (assignment + side rows)")
        out["generic_ilp"] = generic_ilp_run(seed=a.seed)
        log(f"[bench]   {out['generic_ilp']}")
    if not (a.no_search or a.no_gap):   # a time-to-solution figure, like the gap runs
        log("[bench] exact search, 80-face pair with noisy descriptors (noise 1.0, K = 16)")
        out["exact_search"] = exact_search_run()
        log(f"[bench]   {out['exact_search']}")
    log("[bench] copy bandwidth (HBM peak check)")
    out["copy_bandwidth"] = copy_bandwidth()
    log(f"[bench]   {out['copy_bandwidth']}")
    if not a.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(a.config, a.seed, a.cpu_sample_iters)
        log(f"[bench]   {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
