// Exact search on the residual of confident fixing (Appendix "Coarse-to-fine
// solving strategy": the variables left free after fixing are solved exactly;
// the paper hands them to a commercial MILP solver, here a depth-first branch
// and bound of the library's own).
//
// A node is the problem with the base fixings plus the branching decisions on
// its path.  Per node, all on the device: presolve from the node's fixings
// (integer unit propagation; an infeasible node is pruned), Jacobi iterations
// whose best bound is a valid lower bound of the node's ILP (Eq. (D) is a
// Lagrangean dual), perturbation rounding for a primal, and one min-marginal
// sweep for the branching choice: the free variable whose summed min-marginal
// differences are closest to zero (the least confident one; ties to the lower
// variable), with the value its min-marginals prefer explored first.  A node is
// pruned when its bound reaches the incumbent; the search is exact when the
// tree is exhausted.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "dm_internal.h"

namespace {

// key of free variable i: (|sum_j M^j_i| as FP32 bits) << 32 | i, so the
// smallest key is the least confident variable, ties to the lower index
template <typename R>
__global__ void k_branch_keys(const R* mrec, const uint8_t* deg, int64_t nfree, unsigned long long* best) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  unsigned long long key = ~0ull;
  if (i < nfree) {
    const R* m = mrec + size_t(i) * REC;
    double sum = 0.0;
    for (int k = 0; k < deg[i]; ++k) sum += double(m[k]);
    const float a = float(fabs(sum));   // >= 0: its bits order like its value
    key = (static_cast<unsigned long long>(__float_as_uint(a)) << 32) | static_cast<unsigned long long>(i);
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(key, o);
    key = other < key ? other : key;
  }
  if ((threadIdx.x & 63) == 0 && key != ~0ull) atomicMin(best, key);
}

// preferred value of free variable i: 1 when its summed min-marginal
// differences are negative
template <typename R>
__global__ void k_branch_pref(const R* mrec, const uint8_t* deg, const unsigned long long* best,
                              const int32_t* free_var, int32_t* out) {
  const int32_t i = int32_t(*best & 0xFFFFFFFFull);
  const R* m = mrec + size_t(i) * REC;
  double sum = 0.0;
  for (int k = 0; k < deg[i]; ++k) sum += double(m[k]);
  out[0] = free_var[i];
  out[1] = sum < 0.0 ? 1 : 0;
}

__global__ void k_apply_path(const int32_t* path, int32_t n, int8_t* fix) {
  const int32_t k = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < n) fix[path[2 * k]] = int8_t(path[2 * k + 1]);
}

__global__ void k_state_to_x(const int8_t* state, int64_t nP, uint8_t* x) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < nP) x[p] = state[p] == 1 ? 1 : 0;
}

// ---- local repair: the neighbourhood of the rows a primal violates
// rows of the full problem that x violates (one thread per row)
__global__ void k_viol_flags(const int32_t* row_ptr, const int32_t* ent_var, const int8_t* ent_coef,
                             const int32_t* row_b, int64_t nrows, const uint8_t* x, uint8_t* rflag, int* count) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nrows) return;
  int64_t s = 0;
  for (int32_t i = row_ptr[j]; i < row_ptr[j + 1]; ++i)
    if (x[ent_var[i]]) s += ent_coef[i];
  const bool v = s != row_b[j];
  rflag[j] = v ? 1 : 0;
  if (v) atomicAdd(count, 1);
}

// every element of a flagged row joins the neighbourhood (one thread per row;
// a plain store of 1, so concurrent marks of one element agree)
__global__ void k_mark_elems(const int32_t* row_ptr, const int32_t* ent_var, int64_t nrows, const uint8_t* rflag,
                             uint8_t* eflag) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nrows || !rflag[j]) return;
  for (int32_t i = row_ptr[j]; i < row_ptr[j + 1]; ++i) eflag[ent_var[i]] = 1;
}

// a closedness row that touches the neighbourhood is flagged for the next
// step (projection rows span a whole face's candidates and are not followed)
__global__ void k_mark_rows(const int32_t* row_ptr, const int32_t* ent_var, int64_t nc, const uint8_t* eflag,
                            uint8_t* rflag) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nc || rflag[j]) return;
  for (int32_t i = row_ptr[j]; i < row_ptr[j + 1]; ++i)
    if (eflag[ent_var[i]]) {
      rflag[j] = 1;
      return;
    }
}

// fixings of the repair: presolve's own fixings stay, the neighbourhood is
// free, every other element keeps its value in x
__global__ void k_repair_fix(const int8_t* state, const uint8_t* eflag, const uint8_t* x, int64_t nP, int8_t* fix,
                             int* nfree) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= nP) return;
  const int8_t st = state[p];
  const bool free_ = st < 0 && eflag[p];
  fix[p] = st >= 0 ? st : (free_ ? int8_t(-1) : int8_t(x[p] ? 1 : 0));
  if (free_) atomicAdd(nfree, 1);
}

__global__ void k_set_fix(int8_t* fix, int32_t elem, int32_t value) { fix[elem] = int8_t(value); }

struct Decision {
  int32_t elem, value;
};

template <typename R>
dm_status node_bound_and_branch(dm_ctx* ctx, const dm_search_params& P, DArr<unsigned char>& lam_buf,
                                double* lb, bool* branch, Decision* choice) {
  hipStream_t st = ctx->stream;
  const int64_t nnz = ctx->nnz, nf = ctx->n_free;
  DM_ALLOC(ctx, lam_buf, size_t(std::max<int64_t>(nnz, 1)) * sizeof(R));
  R* lam = reinterpret_cast<R*>(lam_buf.p);
  const int32_t prec = sizeof(R) == 4 ? DM_PREC_FP32 : DM_PREC_FP64;
  DM_TRY(dm_init_lambda(ctx, prec, lam));
  DArr<double> trace;
  const int32_t iters = std::max(P.dual_iters, 1);
  DM_ALLOC(ctx, trace, size_t(iters));
  DM_TRY(dm_dual_solve(ctx, iters, P.omega, 0.0, prec, lam, trace.p));
  std::vector<double> tr(static_cast<size_t>(iters), 0.0);
  DM_HIP(ctx, hipMemcpyAsync(tr.data(), trace.p, sizeof(double) * iters, hipMemcpyDeviceToHost, st));
  DM_HIP(ctx, hipStreamSynchronize(st));
  double best = -std::numeric_limits<double>::infinity();
  for (double v : tr) best = std::max(best, v);
  double at_end = 0.0;
  DM_TRY(dm_lower_bound(ctx, lam, 0.0, prec, &at_end));
  *lb = std::max(best, at_end);
  *branch = nf > 0;
  if (!*branch) return DM_OK;
  // min-marginal differences at the final multipliers
  DArr<unsigned char> bufs[2];
  DM_TRY(dual_flush(ctx));
  DM_TRY(dual_import<R>(ctx, lam, bufs));
  const size_t bytes = size_t(nf) * REC * sizeof(R);
  DM_ALLOC(ctx, ctx->mrec, bytes);
  DM_HIP(ctx, hipMemsetAsync(ctx->mrec.p, 0, bytes, st));
  DM_TRY(dual_sweep<R>(ctx, SWEEP_EVAL, false, bufs[0].p, ctx->mrec.p, R(0), R(0), nullptr));
  DArr<unsigned long long> key;
  DArr<int32_t> out;
  DM_ALLOC(ctx, key, 1);
  DM_ALLOC(ctx, out, 2);
  DM_HIP(ctx, hipMemsetAsync(key.p, 0xFF, sizeof(unsigned long long), st));
  k_branch_keys<R><<<grid_for(nf, 256), 256, 0, st>>>(reinterpret_cast<const R*>(ctx->mrec.p), ctx->var_deg.p, nf,
                                                       key.p);
  k_branch_pref<R><<<1, 1, 0, st>>>(reinterpret_cast<const R*>(ctx->mrec.p), ctx->var_deg.p, key.p,
                                    ctx->free_var.p, out.p);
  DM_LAUNCH_CHECK(ctx);
  const int32_t* src[2] = {out.p, out.p + 1};
  int32_t v[2];
  DM_TRY(read_i32s(ctx, 2, src, v));
  choice->elem = v[0];
  choice->value = v[1];
  return DM_OK;
}

template <typename R>
dm_status search_impl(dm_ctx* ctx, const dm_search_params& P, const int8_t* base_fix, uint8_t* x,
                      double* primal_obj, double* bound, int32_t* nodes_out, int32_t* status) {
  hipStream_t st = ctx->stream;
  const int64_t nP = ctx->nP;
  DArr<int8_t> fix;
  DArr<uint8_t> xnode;
  DArr<int32_t> path_dev;
  DArr<unsigned char> lam_buf;
  // presolve fixpoint of the last node that branched, for its preferred child
  DArr<int8_t> parent_state;
  bool parent_ready = false;
  DM_ALLOC(ctx, fix, size_t(std::max<int64_t>(nP, 1)));
  DM_ALLOC(ctx, xnode, size_t(std::max<int64_t>(nP, 1)));
  double incumbent = std::numeric_limits<double>::infinity();
  double root_lb = -std::numeric_limits<double>::infinity();
  bool root_done = false, limit_hit = false;
  int32_t nodes = 0;
  // depth-first: every stack entry is a full path of decisions
  std::vector<std::vector<Decision>> stack;
  stack.emplace_back();
  // One node: its fixings, presolve, bound, primal and children.  A failing
  // call's early return leaves only this function, so every failure still
  // reaches the restore of the base problem after the loop.
  auto visit = [&](std::vector<Decision>& path) -> dm_status {
    // The preferred child is popped right after its parent: its fixings are
    // the parent's presolve fixpoint plus the new decision, the same
    // fixpoint as the base fixings plus the whole path (unit propagation is
    // monotone), reached in fewer propagation rounds.  Every node's
    // multipliers start from c / |J|: starting a child from its parent's
    // multipliers took the 80-face test pair with an integrality gap past
    // 3000 nodes without a proof, where the cold start proves it in 897.
    const bool from_parent = parent_ready;
    parent_ready = false;
    if (from_parent) {
      DM_HIP(ctx, hipMemcpyAsync(fix.p, parent_state.p, size_t(nP), hipMemcpyDeviceToDevice, st));
      k_set_fix<<<1, 1, 0, st>>>(fix.p, path.back().elem, path.back().value);
      DM_LAUNCH_CHECK(ctx);
    } else if (base_fix)
      DM_HIP(ctx, hipMemcpyAsync(fix.p, base_fix, size_t(nP), hipMemcpyDeviceToDevice, st));
    else
      DM_HIP(ctx, hipMemsetAsync(fix.p, 0xFF, size_t(nP), st));
    if (!from_parent && !path.empty()) {
      std::vector<int32_t> flat;
      for (const Decision& d : path) {
        flat.push_back(d.elem);
        flat.push_back(d.value);
      }
      DM_ALLOC(ctx, path_dev, flat.size());
      DM_HIP(ctx, hipMemcpyAsync(path_dev.p, flat.data(), sizeof(int32_t) * flat.size(), hipMemcpyHostToDevice,
                                 st));
      k_apply_path<<<grid_for(int64_t(path.size()), 256), 256, 0, st>>>(path_dev.p, int32_t(path.size()), fix.p);
      DM_LAUNCH_CHECK(ctx);
      DM_HIP(ctx, hipStreamSynchronize(st));   // flat is host memory
    }
    const dm_status ps = presolve_reduce(ctx, fix.p);
    if (ps == DM_ERR_INFEASIBLE) {
      ctx->err.clear();
      if (!root_done) {
        root_done = true;
        root_lb = std::numeric_limits<double>::infinity();
      }
      return DM_OK;
    }
    if (ps != DM_OK) return ps;
    DM_TRY(cost_offset(ctx));
    double lb = 0.0;
    bool branch = false;
    Decision choice{0, 0};
    DM_TRY(node_bound_and_branch<R>(ctx, P, lam_buf, &lb, &branch, &choice));
    if (!root_done) {
      root_done = true;
      root_lb = lb;
    }
    const double tol = P.rel_tol * std::max(1.0, std::fabs(incumbent));
    if (lb >= incumbent - tol) return DM_OK;   // cannot improve on the incumbent
    // a primal at this node
    double pobj = 0.0;
    int32_t feas = 0, used = 0;
    if (!branch) {   // presolve fixed everything: the state is the assignment
      k_state_to_x<<<grid_for(nP, 256), 256, 0, st>>>(ctx->state.p, nP, xnode.p);
      DM_LAUNCH_CHECK(ctx);
      int64_t viol = 0;
      DM_TRY(dm_check_primal(ctx, xnode.p, &viol));
      feas = viol == 0;
      pobj = ctx->offset;
    } else {
      dm_round_params rp = P.round;
      rp.msg_prec = sizeof(R) == 4 ? DM_PREC_FP32 : DM_PREC_FP64;
      DM_TRY(dm_round_primal(ctx, &rp, lam_buf.p, xnode.p, &pobj, &feas, &used));
    }
    if (feas && pobj < incumbent) {
      incumbent = pobj;
      DM_HIP(ctx, hipMemcpyAsync(x, xnode.p, size_t(nP), hipMemcpyDeviceToDevice, st));
    }
    if (!branch || lb >= incumbent - P.rel_tol * std::max(1.0, std::fabs(incumbent))) return DM_OK;
    // children: the preferred value is explored first (pushed last); keep
    // this node's fixpoint for it
    DM_ALLOC(ctx, parent_state, size_t(std::max<int64_t>(nP, 1)));
    DM_HIP(ctx, hipMemcpyAsync(parent_state.p, ctx->state.p, size_t(nP), hipMemcpyDeviceToDevice, st));
    parent_ready = true;
    std::vector<Decision> other = path, pref = std::move(path);
    other.push_back({choice.elem, 1 - choice.value});
    pref.push_back(choice);
    stack.push_back(std::move(other));
    stack.push_back(std::move(pref));
    return DM_OK;
  };
  dm_status result = DM_OK;
  while (!stack.empty()) {
    if (nodes >= P.max_nodes) {
      limit_hit = true;
      break;
    }
    std::vector<Decision> path = std::move(stack.back());
    stack.pop_back();
    ++nodes;
    if ((result = visit(path)) != DM_OK) break;
  }
  // back to the problem with the base fixings only
  const std::string msg = ctx->err;
  dm_status rs = presolve_reduce(ctx, base_fix);
  if (rs == DM_ERR_INFEASIBLE && base_fix) {   // infeasible base fixings: back to no fixings
    ctx->err.clear();
    rs = presolve_reduce(ctx, nullptr);
  }
  if (rs != DM_OK) {
    ctx->has_space = false;   // the reduced problem is half rebuilt: unusable
    return result != DM_OK ? result : rs;
  }
  if (ctx->has_cost) DM_TRY(cost_offset(ctx));
  ++ctx->cost_generation;   // solver state of the node problems is stale
  ctx->err = msg;
  if (result != DM_OK) return result;
  DM_HIP(ctx, hipStreamSynchronize(st));
  *nodes_out = nodes;
  *primal_obj = incumbent;
  if (!limit_hit) {
    *status = std::isfinite(incumbent) ? DM_SEARCH_OPTIMAL : DM_SEARCH_INFEASIBLE;
    *bound = incumbent;
  } else {
    *status = DM_SEARCH_LIMIT;
    *bound = std::min(root_lb, incumbent);
  }
  if (!std::isfinite(incumbent)) DM_HIP(ctx, hipMemsetAsync(x, 0, size_t(nP), st));
  DM_HIP(ctx, hipStreamSynchronize(st));
  return DM_OK;
}

}  // namespace

static dm_status exact_search(dm_ctx* ctx, const dm_search_params* params, const int8_t* base_fix, uint8_t* x,
                              double* primal_obj, double* bound, int32_t* nodes, int32_t* status) {
  if (!ctx->has_space || !ctx->has_cost) return dm_fail(ctx, DM_ERR_STATE, "dm_exact_search: build space and costs first");
  if (!params || !x || !primal_obj || !bound || !nodes || !status)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_exact_search: NULL argument");
  const dm_search_params& P = *params;
  if (P.max_nodes < 1 || P.dual_iters < 1 || !(P.omega > 0.0 && P.omega <= 1.0) || !(P.rel_tol >= 0.0))
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_exact_search: bad parameters");
  if (P.round.msg_prec != DM_PREC_FP32 && P.round.msg_prec != DM_PREC_FP64)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_exact_search: message precision must be FP32 or FP64");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  DM_TRY(dual_flush(ctx));
  return P.round.msg_prec == DM_PREC_FP32 ? search_impl<float>(ctx, P, base_fix, x, primal_obj, bound, nodes, status)
                                          : search_impl<double>(ctx, P, base_fix, x, primal_obj, bound, nodes, status);
}

extern "C" dm_status dm_exact_search(dm_ctx* ctx, const dm_search_params* params, const int8_t* base_fix,
                                     uint8_t* x, double* primal_obj, double* bound, int32_t* nodes,
                                     int32_t* status, dm_space_info* info) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  const dm_status s = exact_search(ctx, params, base_fix, x, primal_obj, bound, nodes, status);
  if (info && ctx->has_space) fill_info(ctx, info);   // also after an error: the sizes in force
  return s;
}

// One neighbourhood of h steps around the violated rows (grown from the
// previous one's marks): fix every element outside it at its value in x and
// search the rest exactly; on success x holds the repaired primal.  The
// search leaves its base problem in place, which the caller restores.
static dm_status repair_hop(dm_ctx* ctx, const dm_search_params& P, int32_t h, uint8_t* x, uint8_t* rflag,
                            uint8_t* eflag, int8_t* fix, uint8_t* xbest, int* cnt, double* primal_obj,
                            int32_t* feasible, int64_t* n_free) {
  hipStream_t st = ctx->stream;
  const int64_t nP = ctx->nP, nrows = ctx->n_rows_full, nc = ctx->n_closed_full;
  if (h > 1)
    k_mark_rows<<<grid_for(std::max<int64_t>(nc, 1), 256), 256, 0, st>>>(ctx->row_ptr.p, ctx->ent_var.p, nc,
                                                                         eflag, rflag);
  k_mark_elems<<<grid_for(std::max<int64_t>(nrows, 1), 256), 256, 0, st>>>(ctx->row_ptr.p, ctx->ent_var.p, nrows,
                                                                           rflag, eflag);
  DM_HIP(ctx, hipMemsetAsync(cnt + 1, 0, sizeof(int), st));
  k_repair_fix<<<grid_for(nP, 256), 256, 0, st>>>(ctx->state.p, eflag, x, nP, fix, cnt + 1);
  DM_LAUNCH_CHECK(ctx);
  int32_t nf = 0;
  DM_TRY(read_i32(ctx, cnt + 1, &nf));
  *n_free = nf;
  double pobj = 0.0, bound = 0.0;
  int32_t nodes = 0, status = 0;
  DM_TRY(exact_search(ctx, &P, fix, xbest, &pobj, &bound, &nodes, &status));
  if (std::isfinite(pobj)) {
    DM_HIP(ctx, hipMemcpyAsync(x, xbest, size_t(nP), hipMemcpyDeviceToDevice, st));
    *primal_obj = pobj;
    *feasible = 1;
  }
  return DM_OK;
}

// Local repair of a primal (Appendix "Coarse-to-fine solving strategy": the
// confident part of an assignment stays fixed and the rest is solved
// exactly).  The neighbourhood of the rows x violates is freed step by step:
// step 1 frees every element of the violated rows; each further step frees
// the elements of the closedness rows that touch the neighbourhood.  Every
// other element keeps its value in x (or its presolve value), and the exact
// search solves the neighbourhood; a neighbourhood without a feasible
// completion grows by one step, up to max_hops.
static dm_status repair_primal(dm_ctx* ctx, const dm_search_params& P, int32_t max_hops, uint8_t* x,
                               double* primal_obj, int32_t* feasible, int32_t* hops_used, int64_t* n_free) {
  hipStream_t st = ctx->stream;
  const int64_t nP = ctx->nP, nrows = ctx->n_rows_full;
  const int64_t generation = ctx->cost_generation;
  *feasible = 0;
  *hops_used = 0;
  *n_free = 0;
  *primal_obj = std::numeric_limits<double>::infinity();
  DArr<uint8_t> rflag, eflag, xbest;
  DArr<int8_t> fix, held;
  DArr<int> cnt;
  DM_ALLOC(ctx, rflag, size_t(std::max<int64_t>(nrows, 1)));
  DM_ALLOC(ctx, eflag, size_t(std::max<int64_t>(nP, 1)));
  DM_ALLOC(ctx, fix, size_t(std::max<int64_t>(nP, 1)));
  DM_ALLOC(ctx, xbest, size_t(std::max<int64_t>(nP, 1)));
  DM_ALLOC(ctx, cnt, 2);
  DM_HIP(ctx, hipMemsetAsync(cnt.p, 0, 2 * sizeof(int), st));
  k_viol_flags<<<grid_for(std::max<int64_t>(nrows, 1), 256), 256, 0, st>>>(
      ctx->row_ptr.p, ctx->ent_var.p, ctx->ent_coef.p, ctx->row_b.p, nrows, x, rflag.p, cnt.p);
  DM_LAUNCH_CHECK(ctx);
  int32_t nviol = 0;
  DM_TRY(read_i32(ctx, cnt.p, &nviol));
  if (nviol == 0) {   // already feasible: nothing to repair
    DM_ALLOC(ctx, ctx->scal, 16);
    DM_TRY(sum_f64(ctx, ctx->cost64.p, nP, x, SUM_U8_NZ, ctx->scal.p + 1));
    DM_HIP(ctx, hipMemcpyAsync(primal_obj, ctx->scal.p + 1, sizeof(double), hipMemcpyDeviceToHost, st));
    DM_HIP(ctx, hipStreamSynchronize(st));
    *feasible = 1;
    return DM_OK;
  }
  // the fixings in force now (a presolve fixpoint), to restore this problem
  DM_ALLOC(ctx, held, size_t(std::max<int64_t>(nP, 1)));
  DM_HIP(ctx, hipMemcpyAsync(held.p, ctx->state.p, size_t(nP), hipMemcpyDeviceToDevice, st));
  DM_HIP(ctx, hipMemsetAsync(eflag.p, 0, size_t(nP), st));
  // every failure from here on still restores the held problem below
  dm_status result = DM_OK;
  for (int32_t h = 1; h <= max_hops && !*feasible; ++h) {
    *hops_used = h;
    result = repair_hop(ctx, P, h, x, rflag.p, eflag.p, fix.p, xbest.p, cnt.p, primal_obj, feasible, n_free);
    if (result != DM_OK) break;
  }
  // back to the problem the context held (the search leaves its base in place)
  const std::string msg = ctx->err;
  const dm_status rs = presolve_reduce(ctx, held.p);
  if (rs != DM_OK) {
    ctx->has_space = false;
    return result != DM_OK ? result : rs;
  }
  if (ctx->has_cost) DM_TRY(cost_offset(ctx));
  // the same problem as before the call (presolve from its own fixpoint
  // rebuilds the same reduced arrays): solver sessions on it stay valid
  ctx->cost_generation = generation;
  ctx->err = msg;
  DM_HIP(ctx, hipStreamSynchronize(st));
  return result;
}

extern "C" dm_status dm_repair_primal(dm_ctx* ctx, const dm_search_params* params, int32_t max_hops, uint8_t* x,
                                      double* primal_obj, int32_t* feasible, int32_t* hops_used, int64_t* n_free) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!ctx->has_space || !ctx->has_cost) return dm_fail(ctx, DM_ERR_STATE, "dm_repair_primal: build space and costs first");
  if (!params || !x || !primal_obj || !feasible || !hops_used || !n_free)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_repair_primal: NULL argument");
  if (max_hops < 1) return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_repair_primal: max_hops must be at least 1");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  DM_TRY(dual_flush(ctx));
  return repair_primal(ctx, *params, max_hops, x, primal_obj, feasible, hops_used, n_free);
}
