// Primal rounding (A9) and the exact feasibility check of A x = b.
//
// The paper drives FastDOG's primal heuristic with its own dual (Sec. 4,
// Fig. "pipeline") without restating it.  This library's heuristic rests on
// the sign semantics of min-marginal differences (Appendix "Coarse-to-fine":
// M > 0 prefers 0, M < 0 prefers 1, a variable agrees when all its rows share
// the sign).  On a copy of (c, lambda), per round: sweep every row; if every
// free variable agrees, read off x and check A x = b in integers; otherwise
// perturb the copied costs (agreeing variables pushed further by delta, the
// rest by delta*u with u in [-1, 1) from a counter-based splitmix64 stream),
// run a few Jacobi iterations and grow delta.
#include <cmath>

#include "dm_internal.h"

namespace {

// splitmix64 (Steele, Lea, Flood 2014): one step of the published mixer
__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// u in [-1, 1) for (seed, round, variable): mix(mix(seed) xor (round<<32 | var))
__device__ inline double counter_uniform(uint64_t seed, uint32_t round, uint32_t var) {
  uint64_t z = mix64(mix64(seed) ^ ((uint64_t(round) << 32) | uint64_t(var)));
  return double(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

template <typename R>
__global__ void k_agree(const R* mrec, const uint8_t* deg, int64_t nfree, int8_t* pref, int64_t* count,
                        double* absm) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nfree) return;
  const R* m = mrec + size_t(i) * REC;
  const int d = deg[i];
  bool neg = true, pos = true;
  double a = 0.0;
  for (int k = 0; k < d; ++k) {
    R v = m[k];
    neg = neg && (v < R(0));
    pos = pos && (v > R(0));
    a += fabs(double(v));
  }
  int8_t p = neg ? 1 : (pos ? 0 : -1);
  pref[i] = p;
  absm[i] = a;
  if (p < 0) atomicAdd(reinterpret_cast<unsigned long long*>(count), 1ull);
}

// one-block sums in a fixed order; eight independent accumulators per thread
// keep its loads from waiting on each other
__global__ void k_make_x(const int8_t* state, const int32_t* var_red, const int8_t* pref, int64_t nP, uint8_t* x) {
  int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= nP) return;
  int8_t s = state[p];
  x[p] = s == 1 ? 1 : (s == 0 ? 0 : (pref[var_red[p]] == 1 ? 1 : 0));
}

__global__ void k_violations(const int32_t* row_ptr, const int32_t* ent_var, const int8_t* ent_coef,
                             const int32_t* row_b, int64_t nrows, const uint8_t* x, int64_t* count) {
  int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nrows) return;
  int64_t s = 0;
  for (int32_t i = row_ptr[j]; i < row_ptr[j + 1]; ++i)
    if (x[ent_var[i]]) s += ent_coef[i];
  if (s != row_b[j]) atomicAdd(reinterpret_cast<unsigned long long*>(count), 1ull);
}

// projection rows (all +1, right-hand side 1): one block per row
__global__ __launch_bounds__(256) void k_violations_proj(const int32_t* row_ptr, const int32_t* ent_var,
                                                         int64_t nc, const uint8_t* x, int64_t* count) {
  __shared__ int sh[4];
  const int64_t j = nc + blockIdx.x;
  int c = 0;
  for (int32_t i = row_ptr[j] + threadIdx.x; i < row_ptr[j + 1]; i += blockDim.x) c += x[ent_var[i]] ? 1 : 0;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0 && sh[0] + sh[1] + sh[2] + sh[3] != 1)
    atomicAdd(reinterpret_cast<unsigned long long*>(count), 1ull);
}

// c~_i += Delta_i in both record buffers; the next projection spreads
// Delta_i / |J_i| over the multipliers of i
template <typename R>
__global__ void k_perturb(const int8_t* pref, int64_t nfree, double delta, uint64_t seed, uint32_t round, R* r0,
                          R* r1) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nfree) return;
  int8_t p = pref[i];
  double d = p == 1 ? -delta : (p == 0 ? delta : delta * counter_uniform(seed, round, uint32_t(i)));
  r0[size_t(i) * REC + REC_COST] += R(d);
  r1[size_t(i) * REC + REC_COST] += R(d);
}

}  // namespace

// violated rows of x into icount[1] (enqueued only)
static dm_status enqueue_violations(dm_ctx* ctx, const uint8_t* x) {
  DM_ALLOC(ctx, ctx->icount, 4);
  DM_HIP(ctx, hipMemsetAsync(ctx->icount.p + 1, 0, sizeof(int64_t), ctx->stream));
  const int64_t nc = ctx->n_closed_full;
  if (nc > 0)
    k_violations<<<grid_for(nc, 256), 256, 0, ctx->stream>>>(ctx->row_ptr.p, ctx->ent_var.p, ctx->ent_coef.p,
                                                             ctx->row_b.p, nc, x, ctx->icount.p + 1);
  if (ctx->n_rows_full > nc)
    k_violations_proj<<<unsigned(ctx->n_rows_full - nc), 256, 0, ctx->stream>>>(ctx->row_ptr.p, ctx->ent_var.p,
                                                                                 nc, x, ctx->icount.p + 1);
  DM_LAUNCH_CHECK(ctx);
  return DM_OK;
}

dm_status count_violations(dm_ctx* ctx, const uint8_t* x, int64_t* out) {
  DM_TRY(enqueue_violations(ctx, x));
  DM_HIP(ctx, hipMemcpyAsync(out, ctx->icount.p + 1, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return DM_OK;
}

template <typename R>
static dm_status round_impl(dm_ctx* ctx, const dm_round_params& P, const R* lam, uint8_t* x, double* pobj,
                            int32_t* feasible, int32_t* rounds_used) {
  hipStream_t st = ctx->stream;
  const int64_t nfree = ctx->n_free;
  DM_TRY(dual_import<R>(ctx, lam, ctx->rrec));
  const size_t bytes = size_t(std::max<int64_t>(nfree, 1)) * REC * sizeof(R);
  DM_ALLOC(ctx, ctx->mrec, bytes);
  DM_HIP(ctx, hipMemsetAsync(ctx->mrec.p, 0, bytes, st));
  DM_ALLOC(ctx, ctx->pref, size_t(std::max<int64_t>(nfree, 1)));
  DM_ALLOC(ctx, ctx->icount, 4);
  DM_ALLOC(ctx, ctx->scal, 16);
  DArr<double> absm;
  DM_ALLOC(ctx, absm, size_t(std::max<int64_t>(nfree, 1)));
  double delta = P.delta0;
  int cur = 0;
  *feasible = 0;
  for (int32_t r = 0; r <= P.rounds; ++r) {
    DM_TRY(dual_sweep<R>(ctx, SWEEP_EVAL, false, ctx->rrec[cur].p, ctx->mrec.p, R(0), R(0), nullptr));
    DM_HIP(ctx, hipMemsetAsync(ctx->icount.p, 0, sizeof(int64_t), st));
    if (nfree > 0)
      k_agree<R><<<grid_for(nfree, 256), 256, 0, st>>>(reinterpret_cast<const R*>(ctx->mrec.p), ctx->var_deg.p,
                                                      nfree, ctx->pref.p, ctx->icount.p, absm.p);
    DM_LAUNCH_CHECK(ctx);
    // the undecided count and, on the first round, the automatic perturbation
    // scale (from the summed |M|) come back with one wait
    const bool auto_delta = r == 0 && delta <= 0.0;
    if (auto_delta) DM_TRY(sum_f64(ctx, absm.p, nfree, nullptr, SUM_ALL, ctx->scal.p));
    int64_t undecided = 0;
    double sum_absm = 0.0;
    DM_HIP(ctx, hipMemcpyAsync(&undecided, ctx->icount.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    if (auto_delta)
      DM_HIP(ctx, hipMemcpyAsync(&sum_absm, ctx->scal.p, sizeof(double), hipMemcpyDeviceToHost, st));
    DM_HIP(ctx, hipStreamSynchronize(st));
    if (auto_delta) delta = ctx->nnz ? 0.1 * sum_absm / double(ctx->nnz) : 0.0;
    k_make_x<<<grid_for(ctx->nP, 256), 256, 0, st>>>(ctx->state.p, ctx->var_red.p, ctx->pref.p, ctx->nP, x);
    DM_LAUNCH_CHECK(ctx);
    *rounds_used = r;
    if (undecided == 0) {
      // violations and the objective of x with one wait
      DM_TRY(enqueue_violations(ctx, x));
      DM_TRY(sum_f64(ctx, ctx->cost64.p, ctx->nP, x, SUM_U8_NZ, ctx->scal.p + 1));
      int64_t viol = 0;
      DM_HIP(ctx, hipMemcpyAsync(&viol, ctx->icount.p + 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
      DM_HIP(ctx, hipMemcpyAsync(pobj, ctx->scal.p + 1, sizeof(double), hipMemcpyDeviceToHost, st));
      DM_HIP(ctx, hipStreamSynchronize(st));
      if (viol == 0) {
        *feasible = 1;
        return DM_OK;
      }
    }
    if (r == P.rounds) break;
    k_perturb<R><<<grid_for(std::max<int64_t>(nfree, 1), 256), 256, 0, st>>>(
        ctx->pref.p, nfree, delta, P.seed, uint32_t(r), reinterpret_cast<R*>(ctx->rrec[0].p),
        reinterpret_cast<R*>(ctx->rrec[1].p));
    DM_LAUNCH_CHECK(ctx);
    for (int32_t t = 0; t < P.iters_per_round; ++t) {
      DM_TRY(dual_sweep<R>(ctx, SWEEP_UPDATE, false, ctx->rrec[cur].p, ctx->rrec[cur ^ 1].p, R(P.omega), R(0), nullptr));
      cur ^= 1;
    }
    delta *= P.gamma;
  }
  DM_TRY(sum_f64(ctx, ctx->cost64.p, ctx->nP, x, SUM_U8_NZ, ctx->scal.p + 1));
  DM_LAUNCH_CHECK(ctx);
  DM_HIP(ctx, hipMemcpyAsync(pobj, ctx->scal.p + 1, sizeof(double), hipMemcpyDeviceToHost, st));
  DM_HIP(ctx, hipStreamSynchronize(st));
  return DM_OK;
}

extern "C" dm_status dm_round_primal(dm_ctx* ctx, const dm_round_params* params, const void* lambda, uint8_t* x,
                                     double* primal_obj, int32_t* feasible, int32_t* rounds_used) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!ctx->has_space || !ctx->has_cost) return dm_fail(ctx, DM_ERR_STATE, "dm_round_primal: build space and costs first");
  if (!params || (!lambda && ctx->nnz > 0) || !x || !primal_obj || !feasible || !rounds_used)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_round_primal: NULL argument");
  const dm_round_params& P = *params;
  if (P.rounds < 0 || P.iters_per_round < 0 || !(P.gamma > 0.0) || !(P.omega > 0.0 && P.omega <= 1.0))
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_round_primal: bad parameters");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  if (P.msg_prec == DM_PREC_FP32)
    return round_impl<float>(ctx, P, static_cast<const float*>(lambda), x, primal_obj, feasible, rounds_used);
  if (P.msg_prec == DM_PREC_FP64)
    return round_impl<double>(ctx, P, static_cast<const double*>(lambda), x, primal_obj, feasible, rounds_used);
  return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_round_primal: message precision must be FP32 or FP64");
}

extern "C" dm_status dm_check_primal(dm_ctx* ctx, const uint8_t* x, int64_t* violations) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  if (!ctx->has_space) return dm_fail(ctx, DM_ERR_STATE, "dm_check_primal: no product space");
  if (!x || !violations) return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_check_primal: NULL argument");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  return count_violations(ctx, x, violations);
}
