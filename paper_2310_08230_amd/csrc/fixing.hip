// Confident-variable fixing (Appendix "Coarse-to-fine solving strategy").
//
// At lambda, one min-marginal sweep gives M^j_i for every multiplier; a free
// variable agrees when all its M^j_i are < 0 (it prefers 1) or all are > 0
// (it prefers 0).  The agreeing variables are ranked by |sum_j M^j_i|
// (largest first, ties to the lower variable: a stable radix sort of the
// complemented FP64 score bits over the variables in index order) and the top
// floor(frac * count) are fixed to their preferred values.  The fixings come
// back per element; dm_fix_variables then propagates them and rebuilds the
// reduced (residual) problem.
#include <cmath>

#include "dm_internal.h"

namespace {

// per variable: preference and score key; agreeing variables flagged
template <typename R>
__global__ void k_agree_score(const R* mrec, const uint8_t* deg, int64_t nfree, uint8_t* flag, int8_t* pref,
                              uint64_t* key) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nfree) return;
  const R* m = mrec + size_t(i) * REC;
  const int d = deg[i];
  bool neg = true, pos = true;
  double sum = 0.0;
  for (int k = 0; k < d; ++k) {
    const R v = m[k];
    neg = neg && v < R(0);
    pos = pos && v > R(0);
    sum += double(v);
  }
  flag[i] = (neg || pos) ? 1 : 0;
  pref[i] = neg ? 1 : 0;
  // scores are >= 0, whose IEEE bits order like the values; complementing
  // makes an ascending sort put the largest first
  key[i] = ~static_cast<uint64_t>(__double_as_longlong(fabs(sum)));
}

__global__ void k_compact(const uint8_t* flag, const int32_t* pos, const uint64_t* key, int64_t nfree,
                          uint64_t* key_out, int32_t* var_out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nfree || !flag[i]) return;
  key_out[pos[i]] = key[i];
  var_out[pos[i]] = int32_t(i);
}

__global__ void k_fix_from_state(const int8_t* state, int64_t nP, int8_t* fix) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < nP) fix[p] = state[p];
}

__global__ void k_fix_top(const int32_t* var_sorted, int64_t take, const int32_t* free_var, const int8_t* pref,
                          int8_t* fix) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= take) return;
  const int32_t v = var_sorted[k];
  fix[free_var[v]] = pref[v];
}

template <typename R>
dm_status confident_impl(dm_ctx* ctx, const R* lam, double frac, int8_t* fix, int64_t* n_agree,
                         int64_t* n_fixed) {
  hipStream_t st = ctx->stream;
  const int64_t nf = ctx->n_free, nP = ctx->nP;
  if (nP > 0) k_fix_from_state<<<grid_for(nP, 256), 256, 0, st>>>(ctx->state.p, nP, fix);
  DM_LAUNCH_CHECK(ctx);
  int32_t na = 0;
  int64_t take = 0;
  if (nf > 0) {
    DArr<unsigned char> bufs[2];
    DM_TRY(dual_flush(ctx));
    DM_TRY(dual_import<R>(ctx, lam, bufs));
    const size_t bytes = size_t(nf) * REC * sizeof(R);
    DM_ALLOC(ctx, ctx->mrec, bytes);
    DM_HIP(ctx, hipMemsetAsync(ctx->mrec.p, 0, bytes, st));
    DM_TRY(dual_sweep<R>(ctx, SWEEP_EVAL, false, bufs[0].p, ctx->mrec.p, R(0), R(0), nullptr));
    DArr<uint8_t> flag;
    DArr<int8_t> pref;
    DArr<uint64_t> key, key_c;
    DArr<int32_t> pos, var_c;
    DM_ALLOC(ctx, flag, size_t(nf));
    DM_ALLOC(ctx, pref, size_t(nf));
    DM_ALLOC(ctx, key, size_t(nf));
    DM_ALLOC(ctx, pos, size_t(nf) + 1);
    k_agree_score<R><<<grid_for(nf, 256), 256, 0, st>>>(reinterpret_cast<const R*>(ctx->mrec.p), ctx->var_deg.p,
                                                         nf, flag.p, pref.p, key.p);
    DM_LAUNCH_CHECK(ctx);
    DM_TRY(scan_u8(ctx, flag.p, pos.p, size_t(nf)));
    DM_TRY(read_i32(ctx, pos.p + nf, &na));
    if (na > 0) {
      DM_ALLOC(ctx, key_c, size_t(na));
      DM_ALLOC(ctx, var_c, size_t(na));
      k_compact<<<grid_for(nf, 256), 256, 0, st>>>(flag.p, pos.p, key.p, nf, key_c.p, var_c.p);
      DM_LAUNCH_CHECK(ctx);
      DM_TRY(sort_pairs_u64(ctx, key_c.p, var_c.p, size_t(na), 64));
      take = int64_t(std::floor(frac * double(na)));
      if (take > 0)
        k_fix_top<<<grid_for(take, 256), 256, 0, st>>>(var_c.p, take, ctx->free_var.p, pref.p, fix);
      DM_LAUNCH_CHECK(ctx);
    }
    // the temporaries are freed on return
    DM_HIP(ctx, hipStreamSynchronize(st));
  }
  if (n_agree) *n_agree = na;
  if (n_fixed) *n_fixed = take;
  return DM_OK;
}

}  // namespace

extern "C" dm_status dm_confident_fixing(dm_ctx* ctx, int32_t msg_prec, const void* lambda, double frac,
                                         int8_t* fix, int64_t* n_agree, int64_t* n_fixed) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!ctx->has_space) return dm_fail(ctx, DM_ERR_STATE, "no product space built");
  if (!ctx->has_cost) return dm_fail(ctx, DM_ERR_STATE, "no costs built");
  if (msg_prec != DM_PREC_FP32 && msg_prec != DM_PREC_FP64)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "message precision must be FP32 or FP64");
  if ((!lambda && ctx->nnz > 0) || !fix || !(frac >= 0.0 && frac <= 1.0))
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_confident_fixing: bad arguments");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  if (msg_prec == DM_PREC_FP32)
    return confident_impl<float>(ctx, static_cast<const float*>(lambda), frac, fix, n_agree, n_fixed);
  return confident_impl<double>(ctx, static_cast<const double*>(lambda), frac, fix, n_agree, n_fixed);
}
