// Gradient of the smoothed dual bound with respect to the descriptors (A11).
//
// L_T(lambda) = offset + sum_j softmin_T over S_j, the temperature-smoothed
// version of the dual objective of Eq. (D).  With lambda^j_i = c_i/|J_i| +
// phi^j_i and phi held fixed, dL/dc_i is the mean over the rows of i of the
// marginals mu^j_i = P(s_i = 1) (1 for variables fixed to 1, 0 for those fixed
// to 0).  Through Eq. (cost) (Sec. 4.2), with areas and candidates constant:
//   dL/dw(m, n)  = sum of dL/dc_p over the corners (m, n) of elements p,
//   dL/dF_X(m)   = sum_n dL/dw(m, n) (A_X(m) + A_Y(n)) (F_X(m) - F_Y(n)) / d(m, n),
//   dL/dF_Y(n)   = - the same terms summed over m.
// All sums run in fixed orders (no floating-point atomics).
#include <cmath>

#include "dm_internal.h"

namespace {

template <typename R>
__global__ void k_gcost(const int8_t* state, const int32_t* var_red, const uint8_t* deg, const R* mu, int64_t nP,
                        double scale, float* g) {
  int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= nP) return;
  int8_t s = state[p];
  double v;
  if (s == 1) v = 1.0;
  else if (s == 0) v = 0.0;
  else {
    int32_t i = var_red[p];
    const R* m = mu + size_t(i) * REC;
    int d = deg[i];
    double a = 0.0;
    for (int k = 0; k < d; ++k) a += double(m[k]);
    v = a / d;
  }
  g[p] = float(scale * v);
}

// one wave per candidate pair: lane-strided partial sums over the pair's
// corner list, then an xor butterfly (a fixed order)
__global__ void k_gw(const int32_t* corner_ptr, const int32_t* corner_list, int64_t nC, const float* gcost,
                     float* gw) {
  const int64_t i = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= nC) return;   // uniform across the wave
  const int lane = threadIdx.x & 63;
  double a = 0.0;
  for (int32_t k = corner_ptr[i] + lane; k < corner_ptr[i + 1]; k += 64) a += double(gcost[corner_list[k] / 3]);
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
  if (lane == 0) gw[i] = float(a);
}

// one thread per (X vertex, descriptor dimension)
__global__ void k_gfx(const int32_t* xstart, const int32_t* cpair, int32_t nvx, int32_t nvy, const float* gw,
                      const float* pa, const float* pd, const float* FX, const float* FY, int32_t D, float* gFX) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(nvx) * D) return;
  int32_t m = int32_t(t / D), k = int32_t(t % D);
  float x = FX[int64_t(m) * D + k];
  double acc = 0.0;
  for (int32_t i = xstart[m]; i < xstart[m + 1]; ++i) {
    float d = pd[i];
    if (d == 0.0f || gw[i] == 0.0f) continue;
    int32_t n = cpair[i] % nvy;
    double coef = double(gw[i]) * double(pa[i]) / double(d);
    acc += coef * double(x - FY[int64_t(n) * D + k]);
  }
  gFX[t] = float(acc);
}

// one thread per (Y vertex, descriptor dimension)
__global__ void k_gfy(const int32_t* ystart, const int32_t* cpair_t, const int32_t* cpair, int32_t nvy,
                      int32_t nvy_count, const float* gw, const float* pa, const float* pd, const float* FX,
                      const float* FY, int32_t D, float* gFY) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(nvy_count) * D) return;
  int32_t n = int32_t(t / D), k = int32_t(t % D);
  float y = FY[int64_t(n) * D + k];
  double acc = 0.0;
  for (int32_t q = ystart[n]; q < ystart[n + 1]; ++q) {
    int32_t i = cpair_t[q];
    float d = pd[i];
    if (d == 0.0f || gw[i] == 0.0f) continue;
    int32_t m = cpair[i] / nvy;
    double coef = double(gw[i]) * double(pa[i]) / double(d);
    acc -= coef * double(FX[int64_t(m) * D + k] - y);
  }
  gFY[t] = float(acc);
}

}  // namespace

template <typename R>
static dm_status backward_impl(dm_ctx* ctx, const R* lam, R T, double scale, const float* FX, const float* FY,
                               int32_t D, float* gcost, float* gFX, float* gFY, double* value) {
  hipStream_t st = ctx->stream;
  DArr<unsigned char> bufs[2];
  DM_TRY(dual_import<R>(ctx, lam, bufs));
  const size_t bytes = size_t(std::max<int64_t>(ctx->n_free, 1)) * REC * sizeof(R);
  DM_ALLOC(ctx, ctx->mrec, bytes);
  DM_HIP(ctx, hipMemsetAsync(ctx->mrec.p, 0, bytes, st));
  DM_ALLOC(ctx, ctx->scal, 16);
  DM_TRY(dual_sweep<R>(ctx, SWEEP_EVAL, true, bufs[0].p, ctx->mrec.p, R(0), T, ctx->scal.p + 2));
  DM_TRY(dual_flush(ctx));
  DM_ALLOC(ctx, ctx->gcost_tmp, size_t(ctx->nP));
  DM_TRY(corner_lists(ctx));
  DM_ALLOC(ctx, ctx->gw, size_t(std::max<int64_t>(ctx->nC, 1)));
  k_gcost<R><<<grid_for(ctx->nP, 256), 256, 0, st>>>(ctx->state.p, ctx->var_red.p, ctx->var_deg.p,
                                                     reinterpret_cast<const R*>(ctx->mrec.p), ctx->nP, scale,
                                                     ctx->gcost_tmp.p);
  if (ctx->nC > 0)
    k_gw<<<grid_for(ctx->nC, 4), 256, 0, st>>>(ctx->corner_ptr.p, ctx->corner_list.p, ctx->nC, ctx->gcost_tmp.p,
                                               ctx->gw.p);
  const int32_t nvx = ctx->X.nv, nvy = ctx->Y.nv;
  k_gfx<<<grid_for(int64_t(nvx) * D, 256), 256, 0, st>>>(ctx->cand_xstart.p, ctx->cpair.p, nvx, nvy, ctx->gw.p,
                                                         ctx->pair_a.p, ctx->pair_d.p, FX, FY, D, gFX);
  k_gfy<<<grid_for(int64_t(nvy) * D, 256), 256, 0, st>>>(ctx->cand_ystart.p, ctx->cpair_t.p, ctx->cpair.p, nvy,
                                                         nvy, ctx->gw.p, ctx->pair_a.p, ctx->pair_d.p, FX, FY, D,
                                                         gFY);
  DM_LAUNCH_CHECK(ctx);
  if (gcost)
    DM_HIP(ctx, hipMemcpyAsync(gcost, ctx->gcost_tmp.p, sizeof(float) * ctx->nP, hipMemcpyDeviceToDevice, st));
  if (value) {
    DM_HIP(ctx, hipMemcpyAsync(value, ctx->scal.p + 2, sizeof(double), hipMemcpyDeviceToHost, st));
    DM_HIP(ctx, hipStreamSynchronize(st));
  }
  return DM_OK;
}

extern "C" dm_status dm_smoothed_backward(dm_ctx* ctx, const void* lambda, double temperature, int32_t msg_prec,
                                          double grad_out, const float* FX, const float* FY, int32_t D,
                                          float* gcost, float* gFX, float* gFY, double* value) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!ctx->has_space || !ctx->has_cost) return dm_fail(ctx, DM_ERR_STATE, "dm_smoothed_backward: build space and costs first");
  if (ctx->generic || !ctx->desc_costs)
    return dm_fail(ctx, DM_ERR_STATE, "dm_smoothed_backward: needs costs from descriptors (dm_build_costs)");
  if ((!lambda && ctx->nnz > 0) || !FX || !FY || !gFX || !gFY || D < 1)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_smoothed_backward: bad arguments");
  if (!(temperature > 0.0)) return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_smoothed_backward: temperature must be > 0");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  if (msg_prec == DM_PREC_FP32)
    return backward_impl<float>(ctx, static_cast<const float*>(lambda), float(temperature), grad_out, FX, FY, D,
                                gcost, gFX, gFY, value);
  if (msg_prec == DM_PREC_FP64)
    return backward_impl<double>(ctx, static_cast<const double*>(lambda), temperature, grad_out, FX, FY, D, gcost,
                                 gFX, gFY, value);
  return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_smoothed_backward: message precision must be FP32 or FP64");
}
