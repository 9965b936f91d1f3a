// Costs of Eq. (cost) (Sec. 4.2):
//   c_p = sum_{v=1..3} (A_X(m_v) + A_Y(n_v)) * ||F_X(m_v) - F_Y(n_v)||
// over the product vertices (m_v, n_v) of element p, with mixed vertex areas
// of the posed meshes.  The per-pair weight w(m, n) is computed once per
// candidate pair and gathered three times per element.
#include <cmath>

#include "dm_internal.h"

namespace {

__global__ void k_pair_w64(const int32_t* cpair, int64_t nC, int32_t nvy, const float* FX, const float* FY,
                           int32_t D, const double* AX, const double* AY, double* w, float* pd, float* pa) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nC) return;
  int32_t q = cpair[i];
  int32_t m = q / nvy, n = q % nvy;
  const float* a = FX + int64_t(m) * D;
  const float* b = FY + int64_t(n) * D;
  double s = 0.0;
  for (int32_t k = 0; k < D; ++k) {
    double d = double(a[k]) - double(b[k]);
    s += d * d;
  }
  double d = sqrt(s);
  double A = AX[m] + AY[n];
  w[i] = A * d;
  pd[i] = float(d);
  pa[i] = float(A);
}

__global__ void k_pair_w32(const int32_t* cpair, int64_t nC, int32_t nvy, const float* FX, const float* FY,
                           int32_t D, const double* AX, const double* AY, double* w, float* pd, float* pa) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nC) return;
  int32_t q = cpair[i];
  int32_t m = q / nvy, n = q % nvy;
  const float* a = FX + int64_t(m) * D;
  const float* b = FY + int64_t(n) * D;
  float s = 0.0f;
  for (int32_t k = 0; k < D; ++k) {
    float d = a[k] - b[k];
    s = fmaf(d, d, s);
  }
  float d = sqrtf(s);
  float A = float(AX[m] + AY[n]);
  w[i] = double(A * d);
  pd[i] = d;
  pa[i] = A;
}

// BF16 form: the cost uses the MFMA distance; the backward pass keeps the
// FP32 distance of the unrounded descriptors (the rounding is treated as the
// identity when differentiating)
__global__ void k_pair_w_from_d2(const int32_t* cpair, int64_t nC, int32_t nvy, const float* d2,
                                 const float* FX, const float* FY, int32_t D, const double* AX,
                                 const double* AY, double* w, float* pd, float* pa) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nC) return;
  int32_t q = cpair[i];
  int32_t m = q / nvy, n = q % nvy;
  float d = sqrtf(d2[q]);
  float A = float(AX[m] + AY[n]);
  w[i] = double(A * d);
  const float* a = FX + int64_t(m) * D;
  const float* b = FY + int64_t(n) * D;
  float s = 0.0f;
  for (int32_t k = 0; k < D; ++k) {
    float e = a[k] - b[k];
    s = fmaf(e, e, s);
  }
  pd[i] = sqrtf(s);
  pa[i] = A;
}

__global__ void k_elem_cost(const int32_t* pv, const int32_t* cidx, int64_t nP, const double* w,
                            double* c64, float* c32, float* out, int* err) {
  int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= nP) return;
  double c = 0.0;
  for (int k = 0; k < 3; ++k) c += w[cidx[pv[3 * p + k]]];
  if (!isfinite(c)) atomicOr(err, 1);
  c64[p] = c;
  c32[p] = float(c);
  if (out) out[p] = float(c);
}

__global__ void k_corner_keys(const int32_t* pv, const int32_t* cidx, int64_t nP, uint32_t* key,
                              int32_t* val) {
  int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= 3 * nP) return;
  key[s] = uint32_t(cidx[pv[s]]);
  val[s] = int32_t(s);
}

__global__ void k_corner_ptr(const uint32_t* key, int64_t n, int64_t nC, int32_t* ptr) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i > nC) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (int64_t(key[mid]) < i) lo = mid + 1;
    else hi = mid;
  }
  ptr[i] = int32_t(lo);
}

}  // namespace

// constant of the dual objective: the summed costs of the elements fixed to 1
// Corners of each candidate pair, ascending (3p+v), for the backward pass;
// they depend on the product space only, so they are built once per space,
// on the first backward.
dm_status corner_lists(dm_ctx* ctx) {
  if (ctx->corners_ready) return DM_OK;
  const int64_t nP = ctx->nP, nC = ctx->nC;
  hipStream_t st = ctx->stream;
  DArr<uint32_t> key;
  DM_ALLOC(ctx, key, size_t(std::max<int64_t>(3 * nP, 1)));
  DM_ALLOC(ctx, ctx->corner_list, size_t(std::max<int64_t>(3 * nP, 1)));
  DM_ALLOC(ctx, ctx->corner_ptr, size_t(nC) + 1);
  if (nP > 0)
    k_corner_keys<<<grid_for(3 * nP, 256), 256, 0, st>>>(ctx->pv.p, ctx->cidx.p, nP, key.p, ctx->corner_list.p);
  DM_LAUNCH_CHECK(ctx);
  DM_TRY(sort_pairs_u32(ctx, key.p, ctx->corner_list.p, size_t(3 * nP), bits_for(uint64_t(nC))));
  k_corner_ptr<<<grid_for(nC + 1, 256), 256, 0, st>>>(key.p, 3 * nP, nC, ctx->corner_ptr.p);
  DM_LAUNCH_CHECK(ctx);
  ctx->corners_ready = true;
  return DM_OK;
}

dm_status cost_offset(dm_ctx* ctx) {
  DM_ALLOC(ctx, ctx->scal, 16);
  DM_TRY(sum_f64(ctx, ctx->cost64.p, ctx->nP, ctx->state.p, SUM_I8_ONE, ctx->scal.p));   // elements fixed to 1
  DM_HIP(ctx, hipMemcpyAsync(&ctx->offset, ctx->scal.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return DM_OK;
}

extern "C" dm_status dm_build_costs(dm_ctx* ctx, const float* FX, const float* FY, int32_t D, int32_t prec,
                                    float* cost) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!ctx->has_space) return dm_fail(ctx, DM_ERR_STATE, "dm_build_costs: no product space");
  if (ctx->generic)
    return dm_fail(ctx, DM_ERR_STATE, "dm_build_costs: descriptor costs need a product space built from meshes");
  if (!FX || !FY || D < 1) return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_build_costs: bad descriptors");
  if (prec != DM_PREC_FP64 && prec != DM_PREC_FP32 && prec != DM_PREC_BF16)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_build_costs: unknown precision %d", prec);
  DM_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  ctx->has_cost = false;
  DM_TRY(mesh_areas(ctx, ctx->X));
  DM_TRY(mesh_areas(ctx, ctx->Y));
  const int32_t nvx = ctx->X.nv, nvy = ctx->Y.nv;
  const int64_t nC = ctx->nC, nP = ctx->nP;
  DArr<double> w;
  DM_ALLOC(ctx, w, size_t(nC));
  DM_ALLOC(ctx, ctx->pair_d, size_t(nC));
  DM_ALLOC(ctx, ctx->pair_a, size_t(nC));
  if (prec == DM_PREC_BF16) {
    DArr<float> d2;
    DM_ALLOC(ctx, d2, size_t(nvx) * nvy);
    DM_TRY(knn_distances(ctx, FX, nvx, FY, nvy, D, DM_PREC_BF16, d2.p));
    k_pair_w_from_d2<<<grid_for(nC, 256), 256, 0, st>>>(ctx->cpair.p, nC, nvy, d2.p, FX, FY, D,
                                                        ctx->X.area.p, ctx->Y.area.p, w.p, ctx->pair_d.p,
                                                        ctx->pair_a.p);
  } else {
    DM_TRY(check_finite(ctx, FX, int64_t(nvx) * D, FY, int64_t(nvy) * D));
    if (prec == DM_PREC_FP64)
      k_pair_w64<<<grid_for(nC, 256), 256, 0, st>>>(ctx->cpair.p, nC, nvy, FX, FY, D, ctx->X.area.p,
                                                    ctx->Y.area.p, w.p, ctx->pair_d.p, ctx->pair_a.p);
    else
      k_pair_w32<<<grid_for(nC, 256), 256, 0, st>>>(ctx->cpair.p, nC, nvy, FX, FY, D, ctx->X.area.p,
                                                    ctx->Y.area.p, w.p, ctx->pair_d.p, ctx->pair_a.p);
  }
  DM_LAUNCH_CHECK(ctx);
  DArr<int> err;
  DM_ALLOC(ctx, err, 1);
  DM_HIP(ctx, hipMemsetAsync(err.p, 0, sizeof(int), st));
  DM_ALLOC(ctx, ctx->cost64, size_t(nP));
  DM_ALLOC(ctx, ctx->cost32, size_t(nP));
  k_elem_cost<<<grid_for(nP, 256), 256, 0, st>>>(ctx->pv.p, ctx->cidx.p, nP, w.p, ctx->cost64.p,
                                                 ctx->cost32.p, cost, err.p);
  DM_LAUNCH_CHECK(ctx);
  // the non-finite flag and the offset of the elements fixed to 1 (FP64,
  // fixed order) come back with one wait
  DM_ALLOC(ctx, ctx->scal, 16);
  DM_TRY(sum_f64(ctx, ctx->cost64.p, ctx->nP, ctx->state.p, SUM_I8_ONE, ctx->scal.p));
  int e = 0;
  double offset = 0.0;
  DM_HIP(ctx, hipMemcpyAsync(&e, err.p, sizeof(int), hipMemcpyDeviceToHost, st));
  DM_HIP(ctx, hipMemcpyAsync(&offset, ctx->scal.p, sizeof(double), hipMemcpyDeviceToHost, st));
  DM_HIP(ctx, hipStreamSynchronize(st));
  if (e) return dm_fail(ctx, DM_ERR_NONFINITE, "non-finite element cost");
  ctx->offset = offset;
  ctx->cost_prec = prec;
  ctx->desc_costs = true;
  ctx->has_cost = true;
  ++ctx->cost_generation;
  return DM_OK;
}
