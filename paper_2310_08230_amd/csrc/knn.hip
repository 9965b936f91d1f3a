// Descriptor distances and candidate pairs.
//
// d(m, n) = ||F_X(m) - F_Y(n)||_2 is the feature distance of Eq. (cost)
// (Sec. 4.2).  Two forms:
//  * BF16: descriptors rounded to BF16 once, squared distances
//    |a|^2 + |b|^2 - 2 a.b with the dot products from a BF16 MFMA GEMM
//    (FP32 accumulation) and the norms of the rounded vectors in FP32, so
//    the result is the distance of the rounded vectors up to FP32 rounding;
//  * FP32: sum of squared differences in FP32 (no cancellation).
// The candidates of a vertex are its K nearest vertices of the other shape,
// ordered by (squared distance, index).
#include <cmath>

#include "dm_internal.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int TOPK_MAX = 4096;

__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return uint16_t(u >> 16);
}

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// one thread per vertex: rounded row (zero padded to Dp) and its FP32 norm
__global__ void k_to_bf16(const float* F, int32_t nv, int32_t D, int32_t nvp, int32_t Dp, uint16_t* out,
                          float* norm) {
  int32_t v = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= nvp) return;
  float s = 0.0f;
  for (int32_t k = 0; k < Dp; ++k) {
    uint16_t h = 0;
    if (v < nv && k < D) h = f32_to_bf16_rne(F[int64_t(v) * D + k]);
    out[int64_t(v) * Dp + k] = h;
    float x = bf16_to_f32(h);
    s = fmaf(x, x, s);
  }
  norm[v] = s;
}

// 64x64 output tile per 256-thread block; each wave owns a 32x32 quarter and
// runs v_mfma_f32_32x32x8bf16_1k over K in steps of 8.  Operand layout of that
// instruction: lane l holds A[l%32][4*(l/32) .. +3] and B[4*(l/32) .. +3][l%32];
// accumulator register r of lane l is C[8*(r/4) + 4*(l/32) + r%4][l%32].
// Both operands are read straight from the row-major [vertex][Dp] arrays (B =
// F_Y^T), 8 bytes per lane per step.
__global__ __launch_bounds__(256) void k_gemm_bf16_dist(const uint16_t* A, const uint16_t* B,
                                                        const float* na, const float* nb, int32_t nva,
                                                        int32_t nvb, int32_t Dp, float* d2) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int32_t m0 = int32_t(blockIdx.y) * 64 + (wave >> 1) * 32;
  const int32_t n0 = int32_t(blockIdx.x) * 64 + (wave & 1) * 32;
  const int row = lane & 31, kg = (lane >> 5) * 4;
  f32x16 acc;
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  // arrays are padded to multiples of 64 rows, so these reads stay in bounds
  const uint16_t* pa = A + int64_t(m0 + row) * Dp + kg;
  const uint16_t* pb = B + int64_t(n0 + row) * Dp + kg;
  for (int32_t k = 0; k < Dp; k += 8) {
    bf16x4 a = *reinterpret_cast<const bf16x4*>(pa + k);
    bf16x4 b = *reinterpret_cast<const bf16x4*>(pb + k);
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
  }
  const int32_t col = n0 + (lane & 31);
  for (int r = 0; r < 16; ++r) {
    int32_t mrow = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (mrow < nva && col < nvb) {
      float v = na[mrow] + nb[col] - 2.0f * acc[r];
      d2[int64_t(mrow) * nvb + col] = v > 0.0f ? v : 0.0f;
    }
  }
}

__global__ void k_dist_fp32(const float* FX, const float* FY, int32_t nvx, int32_t nvy, int32_t D,
                            float* d2) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(nvx) * nvy) return;
  int32_t m = int32_t(i / nvy), n = int32_t(i % nvy);
  const float* a = FX + int64_t(m) * D;
  const float* b = FY + int64_t(n) * D;
  float s = 0.0f;
  for (int32_t k = 0; k < D; ++k) {
    float d = a[k] - b[k];
    s = fmaf(d, d, s);
  }
  d2[i] = s;
}

__global__ void k_nonfinite(const float* a, int64_t n, int* err) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(a[i])) atomicOr(err, 1);
}

// one block per query vertex: bitonic sort of (squared distance, index) keys
// in LDS, first K indices out.  dir 0: rows of d2 (X queries), 1: columns.
__global__ __launch_bounds__(256) void k_topk(const float* d2, int32_t nvx, int32_t nvy, int dir,
                                              int32_t K, int32_t* out) {
  __shared__ uint64_t keys[TOPK_MAX];
  const int32_t q = blockIdx.x;
  const int32_t n = dir == 0 ? nvy : nvx;
  int32_t np2 = 1;
  while (np2 < n) np2 <<= 1;
  for (int32_t i = threadIdx.x; i < np2; i += blockDim.x) {
    uint64_t key = ~uint64_t(0);
    if (i < n) {
      float v = dir == 0 ? d2[int64_t(q) * nvy + i] : d2[int64_t(i) * nvy + q];
      key = (uint64_t(__float_as_uint(v + 0.0f)) << 32) | uint32_t(i);
    }
    keys[i] = key;
  }
  __syncthreads();
  for (int32_t size = 2; size <= np2; size <<= 1) {
    for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (int32_t i = threadIdx.x; i < np2; i += blockDim.x) {
        int32_t j = i ^ stride;
        if (j > i) {
          bool up = (i & size) == 0;
          uint64_t a = keys[i], b = keys[j];
          if ((a > b) == up) {
            keys[i] = b;
            keys[j] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int32_t k = threadIdx.x; k < K; k += blockDim.x) out[int64_t(q) * K + k] = int32_t(keys[k] & 0xFFFFFFFFu);
}

}  // namespace

// both descriptor arrays flag one word, read back once
dm_status check_finite(dm_ctx* ctx, const float* a, int64_t na, const float* b, int64_t nb) {
  DArr<int> err;
  DM_ALLOC(ctx, err, 1);
  DM_HIP(ctx, hipMemsetAsync(err.p, 0, sizeof(int), ctx->stream));
  if (na > 0) k_nonfinite<<<grid_for(na, 256), 256, 0, ctx->stream>>>(a, na, err.p);
  if (nb > 0) k_nonfinite<<<grid_for(nb, 256), 256, 0, ctx->stream>>>(b, nb, err.p);
  DM_LAUNCH_CHECK(ctx);
  int e = 0;
  DM_TRY(read_i32(ctx, err.p, &e));
  if (e) return dm_fail(ctx, DM_ERR_NONFINITE, "non-finite descriptor");
  return DM_OK;
}

dm_status knn_distances(dm_ctx* ctx, const float* FX, int32_t nvx, const float* FY, int32_t nvy,
                        int32_t D, int32_t prec, float* d2) {
  hipStream_t st = ctx->stream;
  DM_TRY(check_finite(ctx, FX, int64_t(nvx) * D, FY, int64_t(nvy) * D));
  if (prec == DM_PREC_BF16) {
    const int32_t Dp = (D + 7) / 8 * 8;
    const int32_t nxp = (nvx + 63) / 64 * 64, nyp = (nvy + 63) / 64 * 64;
    DArr<uint16_t> A, B;
    DArr<float> na, nb;
    DM_ALLOC(ctx, A, size_t(nxp) * Dp);
    DM_ALLOC(ctx, B, size_t(nyp) * Dp);
    DM_ALLOC(ctx, na, size_t(nxp));
    DM_ALLOC(ctx, nb, size_t(nyp));
    k_to_bf16<<<grid_for(nxp, 128), 128, 0, st>>>(FX, nvx, D, nxp, Dp, A.p, na.p);
    k_to_bf16<<<grid_for(nyp, 128), 128, 0, st>>>(FY, nvy, D, nyp, Dp, B.p, nb.p);
    dim3 grid(unsigned(nyp / 64), unsigned(nxp / 64));
    k_gemm_bf16_dist<<<grid, 256, 0, st>>>(A.p, B.p, na.p, nb.p, nvx, nvy, Dp, d2);
    DM_LAUNCH_CHECK(ctx);
    return DM_OK;
  }
  if (prec == DM_PREC_FP32 || prec == DM_PREC_FP64) {
    k_dist_fp32<<<grid_for(int64_t(nvx) * nvy, 256), 256, 0, st>>>(FX, FY, nvx, nvy, D, d2);
    DM_LAUNCH_CHECK(ctx);
    return DM_OK;
  }
  return dm_fail(ctx, DM_ERR_INVALID_ARG, "unknown precision %d", prec);
}

extern "C" dm_status dm_knn_candidates(dm_ctx* ctx, const float* FX, int32_t nvx, const float* FY,
                                       int32_t nvy, int32_t D, int32_t K, int32_t prec, int32_t* cand_xy,
                                       int32_t* cand_yx) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!FX || !FY || !cand_xy || !cand_yx)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_knn_candidates: NULL argument");
  if (nvx < 1 || nvy < 1 || nvx > TOPK_MAX || nvy > TOPK_MAX || D < 1 || K < 1 || K > nvx || K > nvy)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_knn_candidates: nvx=%d nvy=%d D=%d K=%d out of range", nvx,
                   nvy, D, K);
  DM_HIP(ctx, hipSetDevice(ctx->device));
  DArr<float> d2;
  DM_ALLOC(ctx, d2, size_t(nvx) * nvy);
  DM_TRY(knn_distances(ctx, FX, nvx, FY, nvy, D, prec, d2.p));
  k_topk<<<nvx, 256, 0, ctx->stream>>>(d2.p, nvx, nvy, 0, K, cand_xy);
  k_topk<<<nvy, 256, 0, ctx->stream>>>(d2.p, nvx, nvy, 1, K, cand_yx);
  DM_LAUNCH_CHECK(ctx);
  return DM_OK;   // enqueued only; temporaries are freed in stream order
}
