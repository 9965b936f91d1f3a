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
#include <mutex>

#include "dm_internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int TOPK_MAX = 4096;      // keys in the LDS table of one top-K block
constexpr int GEMM_KC = 128;        // K values per LDS stage of the distance GEMM
constexpr int GEMM_LDS_ROW = GEMM_KC + 8;   // bf16 per staged row (16-byte pad)

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
// runs the gfx950 v_mfma_f32_32x32x16_bf16 over K in steps of 16.  Operand
// layout of that instruction: lane l holds A[l%32][8*(l/32) .. +7] and
// B[8*(l/32) .. +7][l%32]; accumulator register r of lane l is
// C[8*(r/4) + 4*(l/32) + r%4][l%32].  The block stages its 64 rows of A and
// 64 rows of B (B = F_Y^T, so rows of F_Y), GEMM_KC values of K at a time, in
// LDS with coalesced 16-byte loads; the waves read their fragments from there
// (row stride padded by 16 bytes, so the 32 rows of a fragment read start in
// different banks).
__global__ __launch_bounds__(256) void k_gemm_bf16_dist(const uint16_t* A, const uint16_t* B,
                                                        const float* na, const float* nb, int32_t nva,
                                                        int32_t nvb, int32_t Dp, float* d2) {
  __shared__ __align__(16) uint16_t As[64 * GEMM_LDS_ROW];
  __shared__ __align__(16) uint16_t Bs[64 * GEMM_LDS_ROW];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int32_t mb = int32_t(blockIdx.y) * 64, nbk = int32_t(blockIdx.x) * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int row = lane & 31, kg = (lane >> 5) * 8;
  f32x16 acc;
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  // arrays are padded to multiples of 64 rows and Dp to a multiple of 16,
  // so every staged load stays in bounds
  for (int32_t k0 = 0; k0 < Dp; k0 += GEMM_KC) {
    const int kc = Dp - k0 < GEMM_KC ? int(Dp - k0) : GEMM_KC;
    const int pieces = kc / 8;   // 16-byte pieces per row
    __syncthreads();             // the previous stage has been read
    for (int idx = threadIdx.x; idx < 64 * pieces; idx += 256) {
      const int r = idx / pieces, c = (idx % pieces) * 8;
      *reinterpret_cast<uint4*>(As + r * GEMM_LDS_ROW + c) =
          *reinterpret_cast<const uint4*>(A + int64_t(mb + r) * Dp + k0 + c);
      *reinterpret_cast<uint4*>(Bs + r * GEMM_LDS_ROW + c) =
          *reinterpret_cast<const uint4*>(B + int64_t(nbk + r) * Dp + k0 + c);
    }
    __syncthreads();
    for (int k = 0; k < kc; k += 16) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(As + (wm + row) * GEMM_LDS_ROW + k + kg);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(Bs + (wn + row) * GEMM_LDS_ROW + k + kg);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
  }
  const int32_t m0 = mb + wm;
  const int32_t col = nbk + wn + (lane & 31);
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

// ascending bitonic sort of np2 keys (a power of two) in LDS by one block
__device__ void bitonic_lds(uint64_t* keys, int32_t np2) {
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
}

// one block per query vertex, K > TOPK_MAX / 2 (then the row has at most
// TOPK_MAX keys): (squared distance, index) keys sorted whole in LDS, first K
// indices out.  dir 0: rows of d2 (X queries), 1: columns.
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
      const float v = dir == 0 ? d2[int64_t(q) * nvy + i] : d2[int64_t(i) * nvy + q];
      key = (uint64_t(__float_as_uint(v + 0.0f)) << 32) | uint32_t(i);
    }
    keys[i] = key;
  }
  __syncthreads();
  bitonic_lds(keys, np2);
  for (int32_t k = threadIdx.x; k < K; k += blockDim.x) out[int64_t(q) * K + k] = int32_t(keys[k] & 0xFFFFFFFFu);
}

// one block per query vertex, K <= TOPK_MAX / 2, any row length: the keys
// (squared distance bits << 32 | index; distances are >= 0, so the bits
// order like the values, and the index makes every key unique) are not
// stored.  A radix selection finds the K-th smallest key digit by digit
// (six digits of 11, 11, 10, 11, 11 and 10 bits, high to low): a histogram
// of the digit over the keys that share the digits found so far, and the
// digit whose cumulative count reaches the rank sought.  The K keys up to
// that one are then gathered and sorted in LDS, so the result is the same
// ordered list as a full sort's first K.
__global__ __launch_bounds__(256) void k_topk_select(const float* d2, int32_t nvx, int32_t nvy, int dir,
                                                     int32_t K, int32_t* out) {
  __shared__ uint32_t hist[2048];
  __shared__ uint32_t part[256];
  __shared__ uint64_t keys[TOPK_MAX / 2];
  __shared__ uint32_t sh_digit, sh_rank, sh_count;
  const int32_t q = blockIdx.x;
  const int32_t n = dir == 0 ? nvy : nvx;
  const int t = threadIdx.x;
  auto key = [&](int32_t i) -> uint64_t {
    const float v = dir == 0 ? d2[int64_t(q) * nvy + i] : d2[int64_t(i) * nvy + q];
    return (uint64_t(__float_as_uint(v + 0.0f)) << 32) | uint32_t(i);
  };
  uint64_t prefix = 0;   // the digits found so far, in place
  int known = 0;         // bits found so far
  uint32_t rank = uint32_t(K);   // 1-based rank sought among the keys with that prefix
  for (int pass = 0; pass < 6; ++pass) {   // uniform across the block
    const int width = pass % 3 == 2 ? 10 : 11;
    const int shift = 64 - known - width;
    const uint32_t mask = (1u << width) - 1u;
    for (int b = t; b < 2048; b += 256) hist[b] = 0u;
    __syncthreads();
    for (int32_t i = t; i < n; i += 256) {
      const uint64_t k = key(i);
      if (known == 0 || (k >> (64 - known)) == (prefix >> (64 - known)))
        atomicAdd(&hist[uint32_t(k >> shift) & mask], 1u);
    }
    __syncthreads();
    // counts of the eight bins of this thread, then an exclusive scan of
    // the 256 partial counts (fixed order, in LDS)
    uint32_t loc = 0;
    for (int j = 0; j < 8; ++j) loc += hist[8 * t + j];
    part[t] = loc;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const uint32_t add = t >= off ? part[t - off] : 0u;
      __syncthreads();
      part[t] += add;
      __syncthreads();
    }
    uint32_t below = part[t] - loc;   // keys in the bins before this thread's
    if (below < rank && rank <= below + loc) {   // exactly one thread
      for (int j = 0; j < 8; ++j) {
        const uint32_t c = hist[8 * t + j];
        if (rank <= below + c) {
          sh_digit = uint32_t(8 * t + j);
          sh_rank = rank - below;
          break;
        }
        below += c;
      }
    }
    __syncthreads();
    prefix |= uint64_t(sh_digit) << shift;
    rank = sh_rank;
    known += width;
    __syncthreads();
  }
  // prefix is now the K-th smallest key: exactly K keys are <= it
  if (t == 0) sh_count = 0u;
  __syncthreads();
  for (int32_t i = t; i < n; i += 256) {
    const uint64_t k = key(i);
    if (k <= prefix) {
      const uint32_t pos = atomicAdd(&sh_count, 1u);
      if (pos < uint32_t(TOPK_MAX / 2)) keys[pos] = k;   // exactly K < TOPK_MAX / 2 + 1 of them
    }
  }
  int32_t np2 = 1;
  while (np2 < K) np2 <<= 1;
  for (int32_t i = K + t; i < np2; i += 256) keys[i] = ~uint64_t(0);
  __syncthreads();
  bitonic_lds(keys, np2);
  for (int32_t k = t; k < K; k += 256) out[int64_t(q) * K + k] = int32_t(keys[k] & 0xFFFFFFFFu);
}

__global__ void k_zero_i32(int* p) { *p = 0; }

// Temporaries of one candidate computation, carved from one block of device
// memory: an error word, the squared distances d2 [nvx*nvy] and, in the BF16
// form, the rounded descriptors padded to 64 rows and 8 columns with their
// norms.  Every piece starts on a 256-byte boundary.
struct KnnBufs {
  int* err = nullptr;
  float* d2 = nullptr;
  uint16_t* A = nullptr;
  uint16_t* B = nullptr;
  float* na = nullptr;
  float* nb = nullptr;
};

inline size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// bytes the temporaries need; with base set, the pieces' addresses in it
size_t knn_layout(int32_t nvx, int32_t nvy, int32_t D, int32_t prec, bool with_d2, unsigned char* base,
                  KnnBufs* out) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align256(bytes);
    return base ? base + at : nullptr;
  };
  KnnBufs b;
  b.err = reinterpret_cast<int*>(take(sizeof(int)));
  if (with_d2) b.d2 = reinterpret_cast<float*>(take(sizeof(float) * size_t(nvx) * size_t(nvy)));
  if (prec == DM_PREC_BF16) {
    const size_t Dp = size_t(D + 15) / 16 * 16;
    const size_t nxp = size_t(nvx + 63) / 64 * 64, nyp = size_t(nvy + 63) / 64 * 64;
    b.A = reinterpret_cast<uint16_t*>(take(sizeof(uint16_t) * nxp * Dp));
    b.B = reinterpret_cast<uint16_t*>(take(sizeof(uint16_t) * nyp * Dp));
    b.na = reinterpret_cast<float*>(take(sizeof(float) * nxp));
    b.nb = reinterpret_cast<float*>(take(sizeof(float) * nyp));
  }
  if (out) *out = b;
  return off;
}

// Scratch of the allocation-free entry point: one array per GPU, alive until
// the process ends.  Host code never passes the array's name to a kernel; it
// uses the device address taken once per device by knn_scratch_init.
constexpr size_t KNN_SCRATCH_BYTES = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[KNN_SCRATCH_BYTES];

constexpr int KNN_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[KNN_MAX_DEVICES] = {};

dm_status check_finite_into(dm_ctx* ctx, const float* a, int64_t na, const float* b, int64_t nb, int* err) {
  k_zero_i32<<<1, 1, 0, ctx->stream>>>(err);
  if (na > 0) k_nonfinite<<<grid_for(na, 256), 256, 0, ctx->stream>>>(a, na, err);
  if (nb > 0) k_nonfinite<<<grid_for(nb, 256), 256, 0, ctx->stream>>>(b, nb, err);
  DM_LAUNCH_CHECK(ctx);
  int e = 0;
  DM_TRY(read_i32(ctx, err, &e));
  if (e) return dm_fail(ctx, DM_ERR_NONFINITE, "non-finite descriptor");
  return DM_OK;
}

dm_status distances_into(dm_ctx* ctx, const float* FX, int32_t nvx, const float* FY, int32_t nvy, int32_t D,
                         int32_t prec, const KnnBufs& w, float* d2) {
  hipStream_t st = ctx->stream;
  DM_TRY(check_finite_into(ctx, FX, int64_t(nvx) * D, FY, int64_t(nvy) * D, w.err));
  if (prec == DM_PREC_BF16) {
    const int32_t Dp = (D + 15) / 16 * 16;
    const int32_t nxp = (nvx + 63) / 64 * 64, nyp = (nvy + 63) / 64 * 64;
    k_to_bf16<<<grid_for(nxp, 128), 128, 0, st>>>(FX, nvx, D, nxp, Dp, w.A, w.na);
    k_to_bf16<<<grid_for(nyp, 128), 128, 0, st>>>(FY, nvy, D, nyp, Dp, w.B, w.nb);
    dim3 grid(unsigned(nyp / 64), unsigned(nxp / 64));
    k_gemm_bf16_dist<<<grid, 256, 0, st>>>(w.A, w.B, w.na, w.nb, nvx, nvy, Dp, d2);
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

dm_status knn_check_args(dm_ctx* ctx, const char* name, const float* FX, int32_t nvx, const float* FY,
                         int32_t nvy, int32_t D, int32_t K, int32_t prec, const int32_t* cand_xy,
                         const int32_t* cand_yx) {
  if (!FX || !FY || !cand_xy || !cand_yx) return dm_fail(ctx, DM_ERR_INVALID_ARG, "%s: NULL argument", name);
  if (nvx < 1 || nvy < 1 || D < 1 || K < 1 || K > nvx || K > nvy ||
      ((nvx > TOPK_MAX || nvy > TOPK_MAX) && K > TOPK_MAX / 2) || nvx > (1 << 21) || nvy > (1 << 21))
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "%s: nvx=%d nvy=%d D=%d K=%d out of range", name, nvx, nvy, D, K);
  if (prec != DM_PREC_BF16 && prec != DM_PREC_FP32 && prec != DM_PREC_FP64)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "%s: unknown precision %d", name, prec);
  return DM_OK;
}

// distances into w.d2, then the K nearest both ways
dm_status knn_run(dm_ctx* ctx, const float* FX, int32_t nvx, const float* FY, int32_t nvy, int32_t D, int32_t K,
                  int32_t prec, int32_t* cand_xy, int32_t* cand_yx, const KnnBufs& w) {
  DM_TRY(distances_into(ctx, FX, nvx, FY, nvy, D, prec, w, w.d2));
  if (K <= TOPK_MAX / 2) {
    k_topk_select<<<nvx, 256, 0, ctx->stream>>>(w.d2, nvx, nvy, 0, K, cand_xy);
    k_topk_select<<<nvy, 256, 0, ctx->stream>>>(w.d2, nvx, nvy, 1, K, cand_yx);
  } else {   // then both sides have at most TOPK_MAX vertices (checked above)
    k_topk<<<nvx, 256, 0, ctx->stream>>>(w.d2, nvx, nvy, 0, K, cand_xy);
    k_topk<<<nvy, 256, 0, ctx->stream>>>(w.d2, nvx, nvy, 1, K, cand_yx);
  }
  DM_LAUNCH_CHECK(ctx);
  return DM_OK;
}

}  // namespace

// device address of this GPU's scratch array, taken once per device with the
// device current (each GPU holds its own copy at its own address)
dm_status knn_scratch_init(dm_ctx* ctx) {
  const int dev = ctx->device;
  if (dev < 0 || dev >= KNN_MAX_DEVICES) return DM_OK;   // the allocation-free entry point refuses such devices
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return DM_OK;
  void* ptr = nullptr;
  DM_HIP(ctx, hipSetDevice(dev));
  DM_HIP(ctx, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) return dm_fail(ctx, DM_ERR_HIP, "no device address for the candidate scratch array");
  g_scratch_ptr[dev] = ptr;
  return DM_OK;
}

// both descriptor arrays flag one word, read back once
dm_status check_finite(dm_ctx* ctx, const float* a, int64_t na, const float* b, int64_t nb) {
  DArr<int> err;
  DM_ALLOC(ctx, err, 1);
  return check_finite_into(ctx, a, na, b, nb, err.p);
}

dm_status knn_distances(dm_ctx* ctx, const float* FX, int32_t nvx, const float* FY, int32_t nvy,
                        int32_t D, int32_t prec, float* d2) {
  // the distances go to the caller's d2: the layout without its d2 piece
  DArr<unsigned char> ws;
  KnnBufs w;
  DM_ALLOC(ctx, ws, knn_layout(nvx, nvy, D, prec, false, nullptr, nullptr));
  knn_layout(nvx, nvy, D, prec, false, ws.p, &w);
  return distances_into(ctx, FX, nvx, FY, nvy, D, prec, w, d2);
}

extern "C" dm_status dm_knn_candidates(dm_ctx* ctx, const float* FX, int32_t nvx, const float* FY,
                                       int32_t nvy, int32_t D, int32_t K, int32_t prec, int32_t* cand_xy,
                                       int32_t* cand_yx) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  DM_TRY(knn_check_args(ctx, "dm_knn_candidates", FX, nvx, FY, nvy, D, K, prec, cand_xy, cand_yx));
  DM_HIP(ctx, hipSetDevice(ctx->device));
  DArr<unsigned char> ws;
  KnnBufs w;
  DM_ALLOC(ctx, ws, knn_layout(nvx, nvy, D, prec, true, nullptr, nullptr));
  knn_layout(nvx, nvy, D, prec, true, ws.p, &w);
  DM_TRY(knn_run(ctx, FX, nvx, FY, nvy, D, K, prec, cand_xy, cand_yx, w));
  return DM_OK;   // the temporaries are freed in stream order
}

extern "C" dm_status dm_knn_candidates_noalloc(dm_ctx* ctx, const float* FX, int32_t nvx, const float* FY,
                                               int32_t nvy, int32_t D, int32_t K, int32_t prec,
                                               int32_t* cand_xy, int32_t* cand_yx) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  DM_TRY(knn_check_args(ctx, "dm_knn_candidates_noalloc", FX, nvx, FY, nvy, D, K, prec, cand_xy, cand_yx));
  const size_t need = knn_layout(nvx, nvy, D, prec, true, nullptr, nullptr);
  if (need > KNN_SCRATCH_BYTES)
    return dm_fail(ctx, DM_ERR_WORKSPACE,
                   "dm_knn_candidates_noalloc: needs %zu bytes of scratch, the limit is %zu (nvx=%d nvy=%d D=%d)",
                   need, KNN_SCRATCH_BYTES, nvx, nvy, D);
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < KNN_MAX_DEVICES) base = g_scratch_ptr[ctx->device];
  }
  if (!base) return dm_fail(ctx, DM_ERR_STATE, "dm_knn_candidates_noalloc: no scratch address for device %d",
                            ctx->device);
  DM_HIP(ctx, hipSetDevice(ctx->device));
  KnnBufs w;
  knn_layout(nvx, nvy, D, prec, true, static_cast<unsigned char*>(base), &w);
  return knn_run(ctx, FX, nvx, FY, nvy, D, K, prec, cand_xy, cand_yx, w);
}
