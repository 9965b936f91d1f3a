// Context lifetime, errors, library primitives (sort, scan) and exports.
#include <cstring>

#include <rocprim/rocprim.hpp>

#include <cstdarg>
#include <vector>

#include "dm_internal.h"

dm_status dm_fail(dm_ctx* ctx, dm_status code, const char* fmt, ...) {
  if (ctx) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

extern "C" dm_status dm_create(int32_t device, void* hip_stream, dm_ctx** out) {
  if (!out) return DM_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DM_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return DM_ERR_HIP;
  // the context's own memory pool: it keeps the blocks the library frees for
  // reuse (the build steps' temporaries come and go per call) until
  // dm_destroy, and leaves the device's default pool as it was
  hipMemPoolProps props;
  std::memset(&props, 0, sizeof(props));
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = device;
  hipMemPool_t pool = nullptr;
  if (hipMemPoolCreate(&pool, &props) != hipSuccess || !pool) return DM_ERR_HIP;
  uint64_t keep = UINT64_MAX;
  (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  dm_ctx* c = new dm_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->pool = pool;
  c->cache.stream = c->stream;
  // pinned landing slots for small device-to-host reads
  if (hipHostMalloc(reinterpret_cast<void**>(&c->host_i32), HOST_SLOTS * sizeof(int32_t), hipHostMallocDefault) !=
      hipSuccess) {
    delete c;
    (void)hipMemPoolDestroy(pool);
    return DM_ERR_HIP;
  }
  // device address of the allocation-free entry point's scratch array
  if (knn_scratch_init(c) != DM_OK) {
    (void)hipHostFree(c->host_i32);
    delete c;
    (void)hipMemPoolDestroy(pool);
    return DM_ERR_HIP;
  }
  *out = c;
  return DM_OK;
}

extern "C" dm_status dm_destroy(dm_ctx* ctx) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->host_i32) (void)hipHostFree(ctx->host_i32);
  hipMemPool_t pool = ctx->pool;
  hipStream_t st = ctx->stream;
  delete ctx;   // frees every owned array and cached block on the stream
  (void)hipStreamSynchronize(st);
  if (pool) (void)hipMemPoolDestroy(pool);
  return DM_OK;
}

extern "C" const char* dm_last_error(const dm_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

extern "C" dm_status dm_set_stream(dm_ctx* ctx, void* hip_stream) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // the context's buffers are ordered on its stream: finish the old stream's
  // work before later calls order work (and frees) on the new one
  if (s != ctx->stream) {
    DM_HIP(ctx, hipSetDevice(ctx->device));
    DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->cache.release_all();   // cached blocks were last used on the old stream
  }
  ctx->stream = s;
  ctx->cache.stream = s;
  return DM_OK;
}

extern "C" const char* dm_version(void) { return "discomatch-gfx950 0.1"; }

// ---------------------------------------------------------------------------
// rocPRIM wrappers (stable radix sort of key/value pairs, exclusive scans)
// ---------------------------------------------------------------------------
// Every sort above one block takes the onesweep (LSD radix) algorithm, whose
// passes follow the key bits actually used; rocPRIM's default sends sizes up
// to 2^20 to a block sort plus merge rounds, whose count grows with the size
// instead (the 64-bit edge-key sort of a 500-face pair: 16 merge kernels).
// Both are stable, so the sorted order is the same.  The double-buffer form
// ping-pongs between the caller's arrays and one pair of temporaries, so the
// result needs copying back only when it ends in the temporaries.
using SortConfig = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                              rocprim::default_config, 0>;

template <typename K>
static dm_status sort_pairs_impl(dm_ctx* ctx, K* keys, int32_t* vals, size_t n, int end_bit) {
  if (n <= 1) return DM_OK;
  DArr<K> k2;
  DArr<int32_t> v2;
  DM_ALLOC(ctx, k2, n);
  DM_ALLOC(ctx, v2, n);
  rocprim::double_buffer<K> kb(keys, k2.p);
  rocprim::double_buffer<int32_t> vb(vals, v2.p);
  size_t temp = 0;
  DM_HIP(ctx, rocprim::radix_sort_pairs<SortConfig>(nullptr, temp, kb, vb, n, 0u, unsigned(end_bit), ctx->stream));
  DArr<unsigned char> tmp;
  DM_ALLOC(ctx, tmp, temp + 16);
  DM_HIP(ctx, rocprim::radix_sort_pairs<SortConfig>(tmp.p, temp, kb, vb, n, 0u, unsigned(end_bit), ctx->stream));
  if (kb.current() != keys)
    DM_HIP(ctx, hipMemcpyAsync(keys, kb.current(), n * sizeof(K), hipMemcpyDeviceToDevice, ctx->stream));
  if (vb.current() != vals)
    DM_HIP(ctx, hipMemcpyAsync(vals, vb.current(), n * sizeof(int32_t), hipMemcpyDeviceToDevice, ctx->stream));
  return DM_OK;   // temporaries are freed in stream order: no wait needed
}

dm_status sort_pairs_u64(dm_ctx* ctx, uint64_t* keys, int32_t* vals, size_t n, int end_bit) {
  return sort_pairs_impl<uint64_t>(ctx, keys, vals, n, end_bit);
}

dm_status sort_pairs_u32(dm_ctx* ctx, uint32_t* keys, int32_t* vals, size_t n, int end_bit) {
  return sort_pairs_impl<uint32_t>(ctx, keys, vals, n, end_bit);
}

// ---------------------------------------------------------------------------
// deterministic FP64 sums
// ---------------------------------------------------------------------------
constexpr int SUM_MAX_BLOCKS = 1024;

__global__ __launch_bounds__(256) void k_sum_ranges(const double* a, int64_t n, const void* sel, int kind,
                                                    int64_t per_block, double* partial) {
  __shared__ double red[4];
  const int64_t lo = int64_t(blockIdx.x) * per_block;
  const int64_t hi = lo + per_block < n ? lo + per_block : n;
  // eight independent accumulators per thread (fixed order)
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256 * 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t q = i + 256 * u;
      if (q >= hi) continue;
      const bool take = kind == SUM_ALL ? true
                        : kind == SUM_I8_ONE ? static_cast<const int8_t*>(sel)[q] == 1
                                             : static_cast<const uint8_t*>(sel)[q] != 0;
      if (take) acc[u] += a[q];
    }
  }
  const double v = ((((((acc[0] + acc[1]) + acc[2]) + acc[3]) + acc[4]) + acc[5]) + acc[6]) + acc[7];
  const double part = block_sum_256(v, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = part;
}

__global__ __launch_bounds__(1024) void k_sum_partials(const double* partial, int n, double* out) {
  __shared__ double red[16];
  const double r = sum_partials_1024(partial, n, red);
  if (threadIdx.x == 0) *out = r;
}

dm_status sum_f64(dm_ctx* ctx, const double* a, int64_t n, const void* sel, int kind, double* out) {
  const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(SUM_MAX_BLOCKS, (n + 4095) / 4096));
  const int64_t per_block = (n + nb - 1) / nb;
  DM_ALLOC(ctx, ctx->sum_part, size_t(SUM_MAX_BLOCKS));
  k_sum_ranges<<<unsigned(nb), 256, 0, ctx->stream>>>(a, n, sel, kind, per_block, ctx->sum_part.p);
  k_sum_partials<<<1, 1024, 0, ctx->stream>>>(ctx->sum_part.p, int(nb), out);
  DM_LAUNCH_CHECK(ctx);
  return DM_OK;
}

__global__ void k_scan_tail(const int32_t* in_last, int32_t* out, size_t n, int is_u8,
                            const uint8_t* u8_last) {
  int32_t last = is_u8 ? int32_t(*u8_last) : *in_last;
  out[n] = out[n - 1] + last;
}

struct U8ToI32 {
  __host__ __device__ int32_t operator()(uint8_t v) const { return int32_t(v); }
};

dm_status scan_i32(dm_ctx* ctx, const int32_t* in, int32_t* out, size_t n) {
  if (n == 0) {
    DM_HIP(ctx, hipMemsetAsync(out, 0, sizeof(int32_t), ctx->stream));
    return DM_OK;
  }
  size_t temp = 0;
  DM_HIP(ctx, rocprim::exclusive_scan(nullptr, temp, in, out, int32_t(0), n,
                                      rocprim::plus<int32_t>(), ctx->stream));
  DArr<unsigned char> tmp;
  DM_ALLOC(ctx, tmp, temp + 16);
  DM_HIP(ctx, rocprim::exclusive_scan(tmp.p, temp, in, out, int32_t(0), n,
                                      rocprim::plus<int32_t>(), ctx->stream));
  k_scan_tail<<<1, 1, 0, ctx->stream>>>(in + n - 1, out, n, 0, nullptr);
  DM_LAUNCH_CHECK(ctx);
  return DM_OK;
}

dm_status scan_u8(dm_ctx* ctx, const uint8_t* in, int32_t* out, size_t n) {
  if (n == 0) {
    DM_HIP(ctx, hipMemsetAsync(out, 0, sizeof(int32_t), ctx->stream));
    return DM_OK;
  }
  auto it = rocprim::make_transform_iterator(in, U8ToI32());
  size_t temp = 0;
  DM_HIP(ctx, rocprim::exclusive_scan(nullptr, temp, it, out, int32_t(0), n,
                                      rocprim::plus<int32_t>(), ctx->stream));
  DArr<unsigned char> tmp;
  DM_ALLOC(ctx, tmp, temp + 16);
  DM_HIP(ctx, rocprim::exclusive_scan(tmp.p, temp, it, out, int32_t(0), n,
                                      rocprim::plus<int32_t>(), ctx->stream));
  k_scan_tail<<<1, 1, 0, ctx->stream>>>(nullptr, out, n, 1, in + n - 1);
  DM_LAUNCH_CHECK(ctx);
  return DM_OK;
}

dm_status read_i32(dm_ctx* ctx, const int32_t* dev, int32_t* host) {
  return read_i32s(ctx, 1, &dev, host);
}

dm_status read_i32s(dm_ctx* ctx, int n, const int32_t* const* dev, int32_t* host) {
  if (n < 0 || n > HOST_SLOTS) return dm_fail(ctx, DM_ERR_STATE, "read_i32s: %d values (at most %d)", n, HOST_SLOTS);
  for (int i = 0; i < n; ++i)
    DM_HIP(ctx, hipMemcpyAsync(ctx->host_i32 + i, dev[i], sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < n; ++i) host[i] = ctx->host_i32[i];
  return DM_OK;
}

// ---------------------------------------------------------------------------
// exports
// ---------------------------------------------------------------------------
template <typename S, typename D>
__global__ void k_widen(const S* in, D* out, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = D(in[i]);
}

__global__ void k_export_code(const int32_t* code, int32_t* out, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = code[i];
}

template <typename S, typename D>
static dm_status widen(dm_ctx* ctx, const S* in, void* out, int64_t n) {
  if (n <= 0) return DM_OK;   // an empty array: dst may be NULL
  if (!out) return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_get_space: dst is NULL");
  k_widen<S, D><<<grid_for(n, 256), 256, 0, ctx->stream>>>(in, static_cast<D*>(out), n);
  DM_LAUNCH_CHECK(ctx);
  return DM_OK;
}

extern "C" dm_status dm_get_space(dm_ctx* ctx, int32_t which, void* dst) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  if (!ctx->has_space) return dm_fail(ctx, DM_ERR_STATE, "dm_get_space: no product space built");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  if (ctx->generic && (which == DM_ARR_PV || which == DM_ARR_CODE || which == DM_ARR_EDGES_X || which == DM_ARR_EDGES_Y || which == DM_ARR_CAND))
    return dm_fail(ctx, DM_ERR_STATE, "dm_get_space: a problem from dm_build_ilp has no meshes or candidates");
  switch (which) {
    case DM_ARR_PV: return widen<int32_t, int32_t>(ctx, ctx->pv.p, dst, ctx->nP * 3);
    case DM_ARR_CODE: return widen<int32_t, int32_t>(ctx, ctx->code.p, dst, ctx->nP * 4);
    case DM_ARR_STATE: return widen<int8_t, int8_t>(ctx, ctx->state.p, dst, ctx->nP);
    case DM_ARR_ROW_KEY: return widen<int64_t, int64_t>(ctx, ctx->row_key.p, dst, ctx->n_rows_full);
    case DM_ARR_ROW_PTR: return widen<int32_t, int64_t>(ctx, ctx->row_ptr.p, dst, ctx->n_rows_full + 1);
    case DM_ARR_ENT_VAR: return widen<int32_t, int64_t>(ctx, ctx->ent_var.p, dst, ctx->nnz_full);
    case DM_ARR_ENT_COEF: return widen<int8_t, int32_t>(ctx, ctx->ent_coef.p, dst, ctx->nnz_full);
    case DM_ARR_ROW_B: return widen<int32_t, int32_t>(ctx, ctx->row_b.p, dst, ctx->n_rows_full);
    case DM_ARR_FREE_VAR: return widen<int32_t, int64_t>(ctx, ctx->free_var.p, dst, ctx->n_free);
    case DM_ARR_RROW_ORIG: return widen<int32_t, int64_t>(ctx, ctx->rrow_orig.p, dst, ctx->n_rows);
    case DM_ARR_RROW_PTR: return widen<int32_t, int64_t>(ctx, ctx->rrow_ptr.p, dst, ctx->n_rows + 1);
    case DM_ARR_RENT_VAR: return widen<int32_t, int64_t>(ctx, ctx->rent_var.p, dst, ctx->nnz);
    case DM_ARR_RENT_COEF: return widen<int8_t, int32_t>(ctx, ctx->rent_coef.p, dst, ctx->nnz);
    case DM_ARR_RROW_B: return widen<int32_t, int32_t>(ctx, ctx->rrow_b.p, dst, ctx->n_rows);
    case DM_ARR_EDGES_X: return widen<int32_t, int32_t>(ctx, ctx->X.edges.p, dst, int64_t(ctx->X.ne) * 2);
    case DM_ARR_EDGES_Y: return widen<int32_t, int32_t>(ctx, ctx->Y.edges.p, dst, int64_t(ctx->Y.ne) * 2);
    case DM_ARR_CAND:
      return widen<uint8_t, uint8_t>(ctx, ctx->cand.p, dst, int64_t(ctx->X.nv) * ctx->Y.nv);
  }
  return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_get_space: unknown array %d", which);
}
