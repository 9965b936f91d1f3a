// Internal declarations of the DiscoMatch gfx950 library: the context, device
// buffers and the entry points of each translation unit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/discomatch.h"

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
dm_status dm_fail(dm_ctx* ctx, dm_status code, const char* fmt, ...);

#define DM_HIP(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return dm_fail((ctx), DM_ERR_HIP, "%s:%d %s: %s", __FILE__, __LINE__, #call,     \
                     hipGetErrorString(e_));                                           \
  } while (0)

#define DM_TRY(expr)                  \
  do {                                \
    dm_status s_ = (expr);            \
    if (s_ != DM_OK) return s_;       \
  } while (0)

#define DM_LAUNCH_CHECK(ctx) DM_HIP(ctx, hipGetLastError())

// ---------------------------------------------------------------------------
// Blocks a context has freed, kept for its later allocations.  Returning a
// block to a stream-ordered pool costs the host about 12 us per
// hipFreeAsync (more for large blocks), and a product-space build frees
// about ninety temporaries, so a context keeps them here by size class
// (bytes rounded up to 256) and an allocation of the same class takes one
// back without a runtime call.  Every block is used on the context's
// stream, so stream order alone makes the reuse safe: a block is taken only
// by work ordered after everything that used it before.  The cache holds at
// most MAX_BYTES; blocks beyond that, and every block when the context's
// stream changes, when an allocation finds the pool out of memory, or when
// the context is destroyed, go back to the pool.
// ---------------------------------------------------------------------------
struct BlockCache {
  static constexpr size_t MAX_BYTES = size_t(4) << 30;
  std::multimap<size_t, void*> blocks;
  size_t bytes = 0;
  hipStream_t stream = nullptr;   // the stream every cached block was last used on
  static size_t size_class(size_t b) { return (b + 255) / 256 * 256; }
  void* take(size_t cls) {
    auto it = blocks.find(cls);
    if (it == blocks.end()) return nullptr;
    void* q = it->second;
    blocks.erase(it);
    bytes -= cls;
    return q;
  }
  bool keep(void* q, size_t cls) {
    if (bytes + cls > MAX_BYTES) return false;
    blocks.emplace(cls, q);
    bytes += cls;
    return true;
  }
  void release_all() {
    for (auto& kv : blocks) (void)hipFreeAsync(kv.second, stream);
    blocks.clear();
    bytes = 0;
  }
  ~BlockCache() { release_all(); }
};

// ---------------------------------------------------------------------------
// device array.  An owned array is allocated stream-ordered on the context's
// stream from the context's own memory pool (hipMallocFromPoolAsync) or from
// the context's block cache, and given back to the cache (or, past its
// limit, freed with hipFreeAsync), so the temporaries of the build steps cost
// no device-wide synchronisation and no other user of the device's default
// pool is affected.  A block freed on a stream is reused only by work
// ordered after the free on that stream.  A view (attach) borrows caller
// memory and never frees it.
// ---------------------------------------------------------------------------
template <typename T>
struct DArr {
  T* p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;   // stream the block was allocated on
  bool view = false;         // borrowed memory: never freed here
  BlockCache* cache = nullptr;   // where the block goes back to, or NULL
  size_t cls = 0;                // its size class in bytes
  DArr() = default;
  DArr(const DArr&) = delete;
  DArr& operator=(const DArr&) = delete;
  ~DArr() { release(); }
  void release() {
    if (p && !view && !(cache && cache->stream == s && cache->keep(p, cls))) (void)hipFreeAsync(p, s);
    p = nullptr;
    n = 0;
    view = false;
    cache = nullptr;
    cls = 0;
  }
  hipError_t resize(size_t count, hipStream_t stream, hipMemPool_t pool, BlockCache* bc = nullptr) {
    if (count == n && p && !view) return hipSuccess;
    release();
    if (count == 0) return hipSuccess;
    const size_t c = BlockCache::size_class(count * sizeof(T));
    void* q = (bc && bc->stream == stream) ? bc->take(c) : nullptr;
    if (!q) {
      hipError_t e = hipMallocFromPoolAsync(&q, c, pool, stream);
      if (e != hipSuccess && bc && bc->bytes > 0) {
        // out of memory while the cache holds idle blocks: give them back
        // to the pool (stream-ordered, so the retry on the same stream may
        // reuse them) and try once more
        (void)hipGetLastError();
        bc->release_all();
        e = hipMallocFromPoolAsync(&q, c, pool, stream);
        if (e == hipSuccess) (void)hipGetLastError();
      }
      if (e != hipSuccess) return e;
    }
    p = static_cast<T*>(q);
    n = count;
    s = stream;
    cache = bc;
    cls = c;
    return hipSuccess;
  }
  void attach(T* ptr, size_t count) {
    release();
    p = ptr;
    n = count;
    view = true;
  }
};

#define DM_ALLOC(ctx, arr, count) DM_HIP(ctx, (arr).resize(count, (ctx)->stream, (ctx)->pool, &(ctx)->cache))

struct MeshDev {
  int32_t nv = 0, nf = 0, ne = 0;
  DArr<float> verts;       // nv*3
  DArr<int32_t> faces;     // nf*3
  DArr<int32_t> edges;     // ne*2 sorted (min, max)
  DArr<int32_t> face_edge; // nf*3: id of edge (f[k], f[k+1])
  DArr<uint64_t> dkey;     // 3*nf sorted directed-edge keys a*nv+b
  DArr<int32_t> dval;      // 3*nf corner id 3f+k of each sorted key
  DArr<double> area;       // nv mixed areas (filled by costs)
};

// Reduced-problem entry word: [31] coefficient is -1, [30] unused, [29:27]
// slot of the entry in its variable's record, [26:0] variable.
constexpr uint32_t W_NEG = 1u << 31;
constexpr int W_SLOT_SHIFT = 27;
constexpr uint32_t W_VAR_MASK = (1u << 27) - 1u;
constexpr int REC = 8;          // record stride: 5 multiplier slots, cost, 1 / degree, 1 spare
constexpr int REC_COST = 5;
constexpr int REC_RDEG = 6;
constexpr int MAX_SHORT_ROW = 64;
constexpr int SOFT_MAX_ROW = 24;
constexpr uint32_t CHUNK_PAD = 0xFFFFFFFFu;   // entry word of an unused chunk slot

// Multipliers of free variable i from its record (slots 0-4 hold s_k, slot 5
// the cost c_i, slot 6 the reciprocal 1/|J_i| of the number of rows the
// variable lies in, 1 to 5, rounded to the record's precision), with dual
// feasibility restored: lambda_k = s_k + (c_i - sum_k s_k) * (1/|J_i|).  The
// product by the stored reciprocal replaces a division on every record read.
// Slots at or above |J_i| hold zero and are never written, so the sum runs
// over all five.  Every reader of a record (the row sweeps and the
// per-variable passes) goes through this one function or its batched copy in
// the row tiles, so they all see bit-identical multipliers.
template <typename R>
__device__ inline void rec_lambdas(const R* __restrict__ rec, size_t i, R lam[5]) {
  const R* r = rec + i * REC;
  R s0, s1, s2, s3, s4, c, rd;
  if constexpr (sizeof(R) == 4) {
    // records are 32-byte aligned: two 16-byte loads of one 32-byte sector
    const float4 lo = *reinterpret_cast<const float4*>(r);
    const float4 hi = *reinterpret_cast<const float4*>(r + 4);
    s0 = lo.x, s1 = lo.y, s2 = lo.z, s3 = lo.w, s4 = hi.x, c = hi.y, rd = hi.z;
  } else {
    const double2 a = *reinterpret_cast<const double2*>(r);
    const double2 b = *reinterpret_cast<const double2*>(r + 2);
    const double2 e = *reinterpret_cast<const double2*>(r + 4);
    const double2 f = *reinterpret_cast<const double2*>(r + 6);
    s0 = a.x, s1 = a.y, s2 = b.x, s3 = b.y, s4 = e.x, c = e.y, rd = f.x;
  }
  const R sum = (((s0 + s1) + s2) + s3) + s4;
  const R corr = (c - sum) * rd;
  lam[0] = s0 + corr;
  lam[1] = s1 + corr;
  lam[2] = s2 + corr;
  lam[3] = s3 + corr;
  lam[4] = s4 + corr;
}

// FP64 sum of a 256-thread block in a fixed order: an xor butterfly inside
// each wave (every lane ends with the same value, since a + b == b + a
// exactly), then the four wave sums in index order.  red: 4 doubles of LDS.
__device__ inline double block_sum_256(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  return r;
}

// Sum of n per-block partials by a 256-thread block, in a fixed order (the
// same value in every block that calls it).  Thread t takes elements
// t + 256 k into eight independent accumulators (k mod 8), so its loads do
// not wait on each other.
__device__ inline double sum_partials_256(const double* p, int n, double* red) {
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = int(threadIdx.x); i < n; i += 256 * 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i + 256 * u < n) a[u] += p[i + 256 * u];
  }
  const double v = ((((((a[0] + a[1]) + a[2]) + a[3]) + a[4]) + a[5]) + a[6]) + a[7];
  return block_sum_256(v, red);
}

// The same for one 1024-thread block (sixteen waves): for the one-block
// kernels that sum the partials of a whole sweep launch.  red: 16 doubles.
__device__ inline double sum_partials_1024(const double* p, int n, double* red) {
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = int(threadIdx.x); i < n; i += 1024 * 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i + 1024 * u < n) a[u] += p[i + 1024 * u];
  }
  double v = ((((((a[0] + a[1]) + a[2]) + a[3]) + a[4]) + a[5]) + a[6]) + a[7];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < 16; ++w) r += red[w];
  __syncthreads();
  return r;
}

constexpr int HOST_SLOTS = 16;

struct dm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipMemPool_t pool = nullptr;   // the context's own pool (every DArr allocation)
  BlockCache cache;              // declared before every array: destroyed after them
  std::string err;
  // caller-owned solver workspace per message precision (0 FP32, 1 FP64),
  // see dm_set_workspace; NULL when the library allocates the state itself
  void* ws_ptr[2] = {nullptr, nullptr};
  size_t ws_bytes[2] = {0, 0};

  MeshDev X, Y;
  int32_t K = 0;
  bool has_space = false;

  // candidates: byte map and compact pair list (sorted by product vertex id)
  DArr<uint8_t> cand;      // nvx*nvy
  DArr<int32_t> cidx;      // nvx*nvy -> pair index or -1
  DArr<int32_t> cpair;     // nC -> m*nvy+n
  DArr<int32_t> cpair_t;   // pairs sorted by (n, m): pair indices
  DArr<int32_t> cand_xstart; // nvx+1: first pair of each X vertex
  DArr<int32_t> cand_ystart; // nvy+1: first position in cpair_t of each Y vertex
  int64_t nC = 0;

  // elements (product triangles) in canonical order
  int64_t nP = 0;
  DArr<int32_t> pv;        // nP*3
  DArr<int32_t> code;      // nP*4 (x class, x id, y class*8+pattern, y id)
  DArr<uint8_t> elem_deg;  // nP: rows each element lies in (1 to 5)

  // full incidence A (rows: closedness | X projection | Y projection)
  int64_t n_rows_full = 0, n_closed_full = 0, nnz_full = 0;
  DArr<int64_t> row_key;
  DArr<int32_t> row_ptr;   // n_rows_full+1
  DArr<int32_t> ent_var;
  DArr<int8_t> ent_coef;
  DArr<uint8_t> ent_slot;
  DArr<int32_t> row_b;
  DArr<int8_t> state;      // -1 free, 0/1 fixed
  int32_t presolve_rounds = 0;

  // reduced problem over free variables
  int64_t n_free = 0, n_fixed1 = 0, n_rows = 0, nnz = 0, n_short = 0, nnz_short = 0;
  int32_t max_short = 0;
  DArr<int32_t> free_var;  // n_free -> element
  DArr<int32_t> var_red;   // nP -> reduced var or -1
  DArr<int32_t> rrow_orig;
  DArr<int32_t> rrow_ptr;  // n_rows+1
  DArr<int32_t> rrow_b;
  DArr<int32_t> rent_var;
  DArr<int8_t> rent_coef;
  DArr<uint32_t> rent_word;
  DArr<uint8_t> var_deg;   // n_free: rows of each free variable (1 to 5)
  int32_t n_chunks = 0;
  DArr<int4> chunk_desc;   // n_chunks wave chunks: (first row, rows, first entry, entries)
  DArr<unsigned long long> chunk_mask;  // per chunk: bit e set when entry e starts a row
  DArr<uint32_t> chunk_word;  // 64 per chunk: the chunk's entry words, CHUNK_PAD past its end
  DArr<int8_t> chunk_b;       // 64 per chunk: right-hand side of each entry's row
  // launch layout of the hard sweep (layout.hip): short rows are packed into
  // the chunks in region/key order; projection rows run in long_perm order;
  // block b takes item xcd_item[(b % 8) * xcd_stride + b / 8] (-1: none)
  int32_t long_wpr = 1;       // waves per projection row: 1 or 4 (4 rows or 1 row per block)
  int32_t n_long_items = 0;   // projection-row blocks
  int32_t xcd_stride = 0;
  int32_t n_tiles = 0;        // 64-row tiles of short rows with b = 0 (one lane per row)
  int32_t n_tile_items = 0;   // blocks of four tiles
  DArr<uint32_t> tile_word;   // per tile 16 x 64 entry words: 8 slots of +1 entries, 8 of -1 entries
  DArr<int32_t> long_perm;    // n_rows - n_short: projection rows (relative to n_short) in launch order
  DArr<int32_t> xcd_item;     // 8 * xcd_stride
  DArr<int32_t> soft_row;     // short rows sorted (stably) by length, for the smoothed sweep
  int64_t soft_c8 = 0, soft_c16 = 0;   // how many of them have <= 7 / 8..15 entries

  // costs
  bool has_cost = false;
  int32_t cost_prec = DM_PREC_FP32;
  double offset = 0.0;
  DArr<double> cost64;     // nP (FP64 copy of the element costs)
  DArr<float> cost32;      // nP
  DArr<float> pair_d;      // nC descriptor distance used by the costs
  DArr<float> pair_a;      // nC A_X(m) + A_Y(n)
  DArr<int32_t> corner_ptr;  // nC+1: corners (3p+v) of each pair
  DArr<int32_t> corner_list; // 3*nP

  // solver state (byte buffers reused for FP32 / FP64)
  DArr<unsigned char> rec[2];    // records n_free * REC * sizeof(real)
  DArr<unsigned char> rrec[2];   // rounding copy
  DArr<unsigned char> mrec;      // min-marginals / marginals per slot
  DArr<double> partial;          // per-block partial sums, two alternating halves
  int pend_half = 0;             // half written by the last sweep launch
  double* pend_partial = nullptr;
  int32_t pend_n = 0;
  double pend_offset = 0.0;
  double* pend_out = nullptr;    // bound of the last launch not yet summed
  DArr<double> scal;             // small device scalars
  DArr<double> sum_part;         // per-block partials of sum_f64
  bool corners_ready = false;    // corner_ptr / corner_list match the product space
  bool generic = false;          // the problem came from dm_build_ilp (no meshes, no candidates)
  bool desc_costs = false;       // the costs came from descriptors (dm_build_costs)
  int32_t* host_i32 = nullptr;   // HOST_SLOTS pinned ints: landing slots of read_i32s
  DArr<int8_t> pref;             // per variable: 1, 0 or -1
  DArr<int64_t> icount;          // integer counters
  DArr<float> gw;                // gradient per pair
  DArr<float> gcost_tmp;         // gradient per element

  // optional per-launch event timing of the sweep kernel
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;

  // quasi-Newton session kept between dm_lbfgs_solve calls (history, step
  // size, Delta_min), owned by lbfgs.hip; invalidated when the costs or the
  // fixed variables change (cost_generation counts those changes)
  void* qn = nullptr;
  void (*qn_free)(void*) = nullptr;
  int64_t cost_generation = 0;

  ~dm_ctx() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    if (qn && qn_free) qn_free(qn);
  }
};

// translation-unit entry points ------------------------------------------------
dm_status mesh_ingest(dm_ctx* ctx, const dm_mesh* in, MeshDev& m, const char* name);
dm_status mesh_areas(dm_ctx* ctx, MeshDev& m);
dm_status space_build(dm_ctx* ctx, const int32_t* cand_xy, const int32_t* cand_yx, int32_t K);
dm_status knn_distances(dm_ctx* ctx, const float* FX, int32_t nvx, const float* FY, int32_t nvy,
                        int32_t D, int32_t prec, float* d2 /* nvx*nvy */);
dm_status sort_pairs_u64(dm_ctx* ctx, uint64_t* keys, int32_t* vals, size_t n, int end_bit);
dm_status sort_pairs_u32(dm_ctx* ctx, uint32_t* keys, int32_t* vals, size_t n, int end_bit);
dm_status scan_i32(dm_ctx* ctx, const int32_t* in, int32_t* out, size_t n);  // exclusive, out[n] = total
dm_status scan_u8(dm_ctx* ctx, const uint8_t* in, int32_t* out, size_t n);   // exclusive, out[n] = total
// Deterministic FP64 sum of a[0..n) into *out (device), in an order fixed by
// n: blocks sum contiguous ranges, one block sums their partials.  sel
// (optional) picks the terms: SUM_I8_ONE takes a[i] where ((int8*)sel)[i] == 1,
// SUM_U8_NZ where ((uint8*)sel)[i] != 0.
enum SumSel { SUM_ALL = 0, SUM_I8_ONE = 1, SUM_U8_NZ = 2 };
dm_status sum_f64(dm_ctx* ctx, const double* a, int64_t n, const void* sel, int kind, double* out);
dm_status read_i32(dm_ctx* ctx, const int32_t* dev, int32_t* host);
// n (<= HOST_SLOTS) device ints into host[0..n) with one wait for the stream
dm_status read_i32s(dm_ctx* ctx, int n, const int32_t* const* dev, int32_t* host);
dm_status check_finite(dm_ctx* ctx, const float* a, int64_t na, const float* b, int64_t nb);
// takes this device's address of the scratch array of dm_knn_candidates_noalloc (once per device)
dm_status knn_scratch_init(dm_ctx* ctx);
dm_status dual_flush(dm_ctx* ctx);  // write the bound of the last sweep launch
// layout of the Jacobi solver's state in a caller workspace: two record
// buffers, then the sweep partials; sizes for the current problem
struct SolverLayout {
  size_t rec_bytes, part_off, part_count, total;
};
SolverLayout solver_layout(const dm_ctx* ctx, size_t real_bytes);
dm_status cost_offset(dm_ctx* ctx);   // offset = summed costs of elements fixed to 1 (synchronises)
dm_status corner_lists(dm_ctx* ctx);  // corners per candidate pair (built once per product space)
void fill_info(dm_ctx* ctx, dm_space_info* info);   // sizes of the current (reduced) problem
dm_status presolve_reduce(dm_ctx* ctx, const int8_t* fix);  // presolve from fixings, reduced problem
dm_status sweep_layout(dm_ctx* ctx);   // chunks, projection-row order and per-XCD items of the hard sweep

// One sweep over all rows of the presolved problem (dual.hip).  Modes: update
// the multipliers (rin -> out), write min-marginals (or soft marginals) per
// slot to out, bound only, or write each row's minimising assignment.
enum SweepMode { SWEEP_UPDATE = 0, SWEEP_EVAL = 1, SWEEP_BOUND = 2, SWEEP_SUBGRAD = 3 };
// Options of the hard sweep used by the quasi-Newton layer: rows see
// lambda + (*gamma) * dir (gamma on the device); the launch does nothing while
// *skip is nonzero; SWEEP_SUBGRAD writes 1 / 0 per slot to gsub.  dir and gsub
// hold five slot planes of n_free values: slot k of variable i at
// k * n_free + i.
struct SweepExt {
  const void* dir = nullptr;
  const double* gamma = nullptr;
  const int32_t* skip = nullptr;
  uint8_t* gsub = nullptr;
};
template <typename R>
dm_status dual_import(dm_ctx* ctx, const R* lam, DArr<unsigned char>* bufs);
template <typename R>
dm_status dual_export(dm_ctx* ctx, const unsigned char* rec, R* lam);
template <typename R>
dm_status dual_sweep(dm_ctx* ctx, int mode, bool soft, const unsigned char* rin, unsigned char* out, R omega,
                     R T, double* bound_out, const SweepExt* ext = nullptr);

// grid size helper
inline unsigned grid_for(int64_t n, int block) {
  return unsigned((n + block - 1) / block);
}

inline int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b < 1 ? 1 : b;
}
