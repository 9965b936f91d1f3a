// Generic 0-1 ILPs with +-1 rows (the paper's claim that the solver handles
// other 0-1 problems, Appendix "Other ILPs"): min c^T x subject to A x = b,
// x in {0,1}^n, every coefficient +1 or -1.  The rows are split as in the
// matching problem: exactly-one rows (all +1, b = 1, any length) and short
// rows (everything else, at most 64 entries).  The Lagrangean decomposition
// is that of Eq. (D): one subproblem per input row, and a variable in d rows
// (1 to 5) has d multipliers that sum to its cost.
//
// Full row order: the short input rows in input order, then the exactly-one
// input rows in input order.  A variable's record slots 0 to d - 1 follow its
// entries in that row order.
#include <algorithm>

#include "dm_internal.h"

namespace {

constexpr int ERR_COEF = 1, ERR_COL = 2, ERR_LONG = 4, ERR_DEG = 8, ERR_DUP = 16, ERR_NONFINITE = 32,
              ERR_PTR = 64;

// Every thread checks its own row's pointers (0 <= start <= end <= total, the
// first start 0) before it reads an entry, so malformed row pointers are
// reported and never index outside the total entries.
__global__ void k_ilp_rows(const int32_t* row_ptr, const int32_t* cols, const int8_t* coefs, const int32_t* b,
                           int32_t n_rows, int32_t n_vars, int32_t total, uint8_t* is_long, uint8_t* is_short,
                           int32_t* len, int32_t* deg, int* err) {
  const int32_t j = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n_rows) return;
  const int32_t s = row_ptr[j], e = row_ptr[j + 1];
  if (s < 0 || e < s || e > total || (j == 0 && s != 0)) {
    atomicOr(err, ERR_PTR);
    is_long[j] = 0;
    is_short[j] = 0;
    len[j] = 0;
    return;
  }
  bool all_pos = true;
  int bad = 0;
  for (int32_t i = s; i < e; ++i) {
    const int c = coefs[i];
    if (c != 1 && c != -1) bad |= ERR_COEF;
    all_pos = all_pos && c == 1;
    const int32_t v = cols[i];
    if (v < 0 || v >= n_vars) bad |= ERR_COL;
    else atomicAdd(&deg[v], 1);
  }
  const bool lg = all_pos && b[j] == 1 && e > s;
  if (!lg && e - s > MAX_SHORT_ROW) bad |= ERR_LONG;
  if (bad) atomicOr(err, bad);
  is_long[j] = lg ? 1 : 0;
  is_short[j] = lg ? 0 : 1;
  len[j] = e - s;
}

// new position of every input row and the lengths of the full rows
__global__ void k_ilp_place(const uint8_t* is_long, const int32_t* pos_short, const int32_t* pos_long,
                            const int32_t* len, int32_t n_rows, int32_t base_long, int32_t* new_row,
                            int32_t* new_len) {
  const int32_t j = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n_rows) return;
  const int32_t r = is_long[j] ? base_long + pos_long[j] : pos_short[j];
  new_row[j] = r;
  new_len[r] = len[j];
}

__global__ void k_ilp_fill(const int32_t* row_ptr, const int32_t* cols, const int8_t* coefs, const int32_t* b,
                           int32_t n_rows, const int32_t* new_row, const int32_t* full_ptr, int32_t* ent_var,
                           int8_t* ent_coef, int32_t* row_b, int64_t* row_key) {
  const int32_t j = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n_rows) return;
  const int32_t r = new_row[j], o = full_ptr[r], s = row_ptr[j];
  for (int32_t i = s; i < row_ptr[j + 1]; ++i) {
    ent_var[o + i - s] = cols[i];
    ent_coef[o + i - s] = coefs[i];
  }
  row_b[r] = b[j];
  row_key[r] = j;
}

// sort key of entry e: (variable, row); value e
__global__ void k_ilp_slot_keys(const int32_t* full_ptr, const int32_t* ent_var, int32_t n_full_rows, uint64_t* key,
                                int32_t* val) {
  const int32_t r = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n_full_rows) return;
  for (int32_t e = full_ptr[r]; e < full_ptr[r + 1]; ++e) {
    key[e] = uint64_t(ent_var[e]) * uint64_t(n_full_rows) + uint64_t(r);
    val[e] = e;
  }
}

// slot of every entry: its rank among its variable's entries (sorted keys);
// a repeated (variable, row) is an input row that names a variable twice
__global__ void k_ilp_slots(const uint64_t* key, const int32_t* val, int64_t nnz, int32_t n_full_rows,
                            uint8_t* slot, int* err) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const uint64_t per_var = uint64_t(n_full_rows);
  const uint64_t v = key[i] / per_var;
  int64_t lo = 0, hi = i;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key[mid] / per_var < v) lo = mid + 1;
    else hi = mid;
  }
  slot[val[i]] = uint8_t(i - lo);
  if (i > 0 && key[i] == key[i - 1]) atomicOr(err, ERR_DUP);   // same variable and row
}

// rows of every variable (checked to be 1 to 5) as the element degree
__global__ void k_ilp_deg(const int32_t* deg, int32_t n_vars, uint8_t* elem_deg, int* err) {
  const int32_t v = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= n_vars) return;
  const int32_t d = deg[v];
  if (d < 1 || d > 5) atomicOr(err, ERR_DEG);
  elem_deg[v] = uint8_t(d < 1 ? 1 : (d > 5 ? 5 : d));
}

__global__ void k_set_cost(const double* c, int64_t n, double* c64, float* c32, int* err) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double v = c[p];
  if (!isfinite(v)) atomicOr(err, ERR_NONFINITE);
  c64[p] = v;
  c32[p] = float(v);
}

dm_status build_ilp(dm_ctx* ctx, int32_t n_vars, int32_t n_rows, int32_t total, const int32_t* row_ptr,
                    const int32_t* cols, const int8_t* coefs, const int32_t* b) {
  hipStream_t st = ctx->stream;
  DArr<uint8_t> is_long, is_short;
  DArr<int32_t> len, deg, pos_short, pos_long, new_row;
  DArr<int> err;
  DM_ALLOC(ctx, is_long, size_t(std::max(n_rows, 1)));
  DM_ALLOC(ctx, is_short, size_t(std::max(n_rows, 1)));
  DM_ALLOC(ctx, len, size_t(std::max(n_rows, 1)));
  DM_ALLOC(ctx, new_row, size_t(std::max(n_rows, 1)));
  DM_ALLOC(ctx, deg, size_t(n_vars));
  DM_ALLOC(ctx, pos_short, size_t(n_rows) + 1);
  DM_ALLOC(ctx, pos_long, size_t(n_rows) + 1);
  DM_ALLOC(ctx, err, 1);
  DM_ALLOC(ctx, ctx->elem_deg, size_t(n_vars));
  DM_HIP(ctx, hipMemsetAsync(deg.p, 0, sizeof(int32_t) * n_vars, st));
  DM_HIP(ctx, hipMemsetAsync(err.p, 0, sizeof(int), st));
  if (n_rows > 0)
    k_ilp_rows<<<grid_for(n_rows, 256), 256, 0, st>>>(row_ptr, cols, coefs, b, n_rows, n_vars, total,
                                                       is_long.p, is_short.p, len.p, deg.p, err.p);
  k_ilp_deg<<<grid_for(n_vars, 256), 256, 0, st>>>(deg.p, n_vars, ctx->elem_deg.p, err.p);
  DM_LAUNCH_CHECK(ctx);
  DM_TRY(scan_u8(ctx, is_short.p, pos_short.p, size_t(n_rows)));
  DM_TRY(scan_u8(ctx, is_long.p, pos_long.p, size_t(n_rows)));
  int32_t v[2];
  {
    const int32_t* src[2] = {err.p, pos_short.p + n_rows};
    DM_TRY(read_i32s(ctx, 2, src, v));
  }
  if (v[0] & ERR_PTR)
    return dm_fail(ctx, DM_ERR_INVALID_ARG,
                   "dm_build_ilp: row pointers must start at 0, never decrease and end at the entry count");
  if (v[0] & ERR_COEF) return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_build_ilp: a coefficient is not +1 or -1");
  if (v[0] & ERR_COL) return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_build_ilp: a column is out of range");
  if (v[0] & ERR_LONG)
    return dm_fail(ctx, DM_ERR_WORKSPACE, "dm_build_ilp: a row that is not exactly-one has more than %d entries",
                   MAX_SHORT_ROW);
  if (v[0] & ERR_DEG) return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_build_ilp: a variable is in no row or in more than 5");
  const int32_t n_short_in = v[1];
  const int64_t n_full = n_rows;
  // full row lengths and pointers
  DArr<int32_t> new_len;
  DM_ALLOC(ctx, new_len, size_t(std::max<int64_t>(n_full, 1)));
  DM_ALLOC(ctx, ctx->row_ptr, size_t(n_full) + 1);
  if (n_rows > 0)
    k_ilp_place<<<grid_for(n_rows, 256), 256, 0, st>>>(is_long.p, pos_short.p, pos_long.p, len.p, n_rows,
                                                        n_short_in, new_row.p, new_len.p);
  DM_LAUNCH_CHECK(ctx);
  DM_TRY(scan_i32(ctx, new_len.p, ctx->row_ptr.p, size_t(n_full)));
  int32_t nnz = 0;
  DM_TRY(read_i32(ctx, ctx->row_ptr.p + n_full, &nnz));
  ctx->nP = n_vars;
  ctx->n_closed_full = n_short_in;
  ctx->n_rows_full = n_full;
  ctx->nnz_full = nnz;
  DM_ALLOC(ctx, ctx->row_key, size_t(std::max<int64_t>(n_full, 1)));
  DM_ALLOC(ctx, ctx->row_b, size_t(std::max<int64_t>(n_full, 1)));
  DM_ALLOC(ctx, ctx->ent_var, size_t(std::max(nnz, 1)));
  DM_ALLOC(ctx, ctx->ent_coef, size_t(std::max(nnz, 1)));
  DM_ALLOC(ctx, ctx->ent_slot, size_t(std::max(nnz, 1)));
  ctx->code.release();   // a generic problem has no element codes
  if (n_rows > 0)
    k_ilp_fill<<<grid_for(n_rows, 256), 256, 0, st>>>(row_ptr, cols, coefs, b, n_rows, new_row.p, ctx->row_ptr.p,
                                                       ctx->ent_var.p, ctx->ent_coef.p, ctx->row_b.p,
                                                       ctx->row_key.p);
  DM_LAUNCH_CHECK(ctx);
  // record slots
  if (nnz > 0) {
    DArr<uint64_t> key;
    DArr<int32_t> val;
    DM_ALLOC(ctx, key, size_t(nnz));
    DM_ALLOC(ctx, val, size_t(nnz));
    k_ilp_slot_keys<<<grid_for(n_full, 256), 256, 0, st>>>(ctx->row_ptr.p, ctx->ent_var.p, int32_t(n_full), key.p,
                                                            val.p);
    DM_LAUNCH_CHECK(ctx);
    DM_TRY(sort_pairs_u64(ctx, key.p, val.p, size_t(nnz), bits_for(uint64_t(n_vars) * uint64_t(n_full))));
    DM_HIP(ctx, hipMemsetAsync(err.p, 0, sizeof(int), st));
    k_ilp_slots<<<grid_for(nnz, 256), 256, 0, st>>>(key.p, val.p, nnz, int32_t(n_full), ctx->ent_slot.p, err.p);
    DM_LAUNCH_CHECK(ctx);
    int e = 0;
    DM_TRY(read_i32(ctx, err.p, &e));
    if (e & ERR_DUP) return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_build_ilp: a row names a variable twice");
  }
  ctx->X.nv = ctx->X.nf = ctx->X.ne = 0;   // no meshes behind a generic problem
  ctx->Y.nv = ctx->Y.nf = ctx->Y.ne = 0;
  ctx->nC = 0;
  ctx->K = 0;
  return presolve_reduce(ctx, nullptr);
}

}  // namespace

extern "C" dm_status dm_build_ilp(dm_ctx* ctx, int32_t n_vars, int32_t n_rows, const int32_t* row_ptr,
                                  const int32_t* cols, const int8_t* coefs, const int32_t* b,
                                  dm_space_info* info) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  ctx->has_space = false;
  ctx->corners_ready = false;
  ctx->has_cost = false;
  ctx->generic = true;
  if (n_vars < 1 || n_rows < 0 || !row_ptr || !b || !info)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_build_ilp: bad arguments");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  DM_TRY(dual_flush(ctx));
  ++ctx->cost_generation;
  int32_t total = 0;
  DM_TRY(read_i32(ctx, row_ptr + n_rows, &total));
  if (total < 0 || (total > 0 && (!cols || !coefs)))
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_build_ilp: bad row pointers or entries");
  DM_TRY(build_ilp(ctx, n_vars, n_rows, total, row_ptr, cols, coefs, b));
  ctx->has_space = true;
  fill_info(ctx, info);
  return DM_OK;
}

extern "C" dm_status dm_set_costs(dm_ctx* ctx, const double* cost) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!ctx->has_space) return dm_fail(ctx, DM_ERR_STATE, "dm_set_costs: no problem built");
  if (!cost && ctx->nP > 0) return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_set_costs: NULL cost");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  DM_TRY(dual_flush(ctx));
  hipStream_t st = ctx->stream;
  ctx->has_cost = false;
  ctx->desc_costs = false;
  DArr<int> err;
  DM_ALLOC(ctx, err, 1);
  DM_HIP(ctx, hipMemsetAsync(err.p, 0, sizeof(int), st));
  DM_ALLOC(ctx, ctx->cost64, size_t(std::max<int64_t>(ctx->nP, 1)));
  DM_ALLOC(ctx, ctx->cost32, size_t(std::max<int64_t>(ctx->nP, 1)));
  if (ctx->nP > 0)
    k_set_cost<<<grid_for(ctx->nP, 256), 256, 0, st>>>(cost, ctx->nP, ctx->cost64.p, ctx->cost32.p, err.p);
  DM_LAUNCH_CHECK(ctx);
  int e = 0;
  DM_TRY(read_i32(ctx, err.p, &e));
  if (e) return dm_fail(ctx, DM_ERR_NONFINITE, "dm_set_costs: a cost is not finite");
  DM_TRY(cost_offset(ctx));
  ctx->cost_prec = DM_PREC_FP64;
  ctx->has_cost = true;
  ++ctx->cost_generation;
  return DM_OK;
}
