// Product space, constraint rows and presolve (Sec. 3.1, Eq. (P)).
//
// The product space P holds triangle-triangle, triangle-edge and
// triangle-vertex matching elements in both directions (Sec. 3.1, Fig.
// "matching elements").  The exact element set is deferred by the paper to
// Windheuser et al. 2011; this library uses: an X face as stored against a
// Y face rotated by r = 0, 1, 2; an X face against a Y edge {b < b'} in the six
// two-symbol sequences (b b b') (b b' b) (b' b b) (b' b' b) (b' b b') (b b' b');
// an X face against a Y vertex (n n n); and the same with X and Y swapped (Y
// face as stored).  An element is kept when its three product vertices
// (m, n), id m*|V_Y|+n, are candidate pairs.  Elements are numbered in the
// order (X class face<edge<vertex, X id, Y class, Y id, rotation/pattern).
//
// Rows of A: one closedness row per undirected product edge (coefficient +1
// when an element walks it from the smaller to the larger product-vertex id,
// -1 otherwise, right-hand side 0), sorted by (min, max) key; one projection
// row per face of X and per face of Y (right-hand side 1).
//
// Presolve: integer unit propagation to its fixpoint, run as rounds of a row
// pass (which variables can no longer take 0 or 1) and a variable pass.  The
// fixpoint of a monotone propagation is unique, so the parallel rounds reach
// the same fixings as any sequential order.
#include "dm_internal.h"

namespace {

struct Geo {
  const int32_t *FX, *FY, *EX, *EY;
  int32_t nfx, nfy, nex, ney, nvx, nvy;
  int64_t W, QA, QB, Q;
};

__device__ inline void two_symbol(int pat, int32_t b, int32_t bp, int32_t out[3]) {
  // bit k of the mask selects b' for position k
  const int masks[6] = {4, 2, 1, 3, 5, 6};   // (b b b') (b b' b) (b' b b) (b' b' b) (b' b b') (b b' b')
  int m = masks[pat];
  out[0] = (m & 1) ? bp : b;
  out[1] = (m & 2) ? bp : b;
  out[2] = (m & 4) ? bp : b;
}

// element sequences for enumeration slot q and rotation/pattern pat; returns
// the number of patterns of the slot's class
__device__ inline int slot_seq(const Geo& g, int64_t q, int pat, int32_t xs[3], int32_t ys[3],
                               int32_t code[4]) {
  if (q < g.QA) {
    int32_t f = int32_t(q / g.W);
    int64_t j = q % g.W;
    xs[0] = g.FX[3 * f];
    xs[1] = g.FX[3 * f + 1];
    xs[2] = g.FX[3 * f + 2];
    code[0] = 0;
    code[1] = f;
    if (j < g.nfy) {
      int32_t gg = int32_t(j);
      for (int k = 0; k < 3; ++k) ys[k] = g.FY[3 * gg + (k + pat) % 3];
      code[2] = pat;
      code[3] = gg;
      return 3;
    }
    if (j < g.nfy + g.ney) {
      int32_t e = int32_t(j - g.nfy);
      two_symbol(pat, g.EY[2 * e], g.EY[2 * e + 1], ys);
      code[2] = 8 + pat;
      code[3] = e;
      return 6;
    }
    int32_t n = int32_t(j - g.nfy - g.ney);
    ys[0] = ys[1] = ys[2] = n;
    code[2] = 16;
    code[3] = n;
    return 1;
  }
  if (q < g.QB) {
    int64_t r = q - g.QA;
    int32_t e = int32_t(r / g.nfy), gg = int32_t(r % g.nfy);
    two_symbol(pat, g.EX[2 * e], g.EX[2 * e + 1], xs);
    for (int k = 0; k < 3; ++k) ys[k] = g.FY[3 * gg + k];
    code[0] = 1;
    code[1] = e;
    code[2] = pat;
    code[3] = gg;
    return 6;
  }
  int64_t r = q - g.QB;
  int32_t m = int32_t(r / g.nfy), gg = int32_t(r % g.nfy);
  xs[0] = xs[1] = xs[2] = m;
  for (int k = 0; k < 3; ++k) ys[k] = g.FY[3 * gg + k];
  code[0] = 2;
  code[1] = m;
  code[2] = 0;
  code[3] = gg;
  return 1;
}

__global__ void k_cand_mark(const int32_t* cand, int32_t nrows, int32_t K, int32_t nother, int dir,
                            int32_t nvy, uint8_t* map, int* err) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(nrows) * K) return;
  int32_t row = int32_t(i / K);
  int32_t o = cand[i];
  if (o < 0 || o >= nother) {
    atomicOr(err, 1);
    return;
  }
  int64_t q = dir == 0 ? int64_t(row) * nvy + o : int64_t(o) * nvy + row;
  map[q] = 1;
}

__global__ void k_cand_index(const uint8_t* map, int32_t* cidx, int32_t* cpair, int64_t npv) {
  int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= npv) return;
  int32_t s = cidx[q];
  if (map[q]) cpair[s] = int32_t(q);
  else cidx[q] = -1;
}

__global__ void k_xstart(const int32_t* scan, int32_t* xstart, int32_t nvx, int32_t nvy) {
  int32_t m = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m <= nvx) xstart[m] = scan[int64_t(m) * nvy];
}

__global__ void k_pair_tkeys(const int32_t* cpair, int64_t nC, int32_t nvx, int32_t nvy, uint32_t* key,
                             int32_t* val) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nC) return;
  int32_t q = cpair[i];
  key[i] = uint32_t(q % nvy) * uint32_t(nvx) + uint32_t(q / nvy);
  val[i] = int32_t(i);
}

__global__ void k_ystart(const uint32_t* key, int64_t nC, int32_t nvx, int32_t nvy, int32_t* ystart) {
  int32_t n = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n > nvy) return;
  uint32_t target = uint32_t(n) * uint32_t(nvx);
  int64_t lo = 0, hi = nC;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (key[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  ystart[n] = int32_t(lo);
}

__global__ void k_enum_mask(Geo g, const uint8_t* cand, uint8_t* mask, uint8_t* count) {
  int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= g.Q) return;
  int32_t xs[3], ys[3], code[4];
  int np = slot_seq(g, q, 0, xs, ys, code);
  uint8_t m = 0, c = 0;
  for (int pat = 0; pat < np; ++pat) {
    slot_seq(g, q, pat, xs, ys, code);
    bool keep = true;
    for (int k = 0; k < 3; ++k) keep = keep && cand[int64_t(xs[k]) * g.nvy + ys[k]];
    if (keep) {
      m |= uint8_t(1u << pat);
      ++c;
    }
  }
  mask[q] = m;
  count[q] = c;
}

__global__ void k_enum_fill(Geo g, const uint8_t* mask, const int32_t* off, int32_t* pv,
                            int32_t* code_out) {
  int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= g.Q) return;
  uint8_t m = mask[q];
  if (!m) return;
  int64_t o = off[q];
  int32_t xs[3], ys[3], code[4];
  for (int pat = 0; pat < 6; ++pat) {
    if (!(m & (1u << pat))) continue;
    slot_seq(g, q, pat, xs, ys, code);
    for (int k = 0; k < 3; ++k) pv[3 * o + k] = xs[k] * g.nvy + ys[k];
    for (int k = 0; k < 4; ++k) code_out[4 * o + k] = code[k];
    ++o;
  }
}

__global__ void k_edge_keys(const int32_t* pv, int64_t nP, uint64_t npv, uint64_t* key, int32_t* val) {
  int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= 3 * nP) return;
  int64_t p = s / 3;
  int k = int(s % 3);
  uint64_t a = uint32_t(pv[3 * p + k]), b = uint32_t(pv[3 * p + (k + 1) % 3]);
  key[s] = (a < b ? a : b) * npv + (a < b ? b : a);
  val[s] = int32_t(s);
}

__global__ void k_row_flags(const uint64_t* key, int64_t n, uint8_t* flag) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

__global__ void k_closed_fill(const uint64_t* key, const int32_t* val, const uint8_t* flag,
                              const int32_t* excl, const int32_t* pv, int64_t n, int32_t* row_ptr,
                              int64_t* row_key, int32_t* row_b, int32_t* ent_var, int8_t* ent_coef,
                              uint8_t* ent_slot) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (flag[i]) {
    int32_t r = excl[i];
    row_ptr[r] = int32_t(i);
    row_key[r] = int64_t(key[i]);
    row_b[r] = 0;
  }
  int32_t s = val[i];
  int32_t p = s / 3, k = s % 3;
  int32_t a = pv[3 * p + k], b = pv[3 * p + (k + 1) % 3];
  ent_var[i] = p;
  ent_coef[i] = a < b ? 1 : -1;
  ent_slot[i] = uint8_t(k);
}

__global__ void k_xproj(const int32_t* off, Geo g, int64_t base, int64_t nc, int64_t nXf,
                        int32_t* row_ptr, int64_t* row_key, int32_t* row_b, int32_t* ent_var,
                        int8_t* ent_coef, uint8_t* ent_slot) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < g.nfx) {
    row_ptr[nc + i] = int32_t(base + off[i * g.W]);
    row_key[nc + i] = i;
    row_b[nc + i] = 1;
  }
  if (i < nXf) {
    ent_var[base + i] = int32_t(i);
    ent_coef[base + i] = 1;
    ent_slot[base + i] = 3;
  }
}

__global__ void k_ykeys(const int32_t* code, int64_t nP, int32_t nfy, uint32_t* key, int32_t* val) {
  int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= nP) return;
  bool yface = (code[4 * p + 2] >> 3) == 0;
  int32_t g = code[4 * p + 3];
  key[p] = yface ? uint32_t(g) : uint32_t(nfy);
  val[p] = int32_t(p);
}

// yptr[g] = first position of key >= g in the sorted keys, g = 0..nfy
__global__ void k_key_starts(const uint32_t* key, int64_t n, int32_t nfy, int32_t* yptr) {
  const int32_t g = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g > nfy) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key[mid] < uint32_t(g)) lo = mid + 1;
    else hi = mid;
  }
  yptr[g] = int32_t(lo);
}

__global__ void k_yproj(const int32_t* yptr, const int32_t* val, const int32_t* code, Geo g,
                        int64_t base, int64_t nc, int64_t nYf, int32_t* row_ptr, int64_t* row_key,
                        int32_t* row_b, int32_t* ent_var, int8_t* ent_coef, uint8_t* ent_slot) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < g.nfy) {
    row_ptr[nc + g.nfx + i] = int32_t(base + yptr[i]);
    row_key[nc + g.nfx + i] = i;
    row_b[nc + g.nfx + i] = 1;
  }
  if (i < nYf) {
    int32_t p = val[i];
    ent_var[base + i] = p;
    ent_coef[base + i] = 1;
    ent_slot[base + i] = code[4 * int64_t(p)] == 0 ? 4 : 3;
  }
}

__global__ void k_set_i32(int32_t* a, int64_t i, int32_t v) { a[i] = v; }

// ---------------------------------------------------------------- presolve
// A presolve round does nothing once the round before it changed nothing or
// found the system infeasible (prev: that round's flags, or NULL).
__device__ inline bool presolve_done(const int* prev) {
  return prev && (prev[0] == 0 || prev[1] != 0);
}

// A row's entries are read PS_BATCH at a time, with indices clamped to the
// row, so that the loads of a batch go out together and need no branch.
constexpr int PS_BATCH = 8;

__global__ void k_presolve_rows(const int32_t* row_ptr, const int32_t* ent_var, const int8_t* ent_coef,
                                const int32_t* row_b, int64_t nrows, const int8_t* state,
                                uint32_t* force, int* flags, const int* prev) {
  if (presolve_done(prev)) return;   // uniform across the grid
  int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nrows) return;
  const int32_t s = row_ptr[j], e = row_ptr[j + 1];
  int32_t r = row_b[j], P = 0, N = 0;
  for (int32_t i0 = s; i0 < e; i0 += PS_BATCH) {
    int32_t v[PS_BATCH];
    int a[PS_BATCH];
#pragma unroll
    for (int u = 0; u < PS_BATCH; ++u) {
      const int32_t i = i0 + u < e ? i0 + u : i0;
      v[u] = ent_var[i];
      a[u] = ent_coef[i];
    }
    int8_t st[PS_BATCH];
#pragma unroll
    for (int u = 0; u < PS_BATCH; ++u) st[u] = state[v[u]];
#pragma unroll
    for (int u = 0; u < PS_BATCH; ++u) {
      if (i0 + u >= e) continue;
      if (st[u] == 1) r -= a[u];
      else if (st[u] < 0) {
        if (a[u] > 0) ++P;
        else ++N;
      }
    }
  }
  if (r < -N || r > P) {
    atomicOr(&flags[1], 1);
    return;
  }
  for (int32_t i0 = s; i0 < e; i0 += PS_BATCH) {
    int32_t v[PS_BATCH];
    int a[PS_BATCH];
#pragma unroll
    for (int u = 0; u < PS_BATCH; ++u) {
      const int32_t i = i0 + u < e ? i0 + u : i0;
      v[u] = ent_var[i];
      a[u] = ent_coef[i];
    }
    int8_t st[PS_BATCH];
#pragma unroll
    for (int u = 0; u < PS_BATCH; ++u) st[u] = state[v[u]];
#pragma unroll
    for (int u = 0; u < PS_BATCH; ++u) {
      if (i0 + u >= e || st[u] >= 0) continue;
      const int32_t Pr = P - (a[u] > 0 ? 1 : 0), Nr = N - (a[u] < 0 ? 1 : 0);
      const bool one_ok = (r - a[u] >= -Nr) && (r - a[u] <= Pr);
      const bool zero_ok = (r >= -Nr) && (r <= Pr);
      if (!one_ok && !zero_ok) atomicOr(&flags[1], 1);
      else if (!one_ok) atomicOr(&force[v[u]], 1u);
      else if (!zero_ok) atomicOr(&force[v[u]], 2u);
    }
  }
}

// The round's (changed, clash) flags: one atomic OR per block and flag (the
// block's threads first meet in LDS), not one per wave on a single word.
__global__ __launch_bounds__(256) void k_presolve_vars(int64_t nP, int8_t* state, uint32_t* force, int* flags,
                                                       const int* prev) {
  __shared__ int any[2];
  if (presolve_done(prev)) return;   // uniform across the grid
  if (threadIdx.x < 2) any[threadIdx.x] = 0;
  __syncthreads();
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < nP) {
    const uint32_t f = force[p];
    if (f) {
      force[p] = 0;
      if (f == 3u) {
        any[1] = 1;
      } else if (state[p] < 0) {
        state[p] = (f == 2u) ? 1 : 0;
        any[0] = 1;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (any[0]) atomicOr(&flags[0], 1);
    if (any[1]) atomicOr(&flags[1], 1);
  }
}

__global__ void k_fix_state(const int8_t* fix, int64_t nP, int8_t* state) {
  int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p < nP) state[p] = fix[p] < 0 ? int8_t(-1) : int8_t(fix[p] ? 1 : 0);
}

__global__ void k_free_flags(const int8_t* state, int64_t nP, uint8_t* flag, int* nfix1) {
  int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= nP) return;
  flag[p] = state[p] < 0 ? 1 : 0;
  if (state[p] == 1) atomicAdd(nfix1, 1);
}

__global__ void k_free_fill(const int8_t* state, const int32_t* excl, int64_t nP, int32_t* var_red,
                            int32_t* free_var) {
  int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= nP) return;
  if (state[p] < 0) {
    var_red[p] = excl[p];
    free_var[excl[p]] = int32_t(p);
  } else {
    var_red[p] = -1;
  }
}

__global__ void k_row_residual(const int32_t* row_ptr, const int32_t* ent_var, const int8_t* ent_coef,
                               const int32_t* row_b, int64_t nrows, const int8_t* state,
                               int32_t* nfree, int32_t* resid, uint8_t* keep, int* flags) {
  int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nrows) return;
  int32_t r = row_b[j], c = 0;
  for (int32_t i = row_ptr[j]; i < row_ptr[j + 1]; ++i) {
    int8_t st = state[ent_var[i]];
    if (st == 1) r -= ent_coef[i];
    else if (st < 0) ++c;
  }
  if (c == 0 && r != 0) atomicOr(&flags[1], 1);
  nfree[j] = c;
  resid[j] = r;
  keep[j] = c > 0 ? 1 : 0;
}

__global__ void k_reduced_fill(const int32_t* row_ptr, const int32_t* ent_var, const int8_t* ent_coef,
                               const uint8_t* ent_slot, int64_t nrows, const int8_t* state,
                               const int32_t* var_red, const int32_t* free_var,
                               const uint8_t* keep, const int32_t* new_id, const int32_t* cnt_excl,
                               const int32_t* resid, int32_t* rrow_orig, int32_t* rrow_ptr,
                               int32_t* rrow_b, int32_t* rent_var, int8_t* rent_coef,
                               uint32_t* rent_word) {
  int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= nrows || !keep[j]) return;
  int32_t nr = new_id[j];
  rrow_orig[nr] = int32_t(j);
  rrow_b[nr] = resid[j];
  int32_t pos = cnt_excl[j];
  rrow_ptr[nr] = pos;
  for (int32_t i = row_ptr[j]; i < row_ptr[j + 1]; ++i) {
    int32_t v = ent_var[i];
    if (state[v] >= 0) continue;
    int32_t rv = var_red[v];
    int a = ent_coef[i];
    rent_var[pos] = rv;
    rent_coef[pos] = int8_t(a);
    rent_word[pos] = (a < 0 ? W_NEG : 0u) | (uint32_t(ent_slot[i]) << W_SLOT_SHIFT) | uint32_t(rv);
    ++pos;
  }
}

// ---- projection rows (all coefficients +1, right-hand side 1, hundreds to
// thousands of entries): one 256-thread block per row
__device__ inline int block_sum_i(int v, int* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  return sh[0] + sh[1] + sh[2] + sh[3];
}

// exclusive prefix of a 0/1 flag over the block (thread order), and the total
__device__ inline int block_excl_flag(bool f, int* sh, int* total) {
  const unsigned long long m = __ballot(f);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int in_wave = __popcll(m & ((1ull << lane) - 1ull));
  __syncthreads();
  if (lane == 0) sh[wave] = __popcll(m);
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wave; ++w) before += sh[w];
  *total = sh[0] + sh[1] + sh[2] + sh[3];
  return before + in_wave;
}

__global__ __launch_bounds__(256) void k_presolve_proj(const int32_t* row_ptr, const int32_t* ent_var, int64_t nc,
                                                       const int8_t* state, uint32_t* force, int* flags,
                                                       const int* prev) {
  __shared__ int sh[4];
  if (presolve_done(prev)) return;   // uniform across the grid
  const int64_t j = nc + blockIdx.x;
  const int32_t s = row_ptr[j], e = row_ptr[j + 1];
  int c1 = 0, cf = 0;
  for (int32_t i = s + threadIdx.x; i < e; i += blockDim.x) {
    int8_t st = state[ent_var[i]];
    c1 += st == 1;
    cf += st < 0;
  }
  const int ones = block_sum_i(c1, sh);
  const int P = block_sum_i(cf, sh);
  const int r = 1 - ones;
  if (r < 0 || r > P) {
    if (threadIdx.x == 0) atomicOr(&flags[1], 1);
    return;
  }
  // r == 0: every free entry must be 0; r == 1 with one free entry: it is 1
  if (r == 0 || P == 1)
    for (int32_t i = s + threadIdx.x; i < e; i += blockDim.x) {
      int32_t v = ent_var[i];
      if (state[v] < 0) atomicOr(&force[v], r == 0 ? 1u : 2u);
    }
}

__global__ __launch_bounds__(256) void k_row_residual_proj(const int32_t* row_ptr, const int32_t* ent_var,
                                                           int64_t nc, const int8_t* state, int32_t* nfree,
                                                           int32_t* resid, uint8_t* keep, int* flags) {
  __shared__ int sh[4];
  const int64_t j = nc + blockIdx.x;
  int c1 = 0, cf = 0;
  for (int32_t i = row_ptr[j] + threadIdx.x; i < row_ptr[j + 1]; i += blockDim.x) {
    int8_t st = state[ent_var[i]];
    c1 += st == 1;
    cf += st < 0;
  }
  const int ones = block_sum_i(c1, sh);
  const int c = block_sum_i(cf, sh);
  if (threadIdx.x == 0) {
    if (c == 0 && 1 - ones != 0) atomicOr(&flags[1], 1);
    nfree[j] = c;
    resid[j] = 1 - ones;
    keep[j] = c > 0 ? 1 : 0;
  }
}

__global__ __launch_bounds__(256) void k_reduced_fill_proj(
    const int32_t* row_ptr, const int32_t* ent_var, const uint8_t* ent_slot, int64_t nc, const int8_t* state,
    const int32_t* var_red, const uint8_t* keep, const int32_t* new_id,
    const int32_t* cnt_excl, const int32_t* resid, int32_t* rrow_orig, int32_t* rrow_ptr, int32_t* rrow_b,
    int32_t* rent_var, int8_t* rent_coef, uint32_t* rent_word) {
  __shared__ int sh[4];
  const int64_t j = nc + blockIdx.x;
  if (!keep[j]) return;   // uniform over the block
  const int32_t nr = new_id[j];
  if (threadIdx.x == 0) {
    rrow_orig[nr] = int32_t(j);
    rrow_b[nr] = resid[j];
    rrow_ptr[nr] = cnt_excl[j];
  }
  int32_t pos = cnt_excl[j];
  for (int32_t t0 = row_ptr[j]; t0 < row_ptr[j + 1]; t0 += blockDim.x) {
    const int32_t i = t0 + threadIdx.x;
    const bool in = i < row_ptr[j + 1];
    const int32_t v = in ? ent_var[i] : 0;
    const bool f = in && state[v] < 0;
    int total = 0;
    const int off = block_excl_flag(f, sh, &total);
    if (f) {
      const int32_t rv = var_red[v];
      rent_var[pos + off] = rv;
      rent_coef[pos + off] = 1;
      rent_word[pos + off] = (uint32_t(ent_slot[i]) << W_SLOT_SHIFT) | uint32_t(rv);
    }
    pos += total;
  }
}

__global__ void k_var_deg(const int32_t* free_var, const uint8_t* elem_deg, int64_t n, uint8_t* deg) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  deg[i] = elem_deg[free_var[i]];
}

// rows of every product triangle: three closedness rows, plus the X projection
// row when its X element is a face and the Y projection row when its Y
// element is a face
__global__ void k_elem_deg(const int32_t* code, int64_t n, uint8_t* deg) {
  int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n) return;
  deg[p] = uint8_t(3 + (code[4 * p] == 0 ? 1 : 0) + ((code[4 * p + 2] >> 3) == 0 ? 1 : 0));
}

// flags[2]: longest short row; flags[3] bit 1: a row with < 2 entries, bit 0:
// a projection row that is not exactly-one.  One update per block at most:
// the block's maximum goes to flags[2] only while it exceeds what is stored
// there (a maximum only grows, so a block that reads a value at least as
// large has nothing to add), since one atomic per wave on that one word
// serialised the kernel on large problems
__global__ void k_row_stats(const int32_t* rrow_ptr, const int32_t* rrow_b, int64_t n_short, int64_t n_rows,
                            int* flags) {
  // no early return: every lane of the wave takes part in the reductions
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool in = j < n_rows;
  const int32_t len = in ? rrow_ptr[j + 1] - rrow_ptr[j] : 2;
  int32_t short_len = 0;
  bool bad_proj = false;
  if (in && j < n_short) short_len = len;
  else if (in) bad_proj = rrow_b[j] != 1;   // coefficients: k_long_coefs
  __shared__ int wmax[4], wbits[4];
  for (int o = 32; o > 0; o >>= 1) short_len = max(short_len, __shfl_xor(short_len, o));
  const unsigned long long few = __ballot(len < 2), bad = __ballot(bad_proj);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    wmax[wave] = short_len;
    wbits[wave] = (few ? 2 : 0) | (bad ? 1 : 0);   // presolve leaves >= 2 free entries per row
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int m = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
    const int bits = wbits[0] | wbits[1] | wbits[2] | wbits[3];
    if (m > 0 && m > __hip_atomic_load(&flags[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(&flags[2], m);
    if (bits) atomicOr(&flags[3], bits);
  }
}

// every coefficient of a projection (exactly-one) row must be +1; those rows
// hold the entries from rrow_ptr[n_short] on, checked one entry per thread
__global__ void k_long_coefs(const int32_t* rrow_ptr, int64_t n_short, int64_t nnz, const int8_t* coef,
                             int* flags) {
  // no early return: every lane of the wave takes part in the ballot
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t start = rrow_ptr[n_short];
  const bool bad = i >= start && i < nnz && coef[i] != 1;
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(&flags[3], 1);
}

__global__ void k_row_len(const int32_t* rrow_ptr, int64_t n_short, uint32_t* len, int32_t* row) {
  int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n_short) return;
  len[j] = uint32_t(rrow_ptr[j + 1] - rrow_ptr[j]);
  row[j] = int32_t(j);
}

// bound[0] / bound[1]: how many of the sorted lengths are <= 7 / <= 15
__global__ void k_len_bounds(const uint32_t* len, int64_t n, int32_t* bound) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t nxt = i + 1 < n ? len[i + 1] : 0xFFFFFFFFu;
  if (len[i] <= 7 && nxt > 7) bound[0] = int32_t(i + 1);
  if (len[i] <= 15 && nxt > 15) bound[1] = int32_t(i + 1);
}

}  // namespace

dm_status space_build(dm_ctx* ctx, const int32_t* cand_xy, const int32_t* cand_yx, int32_t K) {
  MeshDev& X = ctx->X;
  MeshDev& Y = ctx->Y;
  const int32_t nvx = X.nv, nvy = Y.nv;
  const int64_t npv = int64_t(nvx) * nvy;
  hipStream_t st = ctx->stream;
  DArr<int> err;
  DM_ALLOC(ctx, err, 4);
  DM_HIP(ctx, hipMemsetAsync(err.p, 0, 4 * sizeof(int), st));

  // ---- candidate map and pair lists
  DM_ALLOC(ctx, ctx->cand, size_t(npv));
  DM_HIP(ctx, hipMemsetAsync(ctx->cand.p, 0, size_t(npv), st));
  k_cand_mark<<<grid_for(int64_t(nvx) * K, 256), 256, 0, st>>>(cand_xy, nvx, K, nvy, 0, nvy,
                                                               ctx->cand.p, err.p);
  k_cand_mark<<<grid_for(int64_t(nvy) * K, 256), 256, 0, st>>>(cand_yx, nvy, K, nvx, 1, nvy,
                                                               ctx->cand.p, err.p);
  DM_LAUNCH_CHECK(ctx);
  int e0 = 0;
  DM_TRY(read_i32(ctx, err.p, &e0));
  if (e0) return dm_fail(ctx, DM_ERR_INVALID_ARG, "candidate index out of range");
  DM_ALLOC(ctx, ctx->cidx, size_t(npv) + 1);
  DM_TRY(scan_u8(ctx, ctx->cand.p, ctx->cidx.p, size_t(npv)));
  int32_t nC = 0;
  DM_TRY(read_i32(ctx, ctx->cidx.p + npv, &nC));
  ctx->nC = nC;
  DM_ALLOC(ctx, ctx->cpair, size_t(nC));
  DM_ALLOC(ctx, ctx->cand_xstart, size_t(nvx) + 1);
  k_xstart<<<grid_for(nvx + 1, 256), 256, 0, st>>>(ctx->cidx.p, ctx->cand_xstart.p, nvx, nvy);
  k_cand_index<<<grid_for(npv, 256), 256, 0, st>>>(ctx->cand.p, ctx->cidx.p, ctx->cpair.p, npv);
  DM_LAUNCH_CHECK(ctx);
  {
    DArr<uint32_t> tkey;
    DM_ALLOC(ctx, tkey, size_t(nC));
    DM_ALLOC(ctx, ctx->cpair_t, size_t(nC));
    DM_ALLOC(ctx, ctx->cand_ystart, size_t(nvy) + 1);
    k_pair_tkeys<<<grid_for(nC, 256), 256, 0, st>>>(ctx->cpair.p, nC, nvx, nvy, tkey.p, ctx->cpair_t.p);
    DM_LAUNCH_CHECK(ctx);
    DM_TRY(sort_pairs_u32(ctx, tkey.p, ctx->cpair_t.p, size_t(nC), bits_for(uint64_t(npv))));
    k_ystart<<<grid_for(nvy + 1, 256), 256, 0, st>>>(tkey.p, nC, nvx, nvy, ctx->cand_ystart.p);
    DM_LAUNCH_CHECK(ctx);
  }

  // ---- enumeration of the product space in canonical order
  Geo g;
  g.FX = X.faces.p;
  g.FY = Y.faces.p;
  g.EX = X.edges.p;
  g.EY = Y.edges.p;
  g.nfx = X.nf;
  g.nfy = Y.nf;
  g.nex = X.ne;
  g.ney = Y.ne;
  g.nvx = nvx;
  g.nvy = nvy;
  g.W = int64_t(Y.nf) + Y.ne + Y.nv;
  g.QA = int64_t(X.nf) * g.W;
  g.QB = g.QA + int64_t(X.ne) * Y.nf;
  g.Q = g.QB + int64_t(X.nv) * Y.nf;
  if (g.Q >= (int64_t(1) << 31))
    return dm_fail(ctx, DM_ERR_WORKSPACE, "product-space slot count %lld exceeds 2^31", (long long)g.Q);
  DArr<int32_t> off;
  {
    DArr<uint8_t> count;
    DArr<uint8_t> mask;
    DM_ALLOC(ctx, mask, size_t(g.Q));
    DM_ALLOC(ctx, count, size_t(g.Q));
    DM_ALLOC(ctx, off, size_t(g.Q) + 1);
    k_enum_mask<<<grid_for(g.Q, 256), 256, 0, st>>>(g, ctx->cand.p, mask.p, count.p);
    DM_LAUNCH_CHECK(ctx);
    DM_TRY(scan_u8(ctx, count.p, off.p, size_t(g.Q)));
    int32_t nP = 0;
    DM_TRY(read_i32(ctx, off.p + g.Q, &nP));
    ctx->nP = nP;
    if (nP == 0) return dm_fail(ctx, DM_ERR_INFEASIBLE, "no product triangle survives pruning");
    if (int64_t(nP) * 5 >= (int64_t(1) << 31) || nP >= int64_t(W_VAR_MASK))
      return dm_fail(ctx, DM_ERR_WORKSPACE, "product space of %d elements is too large", nP);
    DM_ALLOC(ctx, ctx->pv, size_t(nP) * 3);
    DM_ALLOC(ctx, ctx->code, size_t(nP) * 4);
    k_enum_fill<<<grid_for(g.Q, 256), 256, 0, st>>>(g, mask.p, off.p, ctx->pv.p, ctx->code.p);
    DM_ALLOC(ctx, ctx->elem_deg, size_t(std::max<int64_t>(nP, 1)));
    if (nP > 0) k_elem_deg<<<grid_for(nP, 256), 256, 0, st>>>(ctx->code.p, nP, ctx->elem_deg.p);
    DM_LAUNCH_CHECK(ctx);
  }
  const int64_t nP = ctx->nP;

  // ---- closedness rows: sort the 3|P| directed boundary edges by key
  DArr<uint64_t> ekey;
  DArr<int32_t> eval_;
  DM_ALLOC(ctx, ekey, size_t(3 * nP));
  DM_ALLOC(ctx, eval_, size_t(3 * nP));
  k_edge_keys<<<grid_for(3 * nP, 256), 256, 0, st>>>(ctx->pv.p, nP, uint64_t(npv), ekey.p, eval_.p);
  DM_LAUNCH_CHECK(ctx);
  DM_TRY(sort_pairs_u64(ctx, ekey.p, eval_.p, size_t(3 * nP), bits_for(uint64_t(npv) * uint64_t(npv))));
  DArr<uint8_t> rflag;
  DArr<int32_t> rexcl;
  DM_ALLOC(ctx, rflag, size_t(3 * nP));
  DM_ALLOC(ctx, rexcl, size_t(3 * nP) + 1);
  k_row_flags<<<grid_for(3 * nP, 256), 256, 0, st>>>(ekey.p, 3 * nP, rflag.p);
  DM_LAUNCH_CHECK(ctx);
  DM_TRY(scan_u8(ctx, rflag.p, rexcl.p, size_t(3 * nP)));
  int32_t nc = 0, nXf = 0;
  {
    const int32_t* src[2] = {rexcl.p + 3 * nP, off.p + g.QA};
    int32_t v[2];
    DM_TRY(read_i32s(ctx, 2, src, v));
    nc = v[0];
    nXf = v[1];
  }
  ctx->n_closed_full = nc;

  // ---- Y projection rows: stable sort of Y-face elements by face
  DArr<uint32_t> ykey;
  DArr<int32_t> yval, yptr;
  DM_ALLOC(ctx, ykey, size_t(nP));
  DM_ALLOC(ctx, yval, size_t(nP));
  DM_ALLOC(ctx, yptr, size_t(Y.nf) + 1);
  k_ykeys<<<grid_for(nP, 256), 256, 0, st>>>(ctx->code.p, nP, Y.nf, ykey.p, yval.p);
  DM_LAUNCH_CHECK(ctx);
  DM_TRY(sort_pairs_u32(ctx, ykey.p, yval.p, size_t(nP), bits_for(uint64_t(Y.nf) + 1)));
  k_key_starts<<<grid_for(int64_t(Y.nf) + 1, 256), 256, 0, st>>>(ykey.p, nP, Y.nf, yptr.p);
  DM_LAUNCH_CHECK(ctx);
  int32_t nYf = 0;
  DM_TRY(read_i32(ctx, yptr.p + Y.nf, &nYf));

  const int64_t nrows = int64_t(nc) + X.nf + Y.nf;
  const int64_t nnz = 3 * nP + nXf + nYf;
  if (nnz >= (int64_t(1) << 31)) return dm_fail(ctx, DM_ERR_WORKSPACE, "too many nonzeros");
  ctx->n_rows_full = nrows;
  ctx->nnz_full = nnz;
  DM_ALLOC(ctx, ctx->row_ptr, size_t(nrows) + 1);
  DM_ALLOC(ctx, ctx->row_key, size_t(nrows));
  DM_ALLOC(ctx, ctx->row_b, size_t(nrows));
  DM_ALLOC(ctx, ctx->ent_var, size_t(nnz));
  DM_ALLOC(ctx, ctx->ent_coef, size_t(nnz));
  DM_ALLOC(ctx, ctx->ent_slot, size_t(nnz));
  k_closed_fill<<<grid_for(3 * nP, 256), 256, 0, st>>>(ekey.p, eval_.p, rflag.p, rexcl.p, ctx->pv.p, 3 * nP,
                                                       ctx->row_ptr.p, ctx->row_key.p, ctx->row_b.p,
                                                       ctx->ent_var.p, ctx->ent_coef.p, ctx->ent_slot.p);
  k_xproj<<<grid_for(std::max<int64_t>(X.nf, nXf), 256), 256, 0, st>>>(
      off.p, g, 3 * nP, nc, nXf, ctx->row_ptr.p, ctx->row_key.p, ctx->row_b.p, ctx->ent_var.p,
      ctx->ent_coef.p, ctx->ent_slot.p);
  k_yproj<<<grid_for(std::max<int64_t>(Y.nf, nYf), 256), 256, 0, st>>>(
      yptr.p, yval.p, ctx->code.p, g, 3 * nP + nXf, nc, nYf, ctx->row_ptr.p, ctx->row_key.p,
      ctx->row_b.p, ctx->ent_var.p, ctx->ent_coef.p, ctx->ent_slot.p);
  k_set_i32<<<1, 1, 0, st>>>(ctx->row_ptr.p, nrows, int32_t(nnz));
  DM_LAUNCH_CHECK(ctx);
  ekey.release();
  eval_.release();
  rflag.release();
  rexcl.release();
  ykey.release();
  yval.release();
  off.release();

  return presolve_reduce(ctx, nullptr);
}

// Integer unit propagation to the fixpoint from a starting assignment (fix:
// per element -1 free or 0 / 1, or NULL for none), then the reduced problem,
// its row statistics and the wave chunks of its closedness rows.
dm_status presolve_reduce(dm_ctx* ctx, const int8_t* fix) {
  hipStream_t st = ctx->stream;
  const int64_t nP = ctx->nP, nc = ctx->n_closed_full, nrows = ctx->n_rows_full;
  DArr<int> err;
  DM_ALLOC(ctx, err, 4);
  DM_HIP(ctx, hipMemsetAsync(err.p, 0, 4 * sizeof(int), st));
  // ---- presolve rounds
  DM_ALLOC(ctx, ctx->state, size_t(nP));
  if (fix) {
    if (nP > 0) k_fix_state<<<grid_for(nP, 256), 256, 0, st>>>(fix, nP, ctx->state.p);
    DM_LAUNCH_CHECK(ctx);
  } else {
    DM_HIP(ctx, hipMemsetAsync(ctx->state.p, 0xFF, size_t(nP), st));
  }
  DArr<uint32_t> force;
  DM_ALLOC(ctx, force, size_t(nP));
  DM_HIP(ctx, hipMemsetAsync(force.p, 0, sizeof(uint32_t) * nP, st));
  // Rounds run in batches of PRESOLVE_BATCH with one host read per batch:
  // round k writes its (changed, infeasible) flags to rflags[2k..2k+1], and
  // a round whose predecessor changed nothing (or found infeasibility) does
  // nothing, so the state after the batch is the state at the fixpoint.
  constexpr int PRESOLVE_BATCH = 4;
  DArr<int> rflags;
  DM_ALLOC(ctx, rflags, 2 * PRESOLVE_BATCH);
  int rounds = 0;
  for (bool done = false; !done;) {
    DM_HIP(ctx, hipMemsetAsync(rflags.p, 0, 2 * PRESOLVE_BATCH * sizeof(int), st));
    for (int k = 0; k < PRESOLVE_BATCH; ++k) {
      int* fl = rflags.p + 2 * k;
      const int* prev = k > 0 ? rflags.p + 2 * (k - 1) : nullptr;
      if (nc > 0)
        k_presolve_rows<<<grid_for(nc, 128), 128, 0, st>>>(ctx->row_ptr.p, ctx->ent_var.p, ctx->ent_coef.p,
                                                           ctx->row_b.p, nc, ctx->state.p, force.p, fl, prev);
      if (nrows > nc)
        k_presolve_proj<<<unsigned(nrows - nc), 256, 0, st>>>(ctx->row_ptr.p, ctx->ent_var.p, nc, ctx->state.p,
                                                            force.p, fl, prev);
      k_presolve_vars<<<grid_for(nP, 256), 256, 0, st>>>(nP, ctx->state.p, force.p, fl, prev);
    }
    DM_LAUNCH_CHECK(ctx);
    int flags[2 * PRESOLVE_BATCH];
    DM_HIP(ctx, hipMemcpyAsync(flags, rflags.p, sizeof(flags), hipMemcpyDeviceToHost, st));
    DM_HIP(ctx, hipStreamSynchronize(st));
    for (int k = 0; k < PRESOLVE_BATCH && !done; ++k) {
      ++rounds;
      if (flags[2 * k + 1])
        return dm_fail(ctx, DM_ERR_INFEASIBLE, "presolve proved A x = b infeasible (round %d)", rounds);
      done = !flags[2 * k];
    }
    if (!done && rounds > nP + 2) return dm_fail(ctx, DM_ERR_STATE, "presolve did not converge");
  }
  ctx->presolve_rounds = rounds;

  // ---- reduced problem
  DArr<uint8_t> fflag;
  DArr<int32_t> fexcl;
  DM_ALLOC(ctx, fflag, size_t(nP));
  DM_ALLOC(ctx, fexcl, size_t(nP) + 1);
  DM_HIP(ctx, hipMemsetAsync(err.p, 0, 4 * sizeof(int), st));
  k_free_flags<<<grid_for(nP, 256), 256, 0, st>>>(ctx->state.p, nP, fflag.p, err.p + 1);
  DM_LAUNCH_CHECK(ctx);
  DM_TRY(scan_u8(ctx, fflag.p, fexcl.p, size_t(nP)));
  int32_t nfree = 0, nfix1 = 0;
  {
    const int32_t* src[2] = {fexcl.p + nP, err.p + 1};
    int32_t v[2];
    DM_TRY(read_i32s(ctx, 2, src, v));
    nfree = v[0];
    nfix1 = v[1];
  }
  ctx->n_free = nfree;
  ctx->n_fixed1 = nfix1;
  DM_ALLOC(ctx, ctx->var_red, size_t(nP));
  DM_ALLOC(ctx, ctx->free_var, size_t(std::max(nfree, 1)));
  k_free_fill<<<grid_for(nP, 256), 256, 0, st>>>(ctx->state.p, fexcl.p, nP, ctx->var_red.p, ctx->free_var.p);
  DM_LAUNCH_CHECK(ctx);

  DArr<int32_t> nfr, resid, new_id, cnt_excl;
  DArr<uint8_t> keep;
  DM_ALLOC(ctx, nfr, size_t(nrows));
  DM_ALLOC(ctx, resid, size_t(nrows));
  DM_ALLOC(ctx, keep, size_t(nrows));
  DM_ALLOC(ctx, new_id, size_t(nrows) + 1);
  DM_ALLOC(ctx, cnt_excl, size_t(nrows) + 1);
  DM_HIP(ctx, hipMemsetAsync(err.p, 0, 4 * sizeof(int), st));
  if (nc > 0)
    k_row_residual<<<grid_for(nc, 128), 128, 0, st>>>(ctx->row_ptr.p, ctx->ent_var.p, ctx->ent_coef.p,
                                                      ctx->row_b.p, nc, ctx->state.p, nfr.p, resid.p, keep.p,
                                                      err.p);
  if (nrows > nc)
    k_row_residual_proj<<<unsigned(nrows - nc), 256, 0, st>>>(ctx->row_ptr.p, ctx->ent_var.p, nc, ctx->state.p,
                                                            nfr.p, resid.p, keep.p, err.p);
  DM_LAUNCH_CHECK(ctx);
  DM_TRY(scan_u8(ctx, keep.p, new_id.p, size_t(nrows)));
  DM_TRY(scan_i32(ctx, nfr.p, cnt_excl.p, size_t(nrows)));
  int32_t nr = 0, rnnz = 0, nshort = 0, flg1 = 0;
  {
    const int32_t* src[4] = {err.p + 1, new_id.p + nrows, cnt_excl.p + nrows, new_id.p + nc};
    int32_t v[4];
    DM_TRY(read_i32s(ctx, 4, src, v));
    flg1 = v[0];
    nr = v[1];
    rnnz = v[2];
    nshort = v[3];
  }
  if (flg1) return dm_fail(ctx, DM_ERR_INFEASIBLE, "a fully fixed row is violated");
  ctx->n_rows = nr;
  ctx->nnz = rnnz;
  ctx->n_short = nshort;
  DM_ALLOC(ctx, ctx->rrow_orig, size_t(std::max(nr, 1)));
  DM_ALLOC(ctx, ctx->rrow_ptr, size_t(nr) + 1);
  DM_ALLOC(ctx, ctx->rrow_b, size_t(std::max(nr, 1)));
  DM_ALLOC(ctx, ctx->rent_var, size_t(std::max(rnnz, 1)));
  DM_ALLOC(ctx, ctx->rent_coef, size_t(std::max(rnnz, 1)));
  DM_ALLOC(ctx, ctx->rent_word, size_t(std::max(rnnz, 1)));
  if (nc > 0)
    k_reduced_fill<<<grid_for(nc, 128), 128, 0, st>>>(
        ctx->row_ptr.p, ctx->ent_var.p, ctx->ent_coef.p, ctx->ent_slot.p, nc, ctx->state.p, ctx->var_red.p,
        ctx->free_var.p, keep.p, new_id.p, cnt_excl.p, resid.p, ctx->rrow_orig.p, ctx->rrow_ptr.p,
        ctx->rrow_b.p, ctx->rent_var.p, ctx->rent_coef.p, ctx->rent_word.p);
  if (nrows > nc)
    k_reduced_fill_proj<<<unsigned(nrows - nc), 256, 0, st>>>(
      ctx->row_ptr.p, ctx->ent_var.p, ctx->ent_slot.p, nc, ctx->state.p, ctx->var_red.p, keep.p,
      new_id.p, cnt_excl.p, resid.p, ctx->rrow_orig.p, ctx->rrow_ptr.p, ctx->rrow_b.p, ctx->rent_var.p,
      ctx->rent_coef.p, ctx->rent_word.p);
  k_set_i32<<<1, 1, 0, st>>>(ctx->rrow_ptr.p, nr, rnnz);
  DM_LAUNCH_CHECK(ctx);
  DM_ALLOC(ctx, ctx->var_deg, size_t(std::max(nfree, 1)));
  if (nfree > 0)
    k_var_deg<<<grid_for(nfree, 256), 256, 0, st>>>(ctx->free_var.p, ctx->elem_deg.p, nfree, ctx->var_deg.p);
  DM_HIP(ctx, hipMemsetAsync(err.p, 0, 4 * sizeof(int), st));
  if (nr > 0)
    k_row_stats<<<grid_for(nr, 256), 256, 0, st>>>(ctx->rrow_ptr.p, ctx->rrow_b.p, nshort, nr, err.p);
  if (rnnz > 0)
    k_long_coefs<<<grid_for(rnnz, 256), 256, 0, st>>>(ctx->rrow_ptr.p, nshort, rnnz, ctx->rent_coef.p, err.p);
  DM_LAUNCH_CHECK(ctx);
  int stats[4];
  DM_HIP(ctx, hipMemcpyAsync(stats, err.p, sizeof(stats), hipMemcpyDeviceToHost, st));
  DM_HIP(ctx, hipStreamSynchronize(st));
  ctx->max_short = stats[2];
  if (stats[2] > MAX_SHORT_ROW)
    return dm_fail(ctx, DM_ERR_WORKSPACE, "a closedness row has %d > %d free entries", stats[2], MAX_SHORT_ROW);
  if (stats[3] & 2) return dm_fail(ctx, DM_ERR_STATE, "a presolved row has fewer than two entries");
  if (stats[3]) return dm_fail(ctx, DM_ERR_STATE, "a projection row is not an exactly-one row");
  int32_t nnz_short = 0;
  DM_TRY(read_i32(ctx, ctx->rrow_ptr.p + nshort, &nnz_short));
  ctx->nnz_short = nnz_short;
  DM_TRY(sweep_layout(ctx));
  // the smoothed sweep takes short rows in order of length, in segments of
  // 8, 16 or 32 lanes
  DArr<uint32_t> len;
  DArr<int32_t> bound;
  DM_ALLOC(ctx, ctx->soft_row, size_t(std::max<int64_t>(nshort, 1)));
  DM_ALLOC(ctx, len, size_t(std::max<int64_t>(nshort, 1)));
  DM_ALLOC(ctx, bound, 2);
  DM_HIP(ctx, hipMemsetAsync(bound.p, 0, 2 * sizeof(int32_t), st));
  if (nshort > 0) {
    k_row_len<<<grid_for(nshort, 256), 256, 0, st>>>(ctx->rrow_ptr.p, nshort, len.p, ctx->soft_row.p);
    DM_LAUNCH_CHECK(ctx);
    DM_TRY(sort_pairs_u32(ctx, len.p, ctx->soft_row.p, size_t(nshort), 7));
    k_len_bounds<<<grid_for(nshort, 256), 256, 0, st>>>(len.p, nshort, bound.p);
    DM_LAUNCH_CHECK(ctx);
  }
  int32_t bnd[2];
  DM_HIP(ctx, hipMemcpyAsync(bnd, bound.p, sizeof(bnd), hipMemcpyDeviceToHost, st));
  DM_HIP(ctx, hipStreamSynchronize(st));
  ctx->soft_c8 = bnd[0];
  ctx->soft_c16 = bnd[1] - bnd[0];
  return DM_OK;
}


extern "C" dm_status dm_build_product_space(dm_ctx* ctx, const dm_mesh* Xin, const dm_mesh* Yin,
                                            const int32_t* cand_xy, const int32_t* cand_yx, int32_t K,
                                            dm_space_info* info) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  ctx->has_space = false;
  ctx->corners_ready = false;
  ctx->has_cost = false;
  ctx->generic = false;
  if (!Xin || !Yin || !cand_xy || !cand_yx || !info)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_build_product_space: NULL argument");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  DM_TRY(mesh_ingest(ctx, Xin, ctx->X, "X"));
  DM_TRY(mesh_ingest(ctx, Yin, ctx->Y, "Y"));
  int chiX = ctx->X.nv - ctx->X.ne + ctx->X.nf, chiY = ctx->Y.nv - ctx->Y.ne + ctx->Y.nf;
  if (chiX != chiY)
    return dm_fail(ctx, DM_ERR_GENUS, "Euler characteristics differ (%d vs %d)", chiX, chiY);
  if (K < 1 || K > ctx->X.nv || K > ctx->Y.nv)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "K=%d outside [1, min(nvx, nvy)]", K);
  ctx->K = K;
  DM_TRY(space_build(ctx, cand_xy, cand_yx, K));
  ctx->has_space = true;
  fill_info(ctx, info);
  return DM_OK;
}

extern "C" dm_status dm_fix_variables(dm_ctx* ctx, const int8_t* fix, dm_space_info* info) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!ctx->has_space) return dm_fail(ctx, DM_ERR_STATE, "no product space built");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  DM_TRY(dual_flush(ctx));
  ++ctx->cost_generation;   // solver state of the previous problem is stale
  const dm_status s = presolve_reduce(ctx, fix);
  if (s != DM_OK) {
    // keep the message, restore the problem without fixings
    const std::string msg = ctx->err;
    if (presolve_reduce(ctx, nullptr) != DM_OK) {
      ctx->has_space = false;   // the reduced problem is half rebuilt: unusable
      return DM_ERR_STATE;
    }
    if (ctx->has_cost) DM_TRY(cost_offset(ctx));
    ctx->err = msg;
    if (info) fill_info(ctx, info);
    return s;
  }
  if (ctx->has_cost) DM_TRY(cost_offset(ctx));
  if (info) fill_info(ctx, info);
  return DM_OK;
}

void fill_info(dm_ctx* ctx, dm_space_info* info) {
  dm_space_info& I = *info;
  I.n_prod_tri = ctx->nP;
  I.n_rows_full = ctx->n_rows_full;
  I.nnz_full = ctx->nnz_full;
  I.n_closed_full = ctx->n_closed_full;
  I.n_free = ctx->n_free;
  I.n_fixed1 = ctx->n_fixed1;
  I.n_rows = ctx->n_rows;
  I.nnz = ctx->nnz;
  I.n_short_rows = ctx->n_short;
  I.n_edges_x = ctx->X.ne;
  I.n_edges_y = ctx->Y.ne;
  I.n_cand = ctx->nC;
  I.presolve_rounds = ctx->presolve_rounds;
  I.max_short_row = ctx->max_short;
}
