// Coarse-to-fine pruning (Sec. 5.2): a matching found at a coarser resolution
// restricts the candidate pairs of the next finer one.  For a vertex pair
// (m, n) matched at the coarse level, fine vertices in the ring neighbourhood
// (one- or two-ring) of m's location may match fine vertices in the ring
// neighbourhood of n's location; the union over the coarse matches is the
// fine level's candidate set.  Three pieces, all on the device:
//  * nearest vertices (a coarse vertex's location on the fine mesh): squared
//    distances in FP64, which is exact for FP32 coordinates, ties to the
//    lower index;
//  * the vertex pairs a primal uses (corners of its selected elements);
//  * ring candidates: ring sets from the fine meshes' directed edges, every
//    pair of a seed's two rings marked in a bitmap, then per-vertex lists in
//    ascending order, padded to a common length K by repeating their last
//    entry (the product-space builder takes K candidates per vertex and
//    ignores repeats).
#include <algorithm>

#include "dm_internal.h"

namespace {

constexpr int RING_MAX = 512;   // ring members gathered per seed vertex (with repeats)

__global__ void k_nearest(const float* P, int32_t n, const float* Q, int32_t m, int32_t* out) {
  const int32_t i = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double px = P[3 * i], py = P[3 * i + 1], pz = P[3 * i + 2];
  double best = 0.0;
  int32_t arg = -1;
  for (int32_t j = 0; j < m; ++j) {
    const double dx = px - double(Q[3 * j]), dy = py - double(Q[3 * j + 1]), dz = pz - double(Q[3 * j + 2]);
    const double d = (dx * dx + dy * dy) + dz * dz;   // exact: each term has at most 48 significant bits
    if (arg < 0 || d < best) {
      best = d;
      arg = j;
    }
  }
  out[i] = arg;
}

// pair bitmap of the vertex pairs that selected elements use
__global__ void k_mark_pairs(const int32_t* pv, const uint8_t* x, int64_t nP, uint8_t* mark) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= nP || !x[p]) return;
  for (int k = 0; k < 3; ++k) mark[pv[3 * p + k]] = 1;
}

__global__ void k_pairs_out(const uint8_t* mark, const int32_t* pos, int64_t npv, int32_t nvy, int32_t* pairs) {
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= npv || !mark[q]) return;
  pairs[2 * pos[q]] = int32_t(q / nvy);
  pairs[2 * pos[q] + 1] = int32_t(q % nvy);
}

__device__ inline int64_t lower_bound_key(const uint64_t* key, int64_t n, uint64_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// ring members of vertex a (a itself, its neighbours, for rings == 2 theirs),
// with repeats, into buf; returns the count or -1 past RING_MAX.  One thread.
__device__ int gather_ring(const uint64_t* dkey, int64_t nd, int32_t nv, int32_t a, int rings, int32_t* buf) {
  int cnt = 0;
  buf[cnt++] = a;
  const int64_t s = lower_bound_key(dkey, nd, uint64_t(a) * uint64_t(nv));
  const int64_t e = lower_bound_key(dkey, nd, uint64_t(a + 1) * uint64_t(nv));
  for (int64_t i = s; i < e; ++i) {
    if (cnt >= RING_MAX) return -1;
    buf[cnt++] = int32_t(dkey[i] % uint64_t(nv));
  }
  if (rings >= 2) {
    const int one = cnt;
    for (int t = 1; t < one; ++t) {
      const int32_t b = buf[t];
      const int64_t s2 = lower_bound_key(dkey, nd, uint64_t(b) * uint64_t(nv));
      const int64_t e2 = lower_bound_key(dkey, nd, uint64_t(b + 1) * uint64_t(nv));
      for (int64_t i = s2; i < e2; ++i) {
        if (cnt >= RING_MAX) return -1;
        buf[cnt++] = int32_t(dkey[i] % uint64_t(nv));
      }
    }
  }
  return cnt;
}

// one block per seed pair: both rings into LDS, then every pair marked
__global__ __launch_bounds__(256) void k_ring_mark(const int32_t* seeds, int32_t ns, const uint64_t* xkey,
                                                   int64_t nxd, int32_t nvx, const uint64_t* ykey, int64_t nyd,
                                                   int32_t nvy, int rings, uint8_t* mark, int* err) {
  __shared__ int32_t ra[RING_MAX], rb[RING_MAX];
  __shared__ int na, nb;
  const int32_t s = blockIdx.x;
  const int32_t a = seeds[2 * s], b = seeds[2 * s + 1];
  if (threadIdx.x == 0) {
    const bool ok = a >= 0 && a < nvx && b >= 0 && b < nvy;
    na = ok ? gather_ring(xkey, nxd, nvx, a, rings, ra) : -1;
    nb = ok ? gather_ring(ykey, nyd, nvy, b, rings, rb) : -1;
    if (na < 0 || nb < 0) atomicOr(err, 1);
  }
  __syncthreads();
  if (na < 0 || nb < 0) return;
  const int total = na * nb;
  for (int t = threadIdx.x; t < total; t += blockDim.x)
    mark[int64_t(ra[t / nb]) * nvy + rb[t % nb]] = 1;
}

// per row (dir 0: X vertex u over v) or column (dir 1: Y vertex v over u) of
// the bitmap: the number of marked pairs
__global__ void k_line_count(const uint8_t* mark, int32_t nvx, int32_t nvy, int dir, int32_t* cnt) {
  const int32_t i = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int32_t n = dir == 0 ? nvx : nvy, len = dir == 0 ? nvy : nvx;
  if (i >= n) return;
  int32_t c = 0;
  for (int32_t j = 0; j < len; ++j) c += dir == 0 ? mark[int64_t(i) * nvy + j] : mark[int64_t(j) * nvy + i];
  cnt[i] = c;
}

__global__ void k_line_fill(const uint8_t* mark, int32_t nvx, int32_t nvy, int dir, int32_t K, int32_t* cand) {
  const int32_t i = int32_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int32_t n = dir == 0 ? nvx : nvy, len = dir == 0 ? nvy : nvx;
  if (i >= n) return;
  int32_t k = 0, last = 0;
  for (int32_t j = 0; j < len && k < K; ++j) {
    const uint8_t mk = dir == 0 ? mark[int64_t(i) * nvy + j] : mark[int64_t(j) * nvy + i];
    if (mk) {
      cand[int64_t(i) * K + k++] = j;
      last = j;
    }
  }
  for (; k < K; ++k) cand[int64_t(i) * K + k] = last;   // repeats are ignored by the builder
}

__global__ void k_max_count(const int32_t* cnt, int32_t n, int32_t* out) {
  __shared__ int32_t red[256];
  int32_t mx = 0, mn = INT32_MAX;
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
    mx = max(mx, cnt[i]);
    mn = min(mn, cnt[i]);
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
  __syncthreads();
  red[threadIdx.x] = mn;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (int(threadIdx.x) < w) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[1] = red[0];
}

}  // namespace

extern "C" dm_status dm_nearest_vertices(dm_ctx* ctx, const float* P, int32_t n, const float* Q, int32_t m,
                                         int32_t* out) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  if (n < 0 || m < 1 || (n > 0 && (!P || !Q || !out)))
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_nearest_vertices: bad arguments");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  if (n > 0) k_nearest<<<grid_for(n, 256), 256, 0, ctx->stream>>>(P, n, Q, m, out);
  DM_LAUNCH_CHECK(ctx);
  return DM_OK;
}

extern "C" dm_status dm_matched_pairs(dm_ctx* ctx, const uint8_t* x, int32_t* pairs, int32_t cap,
                                      int32_t* n_pairs) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!ctx->has_space || ctx->generic)
    return dm_fail(ctx, DM_ERR_STATE, "dm_matched_pairs: needs a product space built from meshes");
  if (!x || !n_pairs || cap < 0 || (cap > 0 && !pairs))
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_matched_pairs: bad arguments");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  const int64_t npv = int64_t(ctx->X.nv) * ctx->Y.nv;
  DArr<uint8_t> mark;
  DArr<int32_t> pos;
  DM_ALLOC(ctx, mark, size_t(npv));
  DM_ALLOC(ctx, pos, size_t(npv) + 1);
  DM_HIP(ctx, hipMemsetAsync(mark.p, 0, size_t(npv), st));
  if (ctx->nP > 0) k_mark_pairs<<<grid_for(ctx->nP, 256), 256, 0, st>>>(ctx->pv.p, x, ctx->nP, mark.p);
  DM_LAUNCH_CHECK(ctx);
  DM_TRY(scan_u8(ctx, mark.p, pos.p, size_t(npv)));
  int32_t np = 0;
  DM_TRY(read_i32(ctx, pos.p + npv, &np));
  *n_pairs = np;
  if (np > cap) return dm_fail(ctx, DM_ERR_WORKSPACE, "dm_matched_pairs: %d pairs, capacity %d", np, cap);
  if (np > 0) k_pairs_out<<<grid_for(npv, 256), 256, 0, st>>>(mark.p, pos.p, npv, ctx->Y.nv, pairs);
  DM_LAUNCH_CHECK(ctx);
  DM_HIP(ctx, hipStreamSynchronize(st));
  return DM_OK;
}

extern "C" dm_status dm_ring_candidates(dm_ctx* ctx, const dm_mesh* Xf, const dm_mesh* Yf, const int32_t* seeds,
                                        int32_t n_seeds, int32_t rings, int32_t kcap, int32_t* cand_xy,
                                        int32_t* cand_yx, int32_t* K) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!Xf || !Yf || !K || n_seeds < 1 || !seeds || (rings != 1 && rings != 2) || kcap < 1 || !cand_xy ||
      !cand_yx)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_ring_candidates: bad arguments");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  hipStream_t st = ctx->stream;
  MeshDev X, Y;
  DM_TRY(mesh_ingest(ctx, Xf, X, "X"));
  DM_TRY(mesh_ingest(ctx, Yf, Y, "Y"));
  const int64_t npv = int64_t(X.nv) * Y.nv;
  DArr<uint8_t> mark;
  DArr<int32_t> cx, cy, mm;
  DArr<int> err;
  DM_ALLOC(ctx, mark, size_t(npv));
  DM_ALLOC(ctx, cx, size_t(X.nv));
  DM_ALLOC(ctx, cy, size_t(Y.nv));
  DM_ALLOC(ctx, mm, 4);
  DM_ALLOC(ctx, err, 1);
  DM_HIP(ctx, hipMemsetAsync(mark.p, 0, size_t(npv), st));
  DM_HIP(ctx, hipMemsetAsync(err.p, 0, sizeof(int), st));
  k_ring_mark<<<unsigned(n_seeds), 256, 0, st>>>(seeds, n_seeds, X.dkey.p, int64_t(X.nf) * 3, X.nv, Y.dkey.p,
                                                int64_t(Y.nf) * 3, Y.nv, rings, mark.p, err.p);
  k_line_count<<<grid_for(X.nv, 256), 256, 0, st>>>(mark.p, X.nv, Y.nv, 0, cx.p);
  k_line_count<<<grid_for(Y.nv, 256), 256, 0, st>>>(mark.p, X.nv, Y.nv, 1, cy.p);
  k_max_count<<<1, 256, 0, st>>>(cx.p, X.nv, mm.p);
  k_max_count<<<1, 256, 0, st>>>(cy.p, Y.nv, mm.p + 2);
  DM_LAUNCH_CHECK(ctx);
  int32_t v[5];
  {
    const int32_t* src[5] = {err.p, mm.p, mm.p + 1, mm.p + 2, mm.p + 3};
    DM_TRY(read_i32s(ctx, 5, src, v));
  }
  if (v[0]) return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_ring_candidates: a seed is out of range or a ring "
                                                   "exceeds %d members", RING_MAX);
  if (v[2] == 0 || v[4] == 0)
    return dm_fail(ctx, DM_ERR_INFEASIBLE, "dm_ring_candidates: a fine vertex has no candidate");
  const int32_t k = std::max(v[1], v[3]);
  *K = k;
  if (k > kcap) return dm_fail(ctx, DM_ERR_WORKSPACE, "dm_ring_candidates: K = %d exceeds the capacity %d", k, kcap);
  k_line_fill<<<grid_for(X.nv, 256), 256, 0, st>>>(mark.p, X.nv, Y.nv, 0, k, cand_xy);
  k_line_fill<<<grid_for(Y.nv, 256), 256, 0, st>>>(mark.p, X.nv, Y.nv, 1, k, cand_yx);
  DM_LAUNCH_CHECK(ctx);
  DM_HIP(ctx, hipStreamSynchronize(st));
  return DM_OK;
}
