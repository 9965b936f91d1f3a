// Quasi-Newton powered MMA (Sec. 4.1, Alg. 1; Appendix "Quasi-Newton
// Updates") on top of the Jacobi sweep of dual.hip.
//
// Vectors with one value per multiplier (the subgradient g, the history pairs
// s and y, the direction q / d) are five slot planes of n_free values: slot k
// of variable i (k as in the records; slots at or above the variable's row
// count are zero) at k * n_free + i, so every pass reads and writes
// whole planes coalesced.  g and y only take the values 0/1 and -1/0/1 and
// are stored as bytes, so a history pair costs 5 reals and 5 bytes per
// variable.
//
// One iteration, as launched by the host loop below:
//  1. direction: 2h + 1 variable-major passes over the last h accepted pairs.
//     Each pass first sums the previous pass's per-block dot partials in a
//     fixed order (every block computes the same value, so no extra launch is
//     needed for the reduction), applies one step of the two-loop recursion
//     and emits the per-block partials of the next dot; the last pass removes
//     every variable's mean (dual-feasible direction).  Dots are FP64.
//  2. FindStepSize: K + 1 bound-only sweeps at lambda + gamma d, each followed
//     by a one-block kernel that sums the bound and takes the search decision
//     on the device; sweeps after the search has stopped exit at once.
//  3. the MMA sweep at lambda + step d (step = 0 unless a trial improved).
//  4. the subgradient sweep at the new lambda, which also yields its bound.
//  5. the history pass s = lambda_new - lambda_old, y = g_old - g_new with the
//     dots s^T y and y^T y, and a one-block kernel for the curvature test; its
//     verdict is the only value read back by the host per iteration.
#include <algorithm>
#include <cmath>
#include <vector>

#include "dm_internal.h"

namespace {

constexpr int VB = 256;      // threads per block of the variable-major passes
constexpr int VGRID = 1024;  // at most this many blocks, hence partials per dot

// state of the step-size search, on the device
struct QnState {
  double E_init;  // E(lambda) of the current iteration
  double E0;      // E(lambda^0)
  double dmin;    // Delta_min
  double gamma;   // trial step size of the next probe
  double gm, Em;  // best trial so far and its objective
  double step;    // step applied before the MMA update
  int32_t done;   // search finished (later probes skip)
  int32_t pad;
};

__device__ inline double bsum(double v, double* red) { return block_sum_256(v, red); }

// sum of n per-block partials in a fixed order; every block gets the same value
__device__ inline double sum_partials(const double* p, int n, double* red) { return sum_partials_256(p, n, red); }

// vectors hold five slot planes of n values: slot k of variable i at k n + i
template <typename R>
__device__ inline void load5(const R* __restrict__ a, int64_t i, int64_t n, double v[5]) {
#pragma unroll
  for (int k = 0; k < 5; ++k) v[k] = double(a[k * n + i]);
}

template <typename R>
__device__ inline void store5(R* __restrict__ a, int64_t i, int64_t n, const double v[5]) {
#pragma unroll
  for (int k = 0; k < 5; ++k) a[k * n + i] = R(v[k]);
}

__device__ inline void load5_u8(const uint8_t* __restrict__ a, int64_t i, int64_t n, double v[5]) {
#pragma unroll
  for (int k = 0; k < 5; ++k) v[k] = double(a[k * n + i]);
}

__device__ inline void load5_i8(const int8_t* __restrict__ a, int64_t i, int64_t n, double v[5]) {
#pragma unroll
  for (int k = 0; k < 5; ++k) v[k] = double(a[k * n + i]);
}

__device__ inline double dot5(const double a[5], const double b[5]) {
  return (((a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]) + a[3] * b[3]) + a[4] * b[4];
}

// subtract the mean over the variable's d rows (slots 0 to d - 1; the others
// stay zero)
__device__ inline void project5(double v[5], int d) {
  double sum = 0.0;
  for (int k = 0; k < 5; ++k) sum += k < d ? v[k] : 0.0;
  const double mean = sum / double(d);
  for (int k = 0; k < 5; ++k) v[k] = k < d ? v[k] - mean : 0.0;
}

// ---------------------------------------------------------------- direction passes
// h = 0: d = g minus its per-variable mean
template <typename R>
__global__ __launch_bounds__(VB) void k_qn_project_g(const uint8_t* g8, const uint8_t* deg, int64_t n, R* d) {
  for (int64_t i = int64_t(blockIdx.x) * VB + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) {
    double v[5];
    load5_u8(g8, i, n, v);
    project5(v, deg[i]);
    store5<R>(d, i, n, v);
  }
}

// partials of s^T g (first dot of the first loop)
template <typename R>
__global__ __launch_bounds__(VB) void k_qn_first(const uint8_t* g8, const R* s, int64_t n, double* part_out) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * VB + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) {
    double gv[5], sv[5];
    load5_u8(g8, i, n, gv);
    load5<R>(s, i, n, sv);
    acc += dot5(sv, gv);
  }
  const double b = bsum(acc, red);
  if (threadIdx.x == 0) part_out[blockIdx.x] = b;
}

// first loop, pair j: alpha_j = rho_j s_j^T q (from the partials), q -= alpha_j
// y_j, then the partials of the next dot: s_{j-1}^T q, or y_oldest^T q after
// the last pair (for beta of the second loop)
template <typename R>
__global__ __launch_bounds__(VB) void k_qn_loop1(const uint8_t* g8, const R* q_in, const int8_t* y,
                                                 const R* s_next, const int8_t* y_next, const double* part_in,
                                                 int32_t n_in, const double* sy, double* alpha_out, int64_t n,
                                                 R* q_out, double* part_out) {
  __shared__ double red[4];
  const double alpha = sum_partials(part_in, n_in, red) / *sy;
  if (blockIdx.x == 0 && threadIdx.x == 0) *alpha_out = alpha;
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * VB + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) {
    double qv[5], yv[5], nv[5];
    if (g8) load5_u8(g8, i, n, qv);
    else load5<R>(q_in, i, n, qv);
    load5_i8(y, i, n, yv);
    for (int k = 0; k < 5; ++k) qv[k] = double(R(qv[k] - alpha * yv[k]));
    store5<R>(q_out, i, n, qv);
    if (s_next) load5<R>(s_next, i, n, nv);
    else load5_i8(y_next, i, n, nv);
    acc += dot5(nv, qv);
  }
  const double b = bsum(acc, red);
  if (threadIdx.x == 0) part_out[blockIdx.x] = b;
}

// second loop, pair j: beta = rho_j y_j^T q, q += (alpha_j - beta) s_j; the
// first pass scales q by H0 = s^T y / y^T y of the newest pair; then the
// partials of y_{j+1}^T q, or after the newest pair the projection of d
template <typename R>
__global__ __launch_bounds__(VB) void k_qn_loop2(const R* q_in, const R* s, const int8_t* y_next,
                                                 const double* part_in, int32_t n_in, const double* sy,
                                                 const double* alpha, const double* h0_sy, const double* h0_yy,
                                                 const uint8_t* deg, int64_t n, R* q_out, double* part_out) {
  __shared__ double red[4];
  const double h0 = h0_sy ? *h0_sy / *h0_yy : 1.0;
  const double beta = h0 * sum_partials(part_in, n_in, red) / *sy;
  const double coef = *alpha - beta;
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * VB + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) {
    double qv[5], sv[5];
    load5<R>(q_in, i, n, qv);
    load5<R>(s, i, n, sv);
    for (int k = 0; k < 5; ++k) qv[k] = h0 * qv[k] + coef * sv[k];
    if (y_next) {
      for (int k = 0; k < 5; ++k) qv[k] = double(R(qv[k]));
      double yv[5];
      load5_i8(y_next, i, n, yv);
      acc += dot5(yv, qv);
    } else {
      project5(qv, deg[i]);
    }
    store5<R>(q_out, i, n, qv);
  }
  if (y_next) {
    const double b = bsum(acc, red);
    if (threadIdx.x == 0) part_out[blockIdx.x] = b;
  }
}

// ---------------------------------------------------------------- history
// s = lambda_new - lambda_old (both with feasibility restored exactly as the
// sweeps see them), y = g_old - g_new, and the partials of s^T y and y^T y
template <typename R>
__global__ __launch_bounds__(VB) void k_qn_hist_pass(const R* rec_old, const R* rec_new, const uint8_t* g_old,
                                                     const uint8_t* g_new, const uint8_t* deg, int64_t n, R* s_out,
                                                     int8_t* y_out, double* part_sy, double* part_yy) {
  __shared__ double red[4];
  double a_sy = 0.0, a_yy = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * VB + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) {
    R lo[5], ln[5];
    rec_lambdas<R>(rec_old, size_t(i), lo);
    rec_lambdas<R>(rec_new, size_t(i), ln);
    double go[5], gn[5], sv[5], yv[5];
    load5_u8(g_old, i, n, go);
    load5_u8(g_new, i, n, gn);
    for (int k = 0; k < 5; ++k) {
      sv[k] = double(R(ln[k] - lo[k]));
      yv[k] = go[k] - gn[k];
      y_out[k * n + i] = int8_t(yv[k]);
    }
    store5<R>(s_out, i, n, sv);
    a_sy += dot5(sv, yv);
    a_yy += dot5(yv, yv);
  }
  const double b_sy = bsum(a_sy, red);
  const double b_yy = bsum(a_yy, red);
  if (threadIdx.x == 0) {
    part_sy[blockIdx.x] = b_sy;
    part_yy[blockIdx.x] = b_yy;
  }
}

// partials of s^T y and y^T y of a given pair
template <typename R>
__global__ __launch_bounds__(VB) void k_qn_pair_dots(const R* s, const int8_t* y, int64_t n, double* part_sy,
                                                     double* part_yy) {
  __shared__ double red[4];
  double a_sy = 0.0, a_yy = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * VB + threadIdx.x; i < n; i += int64_t(gridDim.x) * VB) {
    double sv[5], yv[5];
    load5<R>(s, i, n, sv);
    load5_i8(y, i, n, yv);
    a_sy += dot5(sv, yv);
    a_yy += dot5(yv, yv);
  }
  const double b_sy = bsum(a_sy, red);
  const double b_yy = bsum(a_yy, red);
  if (threadIdx.x == 0) {
    part_sy[blockIdx.x] = b_sy;
    part_yy[blockIdx.x] = b_yy;
  }
}

__global__ __launch_bounds__(1024) void k_qn_pair_fin(const double* part_sy, const double* part_yy, int32_t n,
                                                    double* sy, double* yy) {
  __shared__ double red[16];
  const double a = sum_partials_1024(part_sy, n, red);
  const double b = sum_partials_1024(part_yy, n, red);
  if (threadIdx.x == 0) {
    *sy = a;
    *yy = b;
  }
}

// ---------------------------------------------------------------- one-block decisions
// start of a call: the bound at the imported lambda; a fresh search also
// resets the step size and Delta_min (a resumed one keeps them)
__global__ __launch_bounds__(1024) void k_qn_begin(const double* sp, int32_t sn, double offset, QnState* st,
                                                 double* etrace, double gamma0, int32_t resume) {
  __shared__ double red[16];
  const double E = offset + sum_partials_1024(sp, sn, red);
  if (threadIdx.x == 0) {
    etrace[0] = E;
    if (!resume) {
      st->E0 = E;
      st->dmin = INFINITY;
      st->gamma = gamma0;
      st->gm = gamma0;
    }
    st->E_init = E;
    st->Em = -INFINITY;
    st->step = 0.0;
    st->done = 0;
  }
}

// FindStepSize after probe t (t = 0: the previous step size; t = 1..K: the
// rescaled ones): keep the best trial, stop after a gain of Delta_min or at
// t = K, otherwise rescale gamma by the verdict of this trial against E(lambda)
__global__ __launch_bounds__(1024) void k_qn_probe(const double* sp, int32_t sn, double offset, int32_t t, int32_t K,
                                                 double up, double down, QnState* st, double* gtrace,
                                                 int32_t* taken) {
  __shared__ double red[16];
  if (st->done) return;   // uniform
  const double E = offset + sum_partials_1024(sp, sn, red);
  if (threadIdx.x != 0) return;
  if (t == 0 || E >= st->Em) {
    st->gm = st->gamma;
    st->Em = E;
  }
  const bool stop = t == K || (t > 0 && E - st->E_init >= st->dmin);
  if (stop) {
    const bool improve = st->Em > st->E_init;
    st->done = 1;
    st->step = improve ? st->gm : 0.0;
    st->gamma = st->gm;
    if (gtrace) *gtrace = st->gm;
    if (taken) *taken = improve ? 1 : 0;
  } else {
    st->gamma = (E <= st->E_init) ? down * st->gamma : up * st->gamma;
  }
}

// after the subgradient sweep at lambda_{k+1} and the history pass: the bound
// E(lambda_{k+1}), Delta_min after the first iteration, the curvature test
__global__ __launch_bounds__(1024) void k_qn_hist(const double* sp, int32_t sn, double offset, const double* part_sy,
                                                const double* part_yy, int32_t hn, int32_t k, int32_t set_dmin,
                                                double eps, QnState* st, double* etrace, double* sy_out,
                                                double* yy_out, int32_t* accepted) {
  __shared__ double red[16];
  const double E = offset + sum_partials_1024(sp, sn, red);
  const double sy = sum_partials_1024(part_sy, hn, red);
  const double yy = sum_partials_1024(part_yy, hn, red);
  if (threadIdx.x != 0) return;
  etrace[k + 1] = E;
  if (set_dmin) st->dmin = 1e-6 * (E - st->E0);
  st->E_init = E;
  st->done = 0;
  st->Em = -INFINITY;
  const bool ok = hn > 0 && sy >= eps;
  if (ok) {
    *sy_out = sy;
    *yy_out = yy;
  }
  *accepted = ok ? 1 : 0;
}

// ---------------------------------------------------------------- layout conversion
// entry order <-> slot planes
template <typename T>
__global__ void k_scatter(const T* v, const uint32_t* word, int64_t nnz, int64_t n, T* planes) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < nnz) planes[int64_t((word[e] >> W_SLOT_SHIFT) & 7u) * n + (word[e] & W_VAR_MASK)] = v[e];
}

template <typename T>
__global__ void k_gather(const T* planes, const uint32_t* word, int64_t nnz, int64_t n, T* v) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < nnz) v[e] = planes[int64_t((word[e] >> W_SLOT_SHIFT) & 7u) * n + (word[e] & W_VAR_MASK)];
}

__global__ void k_fill_f64(double* a, int64_t n, double v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// device scalars per history buffer b: s^T y, y^T y, alpha
struct Scal {
  double* p;
  int nb;
  double* sy(int b) const { return p + b; }
  double* yy(int b) const { return p + nb + b; }
  double* alpha(int b) const { return p + 2 * nb + b; }
};

unsigned vgrid(int64_t n) {
  return unsigned(std::max<int64_t>(1, std::min<int64_t>(VGRID, (n + VB - 1) / VB)));
}

// d = projected H g into q, over the pairs in `order` (oldest first); part
// holds two VGRID halves
template <typename R>
dm_status direction(dm_ctx* ctx, const std::vector<int>& order, R* const* S, int8_t* const* Y, const uint8_t* g8,
                    R* q, const Scal& sc, double* part) {
  const int64_t n = ctx->n_free;
  const unsigned G = vgrid(n);
  const uint8_t* deg = ctx->var_deg.p;
  hipStream_t st = ctx->stream;
  const int h = int(order.size());
  if (h == 0) {
    k_qn_project_g<R><<<G, VB, 0, st>>>(g8, deg, n, q);
    DM_LAUNCH_CHECK(ctx);
    return DM_OK;
  }
  double* pin = part;
  double* pout = part + VGRID;
  k_qn_first<R><<<G, VB, 0, st>>>(g8, S[order[h - 1]], n, pin);
  for (int i = h - 1; i >= 0; --i) {
    const int b = order[i];
    const R* s_next = i > 0 ? S[order[i - 1]] : nullptr;
    const int8_t* y_next = i > 0 ? nullptr : Y[order[0]];
    k_qn_loop1<R><<<G, VB, 0, st>>>(i == h - 1 ? g8 : nullptr, q, Y[b], s_next, y_next, pin, int32_t(G),
                                     sc.sy(b), sc.alpha(b), n, q, pout);
    std::swap(pin, pout);
  }
  const int newest = order[h - 1];
  for (int i = 0; i < h; ++i) {
    const int b = order[i];
    const int8_t* y_next = i + 1 < h ? Y[order[i + 1]] : nullptr;
    k_qn_loop2<R><<<G, VB, 0, st>>>(q, S[b], y_next, pin, int32_t(G), sc.sy(b), sc.alpha(b),
                                     i == 0 ? sc.sy(newest) : nullptr, i == 0 ? sc.yy(newest) : nullptr, deg, n,
                                     q, pout);
    std::swap(pin, pout);
  }
  DM_LAUNCH_CHECK(ctx);
  return DM_OK;
}

template <typename R>
struct QnBuffers {
  DArr<R> S, q;
  DArr<int8_t> Y;
  DArr<uint8_t> g[2];
  DArr<double> part, scal;
  std::vector<R*> Sp;
  std::vector<int8_t*> Yp;
};

template <typename R>
dm_status qn_alloc(dm_ctx* ctx, int nb, QnBuffers<R>& B) {
  const size_t rec = size_t(std::max<int64_t>(ctx->n_free, 1)) * 5;   // five slot planes
  DM_ALLOC(ctx, B.S, rec * nb);
  DM_ALLOC(ctx, B.Y, rec * nb);
  DM_ALLOC(ctx, B.q, rec);
  DM_ALLOC(ctx, B.g[0], rec);
  DM_ALLOC(ctx, B.g[1], rec);
  DM_ALLOC(ctx, B.part, 4 * VGRID);
  DM_ALLOC(ctx, B.scal, 3 * size_t(nb));
  DM_HIP(ctx, hipMemsetAsync(B.S.p, 0, rec * nb * sizeof(R), ctx->stream));
  DM_HIP(ctx, hipMemsetAsync(B.Y.p, 0, rec * nb, ctx->stream));
  DM_HIP(ctx, hipMemsetAsync(B.q.p, 0, rec * sizeof(R), ctx->stream));
  DM_HIP(ctx, hipMemsetAsync(B.g[0].p, 0, rec, ctx->stream));
  DM_HIP(ctx, hipMemsetAsync(B.g[1].p, 0, rec, ctx->stream));
  DM_HIP(ctx, hipMemsetAsync(B.scal.p, 0, 3 * size_t(nb) * sizeof(double), ctx->stream));
  B.Sp.resize(nb);
  B.Yp.resize(nb);
  for (int b = 0; b < nb; ++b) {
    B.Sp[b] = B.S.p + rec * b;
    B.Yp[b] = B.Y.p + rec * b;
  }
  return DM_OK;
}

// search state kept on the context between calls (history pairs, step size,
// Delta_min), one per message precision
template <typename R>
struct QnSession {
  QnBuffers<R> B;
  DArr<QnState> st;
  DArr<int32_t> flag;
  std::vector<int> order;   // accepted pairs, oldest first
  int spare = 0;            // buffer of the next candidate pair
  int m = -1;
  int64_t n_free = -1, generation = -1;
};

struct QnSessions {
  QnSession<float> f32;
  QnSession<double> f64;
};

void qn_delete(void* p) { delete static_cast<QnSessions*>(p); }

template <typename R>
QnSession<R>& session(dm_ctx* ctx) {
  if (!ctx->qn) {
    ctx->qn = new QnSessions;
    ctx->qn_free = qn_delete;
  }
  QnSessions* q = static_cast<QnSessions*>(ctx->qn);
  if constexpr (sizeof(R) == 4) return q->f32;
  else return q->f64;
}

template <typename R>
dm_status lbfgs_impl(dm_ctx* ctx, int32_t iters, const dm_lbfgs_params& P, R* lam, double* lb_trace,
                     double* gamma_trace, int32_t* taken) {
  hipStream_t stream = ctx->stream;
  if (ctx->n_rows == 0) {   // nothing free: the bound is the constant
    if (lb_trace) k_fill_f64<<<grid_for(iters + 1, 256), 256, 0, stream>>>(lb_trace, iters + 1, ctx->offset);
    if (gamma_trace && iters > 0)
      k_fill_f64<<<grid_for(iters, 256), 256, 0, stream>>>(gamma_trace, iters, P.gamma0);
    if (taken && iters > 0) k_fill_i32<<<grid_for(iters, 256), 256, 0, stream>>>(taken, iters, 0);
    DM_LAUNCH_CHECK(ctx);
    return DM_OK;
  }
  const int m = P.history;
  const int nb = m + 1;   // m history pairs and one candidate
  QnSession<R>& S = session<R>(ctx);
  const bool resume = P.resume != 0 && S.m == m && S.n_free == ctx->n_free &&
                      S.generation == ctx->cost_generation;
  if (P.resume != 0 && !resume)
    return dm_fail(ctx, DM_ERR_STATE,
                   "resume needs an earlier dm_lbfgs_solve on the same costs with the same precision and history");
  if (!resume) {
    DM_TRY(qn_alloc<R>(ctx, nb, S.B));
    DM_ALLOC(ctx, S.st, 1);
    DM_ALLOC(ctx, S.flag, 1);
    S.order.clear();
    S.spare = 0;
    S.m = m;
    S.n_free = ctx->n_free;
    S.generation = ctx->cost_generation;
  }
  QnBuffers<R>& B = S.B;
  QnState* st = S.st.p;
  DArr<double> etrace;
  DM_ALLOC(ctx, etrace, size_t(iters) + 1);
  const Scal sc{B.scal.p, nb};
  const int64_t n = ctx->n_free;
  const unsigned G = vgrid(n);
  DM_TRY(dual_flush(ctx));
  DM_TRY(dual_import<R>(ctx, lam, ctx->rec));
  int cur = 0, gc = 0;
  SweepExt sub;
  sub.gsub = B.g[0].p;
  DM_TRY(dual_sweep<R>(ctx, SWEEP_SUBGRAD, false, ctx->rec[0].p, nullptr, R(0), R(0), nullptr, &sub));
  k_qn_begin<<<1, 1024, 0, stream>>>(ctx->pend_partial, ctx->pend_n, ctx->offset, st, etrace.p, P.gamma0,
                                   resume ? 1 : 0);
  DM_LAUNCH_CHECK(ctx);
  for (int32_t k = 0; k < iters; ++k) {
    DM_TRY(direction<R>(ctx, S.order, B.Sp.data(), B.Yp.data(), B.g[gc].p, B.q.p, sc, B.part.p));
    SweepExt pe;
    pe.dir = B.q.p;
    pe.gamma = &st->gamma;
    pe.skip = &st->done;
    for (int t = 0; t <= P.max_search; ++t) {
      DM_TRY(dual_sweep<R>(ctx, SWEEP_BOUND, false, ctx->rec[cur].p, nullptr, R(0), R(0), nullptr, &pe));
      k_qn_probe<<<1, 1024, 0, stream>>>(ctx->pend_partial, ctx->pend_n, ctx->offset, t, P.max_search, P.step_up,
                                         P.step_down, st, gamma_trace ? gamma_trace + k : nullptr,
                                         taken ? taken + k : nullptr);
      DM_LAUNCH_CHECK(ctx);
      // the search usually stops at the second trial: one read of the flag
      // then spares launching the remaining probes (a skipped launch still
      // dispatches every workgroup of the sweep grid)
      if (t == 1 && t < P.max_search) {
        int32_t done = 0;
        DM_HIP(ctx, hipMemcpyAsync(&done, &st->done, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        DM_HIP(ctx, hipStreamSynchronize(stream));
        if (done) break;
      }
    }
    SweepExt me;
    me.dir = B.q.p;
    me.gamma = &st->step;
    DM_TRY(dual_sweep<R>(ctx, SWEEP_UPDATE, false, ctx->rec[cur].p, ctx->rec[cur ^ 1].p, R(P.omega), R(0),
                         nullptr, &me));
    sub.gsub = B.g[gc ^ 1].p;
    DM_TRY(dual_sweep<R>(ctx, SWEEP_SUBGRAD, false, ctx->rec[cur ^ 1].p, nullptr, R(0), R(0), nullptr, &sub));
    const double* sp = ctx->pend_partial;
    const int32_t sn = ctx->pend_n;
    double* psy = B.part.p + 2 * VGRID;
    double* pyy = B.part.p + 3 * VGRID;
    const int spare = S.spare;
    if (m > 0)
      k_qn_hist_pass<R><<<G, VB, 0, stream>>>(reinterpret_cast<const R*>(ctx->rec[cur].p),
                                               reinterpret_cast<const R*>(ctx->rec[cur ^ 1].p), B.g[gc].p,
                                               B.g[gc ^ 1].p, ctx->var_deg.p, n, B.Sp[spare], B.Yp[spare], psy,
                                               pyy);
    k_qn_hist<<<1, 1024, 0, stream>>>(sp, sn, ctx->offset, psy, pyy, m > 0 ? int32_t(G) : 0, k,
                                    (k == 0 && !resume) ? 1 : 0, P.eps, st, etrace.p, sc.sy(spare),
                                    sc.yy(spare), S.flag.p);
    DM_LAUNCH_CHECK(ctx);
    cur ^= 1;
    gc ^= 1;
    if (m > 0) {
      int32_t ok = 0;
      DM_HIP(ctx, hipMemcpyAsync(&ok, S.flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
      DM_HIP(ctx, hipStreamSynchronize(stream));
      if (ok) {
        S.order.push_back(spare);
        if (int(S.order.size()) > m) {
          S.spare = S.order.front();
          S.order.erase(S.order.begin());
        } else {
          for (int b = 0; b < nb; ++b)
            if (std::find(S.order.begin(), S.order.end(), b) == S.order.end()) {
              S.spare = b;
              break;
            }
        }
      }
    }
  }
  if (lb_trace)
    DM_HIP(ctx, hipMemcpyAsync(lb_trace, etrace.p, (size_t(iters) + 1) * sizeof(double), hipMemcpyDeviceToDevice,
                               stream));
  DM_TRY(dual_export<R>(ctx, ctx->rec[cur].p, lam));
  // the per-call trace buffer is freed on return: wait for the queued work
  DM_HIP(ctx, hipStreamSynchronize(stream));
  return DM_OK;
}

template <typename R>
dm_status subgradient_impl(dm_ctx* ctx, const R* lam, uint8_t* g, double* lb) {
  DArr<unsigned char> bufs[2];
  DArr<uint8_t> g8;
  DM_TRY(dual_flush(ctx));
  DM_TRY(dual_import<R>(ctx, lam, bufs));
  DM_ALLOC(ctx, g8, size_t(std::max<int64_t>(ctx->n_free, 1)) * 5);
  DM_HIP(ctx, hipMemsetAsync(g8.p, 0, g8.n, ctx->stream));
  DM_ALLOC(ctx, ctx->scal, 16);
  SweepExt sub;
  sub.gsub = g8.p;
  DM_TRY(dual_sweep<R>(ctx, SWEEP_SUBGRAD, false, bufs[0].p, nullptr, R(0), R(0), ctx->scal.p, &sub));
  DM_TRY(dual_flush(ctx));
  if (ctx->nnz > 0)
    k_gather<uint8_t><<<grid_for(ctx->nnz, 256), 256, 0, ctx->stream>>>(g8.p, ctx->rent_word.p, ctx->nnz,
                                                                        ctx->n_free, g);
  DM_LAUNCH_CHECK(ctx);
  double v = 0.0;
  DM_HIP(ctx, hipMemcpyAsync(&v, ctx->scal.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (lb) *lb = v;
  return DM_OK;
}

template <typename R>
dm_status direction_impl(dm_ctx* ctx, int32_t h, const R* S, const int8_t* Y, const uint8_t* g, R* d) {
  const int64_t n = ctx->n_free, nnz = ctx->nnz;
  if (nnz == 0) return DM_OK;
  QnBuffers<R> B;
  DM_TRY(qn_alloc<R>(ctx, std::max(h, 1), B));
  const Scal sc{B.scal.p, std::max(h, 1)};
  const unsigned G = vgrid(n);
  const unsigned E = grid_for(nnz, 256);
  std::vector<int> order;
  k_scatter<uint8_t><<<E, 256, 0, ctx->stream>>>(g, ctx->rent_word.p, nnz, n, B.g[0].p);
  for (int b = 0; b < h; ++b) {
    k_scatter<R><<<E, 256, 0, ctx->stream>>>(S + size_t(b) * nnz, ctx->rent_word.p, nnz, n, B.Sp[b]);
    k_scatter<int8_t><<<E, 256, 0, ctx->stream>>>(Y + size_t(b) * nnz, ctx->rent_word.p, nnz, n, B.Yp[b]);
    k_qn_pair_dots<R><<<G, VB, 0, ctx->stream>>>(B.Sp[b], B.Yp[b], n, B.part.p, B.part.p + VGRID);
    k_qn_pair_fin<<<1, 1024, 0, ctx->stream>>>(B.part.p, B.part.p + VGRID, int32_t(G), sc.sy(b), sc.yy(b));
    order.push_back(b);
  }
  DM_LAUNCH_CHECK(ctx);
  DM_TRY(direction<R>(ctx, order, B.Sp.data(), B.Yp.data(), B.g[0].p, B.q.p, sc, B.part.p));
  k_gather<R><<<E, 256, 0, ctx->stream>>>(B.q.p, ctx->rent_word.p, nnz, n, d);
  DM_LAUNCH_CHECK(ctx);
  DM_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return DM_OK;
}

dm_status check_ready(dm_ctx* ctx, int32_t msg_prec) {
  if (!ctx) return DM_ERR_INVALID_ARG;
  if (!ctx->has_space) return dm_fail(ctx, DM_ERR_STATE, "no product space built");
  if (!ctx->has_cost) return dm_fail(ctx, DM_ERR_STATE, "no costs built");
  if (msg_prec != DM_PREC_FP32 && msg_prec != DM_PREC_FP64)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "message precision must be FP32 or FP64");
  return DM_OK;
}

}  // namespace

extern "C" dm_status dm_lbfgs_solve(dm_ctx* ctx, int32_t iters, const dm_lbfgs_params* params, int32_t msg_prec,
                                    void* lambda, double* lb_trace, double* gamma_trace, int32_t* taken) {
  DM_TRY(check_ready(ctx, msg_prec));
  ctx->err.clear();
  if (!params || (!lambda && ctx->nnz > 0) || iters < 0)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_lbfgs_solve: bad arguments");
  const dm_lbfgs_params& P = *params;
  if (P.history < 0 || P.history > 64) return dm_fail(ctx, DM_ERR_INVALID_ARG, "history must be in [0, 64]");
  if (P.max_search < 1 || P.max_search > 64)
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "max_search must be in [1, 64]");
  if (!(P.omega > 0.0 && P.omega <= 1.0)) return dm_fail(ctx, DM_ERR_INVALID_ARG, "omega must be in (0, 1]");
  if (!(P.step_up > 1.0) || !(P.step_down > 0.0 && P.step_down < 1.0) || !(P.gamma0 >= 0.0) ||
      !std::isfinite(P.gamma0) || !std::isfinite(P.step_up) || !std::isfinite(P.eps))
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "need step_up > 1, 0 < step_down < 1, finite gamma0 >= 0, finite eps");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  if (msg_prec == DM_PREC_FP32)
    return lbfgs_impl<float>(ctx, iters, P, static_cast<float*>(lambda), lb_trace, gamma_trace, taken);
  return lbfgs_impl<double>(ctx, iters, P, static_cast<double*>(lambda), lb_trace, gamma_trace, taken);
}

extern "C" dm_status dm_subgradient(dm_ctx* ctx, int32_t msg_prec, const void* lambda, uint8_t* g, double* lb) {
  DM_TRY(check_ready(ctx, msg_prec));
  ctx->err.clear();
  if ((!lambda || !g) && ctx->nnz > 0) return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_subgradient: NULL argument");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  if (msg_prec == DM_PREC_FP32) return subgradient_impl<float>(ctx, static_cast<const float*>(lambda), g, lb);
  return subgradient_impl<double>(ctx, static_cast<const double*>(lambda), g, lb);
}

extern "C" dm_status dm_lbfgs_direction(dm_ctx* ctx, int32_t msg_prec, int32_t h, const void* S, const int8_t* Y,
                                        const uint8_t* g, void* d) {
  DM_TRY(check_ready(ctx, msg_prec));
  ctx->err.clear();
  if (h < 0 || h > 64 || !g || !d || (h > 0 && (!S || !Y)))
    return dm_fail(ctx, DM_ERR_INVALID_ARG, "dm_lbfgs_direction: bad arguments");
  DM_HIP(ctx, hipSetDevice(ctx->device));
  if (msg_prec == DM_PREC_FP32)
    return direction_impl<float>(ctx, h, static_cast<const float*>(S), Y, g, static_cast<float*>(d));
  return direction_impl<double>(ctx, h, static_cast<const double*>(S), Y, g, static_cast<double*>(d));
}
